"""tm_density_filter_noalloc (fixed device scratch, no allocation) against
tm_density_filter (stream-ordered scratch): the two share their kernels, so
the results must be equal bit for bit.  Two calls in a row per case, the second
on a smaller mesh, so the second reads an array the first left behind."""
import ctypes as C

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _filter(fn, nel, x, radius, transpose):
    from paper_2001_01655_amd import _lib as L
    mesh = L.make_mesh(nel)
    out = torch.full_like(x, float("nan"))
    st = fn(C.byref(mesh), radius, transpose, C.c_void_p(x.data_ptr()), C.c_void_p(out.data_ptr()),
            C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == L.TM_OK, L.LIB.tm_last_error().decode()
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("transpose", [1, 0])
@pytest.mark.parametrize("radius", [1.5, 2.6])
@pytest.mark.parametrize("sizes", [((96, 48, 40), (37, 21, 13)), ((700, 333), (129, 65))], ids=["3d", "2d"])
def test_noalloc_equals_allocating_filter(sizes, radius, transpose):
    from paper_2001_01655_amd import _lib as L
    print(f"filter noalloc {sizes} r={radius} transpose={transpose}", flush=True)
    for k, nel in enumerate(sizes):
        n = int(np.prod(nel))
        x = torch.tensor(np.random.default_rng(50 + k).uniform(-1.0, 1.0, n), device="cuda")
        ref = _filter(L.LIB.tm_density_filter, nel, x, radius, transpose)
        got = _filter(L.LIB.tm_density_filter_noalloc, nel, x, radius, transpose)
        assert np.all(np.isfinite(got)) and np.array_equal(got, ref), f"call {k} on {nel}"


def test_noalloc_refuses_meshes_beyond_its_scratch():
    from paper_2001_01655_amd import _lib as L
    mesh = L.make_mesh((256, 256, 129))           # 8,454,144 elements > 2^23
    a = C.c_void_p(16)
    b = C.c_void_p(32)
    st = L.LIB.tm_density_filter_noalloc(C.byref(mesh), 1.5, 1, a, b, None)
    assert st == L.TM_ERR_ARG and "at most 8388608" in L.LIB.tm_last_error().decode()
