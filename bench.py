"""Benchmark: MDoF/s to rtol 1e-8 of the multigrid-preconditioned CG solve.

One step = one full solve of K(rho) u = f (f resident in HBM -> u resident),
setup excluded, on the 3D cantilever 192x96x96 Hex8 (5,447,811 dofs) with a
6-level geometric hierarchy and an FP32 V-cycle inside FP64 flexible CG.  The
FP64-everywhere PCG on the same problem is timed beside it, and the oracle
(CPU, FP64, one thread) on a bounded sample of the same recipe.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

After the timed steps one more solve runs with HIP events around every launch
of three kernel classes (outer FP64 operator, V-cycle fine operator, first
coarse level operator); their mean durations give the roofline fractions.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOADS = {
    # the MBB half-beam of the classic setting: block Jacobi w = 0.6, 2/2 sweeps
    "mbb2d": dict(cfg="mbb_random", levels=3, opts=dict(omega=0.6), smoother="jacobi", sweeps=2,
                  desc="2D MBB half-beam 60x20 Q4, 2,562 dofs, U(0,1) densities"),
    "cantilever3d": dict(cfg="cantilever3d", levels=6, opts={},
                         desc="3D cantilever 192x96x96 Hex8, 5,447,811 dofs"),
    "cantilever2d": dict(cfg="cantilever2d", levels=7, opts=dict(max_iters=20000),
                         desc="2D cantilever 1024x512 Q4, 1,051,650 dofs"),
    "bridge3d": dict(cfg="bridge3d", levels=None, opts=dict(n_geometric=3, max_coarse=1000),
                     desc="3D bridge 256x128x128 Hex8, 12,830,211 dofs, 3 GMG levels + smoothed aggregation "
                          "to <1000 dofs"),
}
SMOOTHERS = {"jacobi": 0, "chebyshev": 2}


def workload_label(wl, args, levels, coarsest):
    s = wl["desc"]
    if wl["levels"] is not None:
        s += f", {levels}-level GMG (coarsest {coarsest} dofs)"
    if getattr(args, "n_geometric", None) is not None:
        s += f", {args.n_geometric} geometric levels before the aggregation"
    w = wl["opts"].get("omega", 0.5)
    sm = f"block Jacobi w={w:g}" if args.smoother == "jacobi" else f"Chebyshev on [{args.cheb_lower:g}, 1.1] x lambda"
    return s + f", {sm} {args.sweeps}/{args.sweeps}, rtol 1e-8"


# MI355X published peaks (dense): HBM3E 8 TB/s; vector FP64 78.6 TFLOP/s; vector
# FP32 157.3 TFLOP/s (the kernels are compiled without packed FP32 instructions;
# plain FP32 FMAs issue at up to about 85% of that rate)
PEAK = {"hbm_GBs": 8000.0, "fp64_TFs": 78.6, "fp32_TFs": 157.3}
KERNEL_SOURCES = {0: ["kernels_fine.hip", "tm_device.h"], 1: ["kernels_fine.hip", "tm_device.h"],
                  2: ["kernels_coarse.hip", "tm_device.h"]}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="cantilever3d", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-profile", action="store_true", help="skip the event-timed solve")
    ap.add_argument("--eigen-only", action="store_true",
                    help="run only the stability eigenproblem leg and print its record (profiling)")
    ap.add_argument("--no-side-legs", action="store_true",
                    help="skip the multi-RHS and density-filter legs (profiled runs: only the headline solves)")
    ap.add_argument("--stability", action="store_true",
                    help="add the stability eigenproblem legs (generalized Davidson on the 2D column)")
    ap.add_argument("--served", type=int, default=200, help="requests in the served-stream leg (0: skip)")
    ap.add_argument("--served-hybrid-every", type=int, default=8,
                    help="every n-th served request is a hybrid (aggregation) hierarchy (0: none)")
    ap.add_argument("--served-designs", type=int, default=20)
    ap.add_argument("--served-smoother", default="chebyshev", choices=sorted(SMOOTHERS))
    ap.add_argument("--served-sweeps", type=int, default=2)
    ap.add_argument("--served-warm-steps", type=int, default=4,
                    help="power steps of a design update's Chebyshev estimate, from the previous vector (0: 12 cold)")
    ap.add_argument("--levels", type=int, default=None, help="multigrid levels (default: the workload's)")
    ap.add_argument("--n-geometric", type=int, default=None,
                    help="geometric levels before smoothed aggregation (hybrid workloads; default: the workload's)")
    ap.add_argument("--smoother", default=None, choices=sorted(SMOOTHERS),
                    help="default: the workload's (chebyshev, block Jacobi for the MBB half-beam)")
    ap.add_argument("--sweeps", type=int, default=None, help="pre- and post-smoothing sweeps (default: the workload's, 2)")
    ap.add_argument("--cheb-lower", type=float, default=0.1,
                    help="Chebyshev interval [cheb_lower, 1.1] x the estimated largest eigenvalue of D^-1 A")
    ap.add_argument("--fine-mfma", type=int, default=0, choices=[0, 1],
                    help="FP32 fine operator on the matrix cores (1) or vector FMAs (0)")
    ap.add_argument("--fine-tensor", type=int, default=None,
                    help="FP32 3D fine operator: 1 tensor-product form, n >= 2 the same with n node "
                         "planes per workgroup, 0 node gather (default: the library's)")
    ap.add_argument("--adaptive-stream", type=int, default=0,
                    help="designs in the automated-hybrid comparison on the bridge recipe (0: skip)")
    ap.add_argument("--grid-study", action="store_true",
                    help="the varying-spaced grid comparison (GMG / hybrids) of the 520x520 recipe")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="copy 256 MiB device-to-device first (counter calibration under rocprofv3 --pmc)")
    args = ap.parse_args()
    wl = WORKLOADS[args.workload]
    if args.smoother is None:
        args.smoother = wl.get("smoother", "chebyshev")
    if args.sweeps is None:
        args.sweeps = wl.get("sweeps", 2)
    return args


def progress(msg: str) -> None:
    """A progress line on stderr (the JSON record alone goes to stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def src_hash(names) -> str:
    h = hashlib.sha256()
    for n in names:
        h.update(open(os.path.join(ROOT, "paper_2001_01655_amd", "csrc", n), "rb").read())
    return h.hexdigest()[:16]


def timed_solves(H, f, steps, warmup, rtol):
    import torch
    res = None
    for _ in range(warmup):
        res = H.solve(f, rtol=rtol)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        res = H.solve(f, rtol=rtol)
    torch.cuda.synchronize()
    return time.perf_counter() - t0, res


def event_solves(H, f, n, rtol):
    """Device time of n single solves, each from f resident to u resident,
    between HIP events on the stream the solve runs on (median and range)."""
    import torch
    ts = []
    for _ in range(n):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        H.solve(f, rtol=rtol)
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1))
    ts.sort()
    return {"median_ms": round(ts[len(ts) // 2], 3), "min_ms": round(ts[0], 3), "max_ms": round(ts[-1], 3),
            "solves": n}


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def vcycle_mix(smoother, nu):
    """Operator launches of one level per V-cycle as (reads D^-1, reads the
    previous Chebyshev direction, writes the direction).  The first
    pre-smoothing step is fused into the transfer that makes the level's
    right-hand side; the last step of each smoothing phase keeps no direction."""
    if smoother == "jacobi":
        return [(True, False, False)] * (2 * nu - 1) + [(False, False, False)]
    pre = [(True, k >= 2, k < nu - 1) for k in range(1, nu)]
    post = [(True, k >= 1, k < nu - 1) for k in range(nu)]
    return pre + [(False, False, False)] + post


def fine_prolong_fused(H, p, args):
    """True where the fine level's first post-smoothing step carries the
    prolongation from level 1 (3D, FP32 tensor form, level 1 geometric, every
    element count even): that launch counts with the fine FP32 operator."""
    return (p.dim == 3 and args.fine_tensor != 0 and not args.fine_mfma and H.num_levels() >= 2
            and H.level_info(1)["kind"] == 1 and all(n % 2 == 0 for n in p.nel))


def algorithmic(cls, H, p, args):
    """(flops, bytes) one launch of the class must do, averaged over the
    launches of a V-cycle: the operator's own arithmetic and each operand read
    or written once."""
    dim, n_el, n_nodes = p.dim, p.n_el, p.n_nodes
    nd = dim * 2 ** dim
    mix = vcycle_mix(args.smoother, args.sweeps)

    def extra(w):  # smoother operands per node (upper triangle of D^-1, direction), mean over the mix
        return sum(dv * dim * (dim + 1) // 2 * w + (dr + dw) * dim * w for dv, dr, dw in mix) / len(mix)

    if cls in (0, 1):
        flops = 2.0 * nd * (nd + 1) * n_el                   # KE rows x U_e, then E_e scaling
        w = 8 if cls == 0 else 4
        # x, b (r), y per node, modulus per element, support mask per node,
        # plus the smoother's operands (V-cycle launches only)
        byts = 3 * dim * w * n_nodes + w * n_el + n_nodes + (0 if cls == 0 else extra(w) * n_nodes)
        if cls == 1 and fine_prolong_fused(H, p, args):
            # the first post-smoothing step also reads the level-1 correction
            n1 = H.level_info(1)["n_rows"]
            byts += w * n1 / len(mix)
        return flops, byts
    # level-1 operator, stored in symmetric form: the blocks towards the upper
    # half of the neighbours plus the diagonal block's upper triangle; the
    # lower blocks are the neighbours' stored ones (re-reads, not counted)
    info = H.level_info(1)
    n1 = info["n_rows"] // dim
    nst = 27 if dim == 3 else 9
    nq = (nst - 1) // 2 * dim * dim + dim * (dim + 1) // 2
    flops = 2.0 * nst * dim * dim * n1
    byts = ((nq + 3 * dim) * 4 + extra(4)) * n1
    return flops, byts


def roofline_entry(cls, launches, total_ms, H, p, args):
    avg_s = total_ms / 1e3 / max(launches, 1)
    flops, byts = algorithmic(cls, H, p, args)
    # the fine operators in the tensor-product form (3D) do about a fifth of
    # the dense KE arithmetic, far below their HBM time: HBM is their roof
    tensor = cls in (0, 1) and p.dim == 3 and args.fine_tensor != 0 and not (cls == 1 and args.fine_mfma)
    if cls == 2 or tensor:
        ach = byts / avg_s / 1e9
        e = {"bound": "hbm", "achieved": round(ach, 1), "peak": PEAK["hbm_GBs"], "unit": "GB/s",
             "frac": round(ach / PEAK["hbm_GBs"], 4)}
    else:
        peak = PEAK["fp64_TFs"] if cls == 0 else PEAK["fp32_TFs"]
        ach = flops / avg_s / 1e12
        e = {"bound": "alu", "achieved": round(ach, 2), "peak": peak, "unit": "TFLOP/s",
             "frac": round(ach / peak, 4)}
    e.update({"kernel": {0: "fine operator FP64 (q = K~p, outer loop)",
                         1: "fine operator FP32 (V-cycle smoothing / residual)",
                         2: "level-1 stencil operator FP32 (V-cycle)"}[cls] +
                        (", tensor-product form" if tensor else ""),
              "launches": launches, "avg_us": round(avg_s * 1e6, 2),
              "algorithmic_flops_per_launch": flops, "algorithmic_bytes_per_launch": byts,
              "traffic": None})
    # HBM bytes per launch from committed rocprofv3 counter summaries, valid
    # only while the kernel source is the one that was profiled
    tp = os.path.join(ROOT, "profiles", f"traffic_class{cls}.json")
    if os.path.exists(tp):
        t = json.load(open(tp))
        # (the summaries are taken on the default workload, the 3D cantilever)
        if (t.get("source_sha") == src_hash(KERNEL_SOURCES[cls]) and t.get("mix") == [args.smoother, args.sweeps]
                and args.workload == t.get("workload", "cantilever3d")):
            e["traffic"] = t.get("bytes_per_launch")
            e["traffic_ratio_to_algorithmic"] = round(t["bytes_per_launch"] / byts, 3)
    return e


def oracle_error(cfg_name, u, c):
    """Relative error of the headline solution against the oracle's solution at
    rtol 1e-12 (stored by tests/golden/make_golden.py, which calls only the
    oracle): u over 4096 seeded free dofs, ||u||_2, and the compliance."""
    path = os.path.join(ROOT, "tests", "golden", f"solve_{cfg_name}.json")
    if not os.path.exists(path):
        return None
    g = json.load(open(path))
    import numpy as np
    idx = np.asarray(g["sample_dofs"], dtype=np.int64)
    ref = np.asarray(g["sample_u"])
    uu = u.detach().cpu().numpy().reshape(-1)
    return {"err_u_sampled": float(np.linalg.norm(uu[idx] - ref) / np.linalg.norm(ref)),
            "err_norm_u": abs(float(np.linalg.norm(uu)) - g["norm_u"]) / g["norm_u"],
            "err_c": abs(c - g["compliance"]) / abs(g["compliance"]),
            "reference": f"oracle FP64 MG-PCG at rtol 1e-12 (true relres {g['oracle']['true_relres']:.1e}), "
                         f"{len(idx)} sampled dofs"}


def cpu_baseline(cfg_name, args):
    """Oracle (CPU, FP64, single thread) on a bounded sample of the same
    recipe; solve to rtol 1e-8 timed, setup excluded."""
    from threadpoolctl import threadpool_limits

    import synth
    from oracle import fem, mg
    if cfg_name == "cantilever3d":
        p = synth.cantilever_3d(nel=(128, 64, 64))
        L = 5
        sample = ("3D cantilever recipe at 128x64x64 (1,623,075 dofs, 30% of the volume), 5 levels, "
                  "three solves to rtol 1e-8, mean")
    elif cfg_name == "cantilever2d":
        p = synth.cantilever_2d(nel=(512, 256))
        L = 6
        sample = "2D cantilever recipe at 512x256 (263,682 dofs), 6 levels, three solves to rtol 1e-8, mean"
    else:
        return None
    KE = fem.element_stiffness(p.dim, p.nu)
    E = fem.simp(p.rho, p.p, p.E0, p.Emin)
    H = mg.build_geometric(p.nel, E, KE, p.fixed, L, omega=0.5, nu_pre=args.sweeps, nu_post=args.sweeps,
                           smoother=args.smoother, cheb_lower=args.cheb_lower)
    reps = 3

    def timed():
        t0 = time.perf_counter()
        for _ in range(reps):
            r = mg.mg_pcg(H, p.loads[0], 1e-8)
        return (time.perf_counter() - t0) / reps, r

    with threadpool_limits(limits=1):
        dt, r = timed()
    # the same solves with the BLAS thread pool at its default size: SciPy's
    # sparse products (every operator and transfer) run on one thread either
    # way; only the dense coarsest solve can use more
    dt_all, _ = timed()
    return {"value": round(p.n_dof / dt / 1e6, 4), "unit": "MDoF/s", "cores": 1, "kind": "oracle",
            "sample": sample + f", {args.smoother} {args.sweeps}/{args.sweeps} smoothing as on the GPU",
            "seconds": round(dt, 3), "iters": r.iters,
            "all_cores": {"value": round(p.n_dof / dt_all / 1e6, 4), "seconds": round(dt_all, 3),
                          "threads_available": os.cpu_count(),
                          "parallel_parts": "dense coarsest Cholesky solve (BLAS); sparse products single-threaded"},
            "host": cpu_model(), "host_cpus": os.cpu_count()}


def served_requests(n: int, rate_per_s: float, n_designs: int = 20, seed: int = 5) -> list:
    """The served stream: sizes drawn from {2D 128x64, 2D 512x256, 3D 48^3,
    3D 96x48x48}, 1-4 load cases, smoothed seeded densities and a sequence of
    seeded design updates, Poisson arrivals."""
    import synth
    from paper_2001_01655_amd.serving import Request
    arrivals = synth.poisson_arrivals(n, rate_per_s, seed)
    out = []
    for rid in range(n):
        p = synth.served_request(rid, seed)
        dens = synth.design_sequence(p.rho, p.nel, seed + rid)
        out.append(Request(rid, float(arrivals[rid]), p.nel, p.fixed, p.loads, dens, n_designs,
                           material=dict(p=p.p, E0=p.E0, Emin=p.Emin, nu=p.nu)))
    return out


def served_leg(n_req: int, n_designs: int, smoother: str = "chebyshev", sweeps: int = 2, seed: int = 5,
               warm_steps: int = 4, hybrid_every: int = 8, fractions=(0.5, 0.7, 0.9)):
    """The served stream (mixed 2D/3D sizes, 1-4 load cases, design updates
    with warm starts, rtol 1e-6; every hybrid_every-th request a hybrid
    hierarchy, smoothed aggregation below two geometric levels): first every
    request at t = 0 to find the saturation throughput, then Poisson arrivals
    at fractions of that request rate; latency = arrival to the request's last
    solve.  The record's p50 / p99 / solves_per_s are those at 70%.  Densities
    are generated before the timed runs."""
    import dataclasses

    import numpy as np

    import synth
    from paper_2001_01655_amd.serving import GpuEngine, Server
    reqs = served_requests(n_req, rate_per_s=1.0, n_designs=n_designs, seed=seed)
    if hybrid_every > 0:
        for r in reqs:
            if r.rid % hybrid_every == hybrid_every - 1:
                r.options = dict(r.options, n_geometric=2, max_coarse=1000)
    hybrid_ids = {r.rid for r in reqs if "n_geometric" in r.options}
    for i, r in enumerate(reqs):
        for t in range(n_designs):
            r.densities(t)
        if (i + 1) % 25 == 0:
            progress(f"served: densities of {i + 1}/{n_req} requests")
    warm = warm_steps if smoother == "chebyshev" else 0
    eng = GpuEngine(smoother=SMOOTHERS[smoother], nu_pre=sweeps, nu_post=sweeps, cheb_warm_steps=warm)
    budget = 64 << 30
    Server(eng, budget, max_slots=8, chunk=4, rtol=1e-6, workers=4).run(
        [dataclasses.replace(r, arrival=0.0, n_designs=2) for r in reqs[:8]])          # warm-up
    sat = Server(eng, budget, max_slots=8, chunk=4, rtol=1e-6, workers=4).run(
        [dataclasses.replace(r, arrival=0.0) for r in reqs])
    progress(f"served: saturation {sat['solves_per_s']:.0f} solves/s")
    sweep = []
    main = None
    for fr in fractions:
        rate = fr * n_req / sat["makespan_s"]
        arr = synth.poisson_arrivals(n_req, rate, seed)
        res = Server(eng, budget, max_slots=8, chunk=4, rtol=1e-6, workers=4).run(
            [dataclasses.replace(r, arrival=float(a)) for r, a in zip(reqs, arr)])
        ok = all(st == 0 for o in res["outcomes"] for st in o.status)
        by_kind = {}
        for kind, sel in (("geometric", False), ("hybrid", True)):
            lat = [o.latency * 1e3 for o in res["outcomes"] if hybrid_ids.__contains__(o.rid) == sel]
            if lat:
                by_kind[kind] = {"requests": len(lat), "p50_ms": round(float(np.percentile(lat, 50)), 2),
                                 "p99_ms": round(float(np.percentile(lat, 99)), 2)}
        sweep.append({"fraction_of_saturation": fr, "arrival_rate_per_s": round(rate, 3),
                      "p50_ms": round(res["p50_ms"], 2), "p99_ms": round(res["p99_ms"], 2),
                      "solves_per_s": round(res["solves_per_s"], 1), "all_converged": ok,
                      "latency_by_kind": by_kind})
        progress(f"served: {fr:.0%} of saturation, p50 {res['p50_ms']:.1f} ms, p99 {res['p99_ms']:.1f} ms")
        if abs(fr - 0.7) < 1e-9:
            main = res
    res = main
    iters = [i for o in res["outcomes"] for d in o.iters for i in d]
    ok = all(st == 0 for o in res["outcomes"] for st in o.status)
    return {"p50_ms": round(res["p50_ms"], 2), "p99_ms": round(res["p99_ms"], 2),
            "solves_per_s": round(res["solves_per_s"], 1),
            "arrival_rate_per_s": next(x["arrival_rate_per_s"] for x in sweep if x["fraction_of_saturation"] == 0.7),
            "latency_by_kind": next(x["latency_by_kind"] for x in sweep if x["fraction_of_saturation"] == 0.7),
            "saturation_solves_per_s": round(sat["solves_per_s"], 1), "rate_sweep": sweep, "requests": n_req,
            "hybrid_requests": sum(1 for r in reqs if "n_geometric" in r.options),
            "designs_per_request": n_designs, "solves": res["solves"], "all_converged": ok,
            "mean_iters": round(float(np.mean(iters)), 2) if iters else None,
            "max_slots": 8, "chunk": 4, "workers": 4, "latency": "request arrival to its last solve",
            "grouping": "idle solves advance together once no chunk of another solve is running",
            "launches": "right-hand sides of requests with the same level structure share each launch",
            "sizes": "2D 128x64, 2D 512x256, 3D 48^3, 3D 96x48x48; 1-4 load cases; rtol 1e-6",
            "smoothing": f"{smoother} {sweeps}/{sweeps}", "cheb_warm_steps": warm}


def adaptive_leg(n_designs: int, nel=(128, 64, 64), seed: int = 4):
    """Design stream on the thin-strut bridge recipe (warm-started solves to
    rtol 1e-8, FP32 V-cycle in FCG, block Jacobi 1/1): pure GMG with 6 levels,
    the fixed hybrid (2 geometric levels, then aggregation below 1000 dofs) and
    the automated hybrid (start with 6 geometric levels, one fewer after every
    solve over 200 iterations).  Setup/update and solve are timed per design."""
    import torch

    import synth
    from paper_2001_01655_amd import Hierarchy
    p = synth.bridge_3d(nel=nel, seed=seed)
    rhos = [p.rho]
    for t in range(1, n_designs):
        rhos.append(synth.density_update(rhos[-1], p.nel, seed=seed, step=t))
    f = torch.tensor(p.loads[0], device="cuda")
    variants = {"gmg6": dict(n_levels=6), "hybrid2": dict(n_geometric=2, max_coarse=1000),
                "adaptive": dict(n_levels=6, max_coarse=1000, adapt_iters=200)}
    out = {}
    for name, o in variants.items():
        rec = dict(iters=[], geometric=[], setup_ms=[], solve_ms=[])
        H, u = None, None
        for t, rho in enumerate(rhos):
            rd = torch.tensor(rho, device="cuda")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if H is None:
                H = Hierarchy(p.nel, rd, p.fixed, p=p.p, E0=p.E0, Emin=p.Emin, nu=p.nu, omega=0.5, nu_pre=1,
                              nu_post=1, vcycle_fp=32, outer=0, max_iters=5000, **o)
            else:
                H.update_density(rd)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            r = H.solve(f, rtol=1e-8, u0=u)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            u = r.u
            kinds = [H.level_info(l)["kind"] for l in range(H.num_levels())]
            rec["iters"].append(int(r.iters[0]))
            rec["geometric"].append(sum(k != 2 for k in kinds))
            rec["setup_ms"].append(round((t1 - t0) * 1e3, 2))
            rec["solve_ms"].append(round((t2 - t1) * 1e3, 2))
        H.close()
        rec["total_ms"] = round(sum(rec["setup_ms"]) + sum(rec["solve_ms"]), 1)
        out[name] = rec
    out["workload"] = (f"3D bridge recipe {nel[0]}x{nel[1]}x{nel[2]} ({p.n_dof:,} dofs), {n_designs} designs, "
                       "warm-started, rtol 1e-8")
    return out


def multi_rhs_leg(H, p, n_rhs: int = 6, reps: int = 3):
    """Six load cases of the workload's mesh solved together (x0 = 0, rtol 1e-8;
    one launch per operation serves all six) against the same six solved one
    after another."""
    import torch

    import synth
    F = torch.tensor(synth.served_loads(p.nel, p.dim, n_rhs), device="cuda")
    H.solve(F, rtol=1e-8)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        r = H.solve(F, rtol=1e-8)
    torch.cuda.synchronize()
    together = (time.perf_counter() - t0) / reps
    t0 = time.perf_counter()
    for _ in range(reps):
        for k in range(n_rhs):
            H.solve(F[k], rtol=1e-8)
    torch.cuda.synchronize()
    alone = (time.perf_counter() - t0) / reps
    return {"n_rhs": n_rhs, "ms_together": round(together * 1e3, 2), "ms_one_by_one": round(alone * 1e3, 2),
            "speedup": round(alone / together, 3), "iters": [int(i) for i in r.iters],
            "MDoF_s_together": round(p.n_dof * n_rhs / together / 1e6, 1)}


def grid_leg(pairs=((16, 16), (16, 256), (256, 16), (64, 64))):
    """Varying-spaced grid of Sec. 4.3 (520x520, 8-element beams and columns at
    spacings sx, sy; rtol 1e-8, FP32 V-cycle in FCG, block Jacobi w = 0.5 1/1):
    setup and solve per hierarchy, pure GMG with 5 levels (ceil(n/2) coarsening,
    2312 coarsest dofs), the hybrid with 4 geometric levels and aggregation below
    1500 dofs, and aggregation from the second level on."""
    import torch

    import synth
    from paper_2001_01655_amd import Hierarchy
    variants = {"gmg5": dict(n_levels=5), "hybrid4": dict(n_geometric=4, max_coarse=1500),
                "hybrid2": dict(n_geometric=2, max_coarse=1500)}
    out = {}
    for sx, sy in pairs:
        p = synth.grid_2d(sx, sy)
        f = torch.tensor(p.loads[0], device="cuda")
        rec = {}
        for name, o in variants.items():
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            H = Hierarchy(p.nel, p.rho, p.fixed, p=p.p, E0=p.E0, Emin=p.Emin, nu=p.nu, omega=0.5, nu_pre=1,
                          nu_post=1, vcycle_fp=32, outer=0, max_iters=20000, **o)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            r = H.solve(f, rtol=1e-8)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            rec[name] = {"iters": int(r.iters[0]), "setup_ms": round((t1 - t0) * 1e3, 1),
                         "solve_ms": round((t2 - t1) * 1e3, 1), "levels": H.num_levels(),
                         "coarsest_dofs": H.level_info(H.num_levels() - 1)["n_rows"]}
            H.close()
        out[f"{sx}x{sy}"] = rec
    out["workload"] = "2D grid 520x520 Q4 (543,762 dofs), 8-element features, rtol 1e-8"
    return out


def eigen_leg(reps: int = 3):
    """Stability eigenproblem (Sec. 2) on the 256x1024 column of Sec. 4
    (prismatic start design, unit compressive load on the top edge, bottom
    clamped; 526,850 dofs): displacements by the mixed FCG to rtol 1e-8, the
    stress stiffness, then the six largest eigenvalues of
    K_sigma Phi = lambda K Phi by generalized Davidson (Algorithm 2; j_min 10,
    j_max 25, tol 1e-6, stagnation 1e-13) with one FP32 V-cycle (5 geometric
    levels, 2210 coarsest dofs, block Jacobi 0.5, 1/1) as the preconditioner,
    from 10 seeded start vectors.  Wall time of tm_eigs (host decisions and
    transfers included), mean over reps after one warm call.  The web design
    (voids) is run with a cap of 2000 expansions, for its convergence only."""
    import numpy as np
    import torch

    import synth
    from paper_2001_01655_amd import Hierarchy
    out = {}
    for name, uni in (("prismatic", True), ("web_design", False)):
        p = synth.column_2d(uniform=uni)
        H = Hierarchy(p.nel, p.rho, p.fixed, p=p.p, E0=p.E0, Emin=p.Emin, nu=p.nu, n_levels=5, omega=0.5,
                      nu_pre=1, nu_post=1, vcycle_fp=32)
        r = H.solve(torch.tensor(p.loads[0], device="cuda"), rtol=1e-8)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        H.stress_stiffness(r.u)
        torch.cuda.synchronize()
        t_ks = time.perf_counter() - t0
        V0 = np.random.default_rng(3).standard_normal((10, p.n_dof))
        V0[:, p.fixed] = 0.0
        v0 = torch.tensor(V0, device="cuda")
        cap = 1000 if uni else 2000
        H.eigs(v0, nev=6, max_iters=cap, want_vectors=False)
        n_rep = reps if uni else 1
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(n_rep):
            lam, _, it, nc, st = H.eigs(v0, nev=6, max_iters=cap)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / n_rep
        rec = {"iters": int(it), "n_conv": int(nc), "ms": round(dt * 1e3, 1),
               "ms_per_iter": round(dt * 1e3 / max(it, 1), 3), "stress_stiffness_ms": round(t_ks * 1e3, 2),
               "lambda": [float(f"{v:.8g}") for v in lam], "linear_iters": int(r.iters[0])}
        if uni:
            pcr = np.pi ** 2 * (p.nel[0] ** 3 / 12.0) / (4.0 * p.nel[1] ** 2)
            rec["lambda1_x_euler_load"] = round(float(lam[0] * pcr), 4)
        else:
            rec["max_iters"] = cap
        out[name] = rec
        H.close()
    out["workload"] = "2D column 256x1024 Q4 (526,850 dofs), 6 eigenpairs, GMG5 FP32 V-cycle preconditioner"
    return out


def stability_stream_leg(n_designs: int = 4):
    """The stability workflow over a stream of designs (Sec. 2 / Sec. 4 column
    example): the 256x1024 column starting from the prismatic design, each next
    design a seeded smooth perturbation (rho + 0.05 G(N(0,1)), clipped to
    [1e-3, 1]); per design: density update, displacement solve warm-started
    from the previous u (rtol 1e-8), stress stiffness, six eigenpairs by
    generalized Davidson started from the previous design's eigenvectors plus
    four seeded vectors (Sec. 4: previous eigenvectors as the initial search
    space), and, for comparison, from ten seeded vectors."""
    import numpy as np
    import torch

    import synth
    from paper_2001_01655_amd import Hierarchy
    p = synth.column_2d(uniform=True)
    seq = synth.design_sequence(p.rho, p.nel, seed=7)
    H = Hierarchy(p.nel, p.rho, p.fixed, p=p.p, E0=p.E0, Emin=p.Emin, nu=p.nu, n_levels=5, omega=0.5,
                  nu_pre=1, nu_post=1, vcycle_fp=32)
    f = torch.tensor(p.loads[0], device="cuda")
    rng = np.random.default_rng(11)
    cold = rng.standard_normal((10, p.n_dof))
    cold[:, p.fixed] = 0.0
    cold = torch.tensor(cold, device="cuda")
    u, phi, out = None, None, []
    for t in range(n_designs):
        if t > 0:
            H.update_density(torch.tensor(seq(t), device="cuda"))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = H.solve(f, rtol=1e-8, u0=u)
        u = r.u
        H.stress_stiffness(u)
        v0 = cold if phi is None else torch.cat([phi, cold[:4]])
        lam, phi, it, nc, st = H.eigs(v0, nev=6)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        lam_c, _, it_c, nc_c, _ = H.eigs(cold, nev=6, want_vectors=False)
        out.append({"design": t, "solve_iters": int(r.iters[0]), "eig_iters": int(it), "eig_iters_cold_start": int(it_c),
                    "n_conv": int(nc), "lambda1": float(f"{lam[0]:.8g}"), "ms_solve_and_eigs": round(dt * 1e3, 1)})
    H.close()
    return {"designs": out, "workload": "2D column 256x1024, prismatic start then seeded perturbations, GMG5"}


def filter_leg(nel, reps: int = 50):
    """tm_density_filter (radius 1.5) on the workload's element grid: mean time
    per launch from events around reps back-to-back calls of the C function on
    the current stream (buffers and arguments prepared once); algorithmic
    bytes = one FP64 read and one write per element."""
    import ctypes as C

    import torch

    from paper_2001_01655_amd import _lib as L
    n = 1
    for v in nel:
        n *= int(v)
    x = torch.rand(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    mesh = L.make_mesh(tuple(int(v) for v in nel))
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    xp, yp = C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr())
    out = {}
    for tr in (0, 1):
        L.check(L.LIB.tm_density_filter(C.byref(mesh), 1.5, tr, xp, yp, stream))
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            L.LIB.tm_density_filter(C.byref(mesh), 1.5, tr, xp, yp, stream)
        e1.record()
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) * 1e3 / reps
        gbs = 16.0 * n / (us * 1e-6) / 1e9
        out["transpose" if tr else "forward"] = {"avg_us": round(us, 2), "achieved_GBs": round(gbs, 1),
                                                 "frac_hbm": round(gbs / PEAK["hbm_GBs"], 4)}
    out["elements"] = n
    out["radius"] = 1.5
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; a multi-GPU decomposition of the "
                                   "solve is not implemented", "n_gpus": args.gpus}))
        sys.exit(2)
    import torch

    import synth
    from paper_2001_01655_amd import Hierarchy

    if args.eigen_only:
        print(json.dumps({"eigen": eigen_leg()}))
        return
    wl = WORKLOADS[args.workload]
    p = synth.get(wl["cfg"])
    if args.calibrate_copy:
        a = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    f = torch.tensor(p.loads[0], device="cuda")
    rtol = 1e-8
    opts = dict(wl["opts"])
    if args.n_geometric is not None:
        if "n_geometric" not in opts:
            sys.exit("--n-geometric applies to the hybrid workloads only")
        opts["n_geometric"] = args.n_geometric
    if wl["levels"] is not None:
        opts["n_levels"] = args.levels or wl["levels"]

    def build(vfp, outer):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        kw = dict(omega=0.5)
        kw.update(opts)
        if args.fine_tensor is not None:
            kw["fine_tensor"] = args.fine_tensor
        H = Hierarchy(p.nel, p.rho, p.fixed, p=p.p, E0=p.E0, Emin=p.Emin, nu=p.nu,
                      nu_pre=args.sweeps, nu_post=args.sweeps, smoother=SMOOTHERS[args.smoother],
                      cheb_lower=args.cheb_lower, vcycle_fp=vfp,
                      outer=outer, fine_mfma=args.fine_mfma, **kw)
        torch.cuda.synchronize()
        return H, time.perf_counter() - t0

    H, t_setup = build(32, 0)
    progress("headline solves")
    dt, res = timed_solves(H, f, args.steps, args.warmup, rtol)
    ms = dt / args.steps * 1e3
    value = p.n_dof * args.steps / dt / 1e6
    detail = {"mixed": dict(iters=res.iters[0], relres=res.relres[0], compliance=res.compliance[0],
                            setup_ms=round(t_setup * 1e3, 2), levels=H.num_levels(),
                            device_time_per_solve=event_solves(H, f, 5, rtol))}
    coarsest = H.level_info(H.num_levels() - 1)["n_rows"]
    line = {
        "metric": "MDoF/s to rtol 1e-8 (FP32 V-cycle vs FP64 PCG)",
        "value": round(value, 2),
        "unit": "MDoF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 V-cycle + f64 CG",
        "data": "synthetic",
        "config": {"workload": workload_label(wl, args, H.num_levels(), coarsest), "n_dof": p.n_dof,
                   "iterations": res.iters[0]},
    }
    if not args.no_profile:
        classes = [0, 1, 2]
        for c in classes:
            H.kernel_timing(c, True)
        H.solve(f, rtol=rtol)
        torch.cuda.synchronize()
        ents = {}
        for c in classes:
            n, tot = H.kernel_timing_read(c)
            H.kernel_timing(c, False)
            if n:
                ents[c] = roofline_entry(c, n, tot, H, p, args)
                ents[c]["share_of_step_time"] = round(tot / ms, 4)
        if ents:
            dom = max(ents, key=lambda c: ents[c]["share_of_step_time"])
            line["roofline"] = ents[dom]
            line["roofline_other_kernels"] = [ents[c] for c in ents if c != dom]
    u_mixed = res.u.clone()
    ref = oracle_error(wl["cfg"], u_mixed, res.compliance[0])
    if ref:
        line["oracle_error"] = ref
    if not args.no_side_legs:
        progress("multi-RHS leg")
        line["multi_rhs"] = multi_rhs_leg(H, p)
    H.close()
    if not args.no_side_legs:
        line["density_filter"] = filter_leg(p.nel)
    if args.stability:
        line["eigen"] = eigen_leg()
        line["stability_stream"] = stability_stream_leg()
    if not args.no_fp64:
        progress("FP64 PCG comparison")
        H64, t64s = build(64, 1)
        k64 = max(1, args.steps // 2)
        dt64, r64 = timed_solves(H64, f, k64, 1, rtol)
        v64 = p.n_dof * k64 / dt64 / 1e6
        du = float((r64.u - u_mixed).norm() / r64.u.norm())
        detail["fp64_pcg"] = dict(value=round(v64, 2), unit="MDoF/s", iters=r64.iters[0], relres=r64.relres[0],
                                  setup_ms=round(t64s * 1e3, 2), rel_diff_u_vs_mixed=du)
        line["speedup_vs_fp64_pcg"] = round(value / v64, 3)
        H64.close()
    line["detail"] = detail
    if args.served > 0:
        progress("served stream")
        line["served"] = served_leg(args.served, args.served_designs, args.served_smoother, args.served_sweeps,
                                    hybrid_every=args.served_hybrid_every,
                                    warm_steps=args.served_warm_steps)
    if args.grid_study:
        line["grid_study"] = grid_leg()
    if args.adaptive_stream > 0:
        line["adaptive_stream"] = adaptive_leg(args.adaptive_stream)
    if not args.no_cpu_baseline:
        progress("oracle baseline on the host")
        cb = cpu_baseline(wl["cfg"], args)
        if cb:
            line["cpu_baseline"] = cb
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
