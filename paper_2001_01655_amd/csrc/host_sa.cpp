// Smoothed-aggregation levels of the hybrid hierarchy (placeholder until the
// aggregation setup is built).
#include "tm_internal.h"

namespace tmi {

void build_sa_levels(tm_hierarchy* h, hipStream_t s) {
    (void)h;
    (void)s;
    fail(TM_ERR_ARG, "smoothed-aggregation levels are not available in this build");
}

void numeric_sa_levels(tm_hierarchy* h, hipStream_t s) {
    (void)h;
    (void)s;
    fail(TM_ERR_ARG, "smoothed-aggregation levels are not available in this build");
}

}  // namespace tmi
