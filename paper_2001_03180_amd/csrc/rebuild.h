// Interface between the host driver and the coordinate round-trip kernel
// (kernels_rebuild.hip).
#pragma once
#include "common.h"

namespace mstar {

constexpr int kRebuildMaxN = 512;   // bodies per system (one wave, 8 bodies per lane)

struct RebuildArgs {
    const int64_t *off;        // [n_sys + 1] body offsets
    const int32_t *kind;       // [n_sys] 0: MST, 1: chain; + 2: plain centre-of-mass sums
    const double *m;           // [n_tot]
    double *x, *v;             // [n_tot][3] state, carried from launch to launch
    int64_t n_cycles, n_tot;
    int32_t n_out;
    double *x_out, *v_out;     // [n_out][n_tot][3]
    double *level_sum;         // [n_sys] sum over cycles of the structure's mean level
    int32_t *next_out;         // [n_sys] next output slot
};

void launch_rebuild(hipStream_t s, const RebuildArgs *a, int n_sys, int64_t c0, int64_t c1);

}  // namespace mstar
