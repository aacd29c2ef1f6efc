// Interface between the host driver and the batched small-system kernel
// (kernels_batch.hip).
#pragma once
#include "common.h"

namespace mstar {

constexpr int kBatchMaxN = 64;     // bodies per system in the batched path
constexpr int kBatchMaxKF = 8;     // k_fix supported by the batched path

struct BatchParams {
    double G, eta, alpha, gamma, a_gbs, f_min, f_max, q_first, t_tol, h_init;
    int64_t max_steps;
    int32_t k_fix, n_d, max_halvings, max_time_iter, rebuild_every, pad;
};

// Same layout as mstar_batch_stats.
struct BatchStat {
    int32_t status, reserved;
    int64_t acc, rej, nforce, nrebuild, ntopo, time_iters;
    double t_reached, eps_last, h_next, h_last;
};

struct BatchArgs {
    int32_t n_coop;           // systems integrated by a whole workgroup (64-lane tiles)
    int32_t n_wave;           // systems integrated by a single wave (wave_lanes-wide tiles)
    const int32_t *order;     // [n_coop] cooperative systems, then [n_wave] wave systems, each by decreasing cost
    int32_t *queue;           // [2] next positions in the two lists (zeroed by the reset kernel)
    const int64_t *off;       // [n_sys + 1] body offsets
    const double *m;          // [N_total]
    double *x, *v;            // [N_total][3], read at t0 and overwritten with the end state
    const double *t0, *t_end; // [n_sys]
    BatchStat *stat;          // [n_sys]
    double *hrec;             // [n_sys][hrec_cap] fictitious step of every accepted step (nullptr: none)
    int64_t hrec_cap;
    BatchParams p;
};

// Launch the queue reset and the persistent batch kernel on stream s.  `a`
// is a device copy of the arguments (its queue pointer must equal `queue`).
// wave_lanes in {0, 16, 32, 64}; nwg persistent workgroups of 256 threads.
int launch_batch(hipStream_t s, const BatchArgs *a, int32_t *queue, int kf, int wave_lanes, int nwg);
// Dynamic LDS bytes of the batch kernel for (kf, wave_lanes); 0 if unsupported.
size_t batch_smem_bytes(int kf, int wave_lanes);
// Resident workgroups per CU of that kernel (0 if it cannot launch).
int batch_blocks_per_cu(int kf, int wave_lanes);

}  // namespace mstar
