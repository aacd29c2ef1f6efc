// Issue-rate probe for the roofline of the FP64 pair loop: SIMD cycles per
// wave-level v_fma_f64 and per v_rsq_f64 when the whole chip runs
// independent streams of them.  The force loop's cost per pair is a fixed
// mix of these two kinds of instruction, so the two rates give the pair
// throughput its instruction mix allows at the clock the chip sustains under
// FP64 load, next to the nominal FP64 peak.
#include "common.h"

namespace mstar {

namespace {

constexpr int kProbeBlocks = 2048, kProbeThreads = 256, kProbeIters = 4096, kProbeChains = 8;

// MODE 0: chains of fused multiply-adds; MODE 1: chains of hardware 1/sqrt.
template <int MODE>
__global__ __launch_bounds__(kProbeThreads) void k_issue_probe(double *out, double seed) {
    const int t = blockIdx.x * kProbeThreads + threadIdx.x;
    double a[kProbeChains];
#pragma unroll
    for (int q = 0; q < kProbeChains; ++q) a[q] = seed + 1e-3 * (double)(t + q);
    for (int i = 0; i < kProbeIters; ++i) {
#pragma unroll
        for (int q = 0; q < kProbeChains; ++q) {
            if (MODE == 0) a[q] = fma(a[q], 0.999999, 1e-7);
            else a[q] = __builtin_amdgcn_rsq(a[q]);
        }
    }
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < kProbeChains; ++q) s = s + a[q];
    out[t] = s;   // t < kProbeBlocks * kProbeThreads, the size of out
}

}  // namespace

size_t issue_probe_bytes() { return sizeof(double) * (size_t)kProbeBlocks * kProbeThreads; }

// Cycles (at clock_ghz) per wave-level instruction per SIMD for both modes;
// `out` must hold issue_probe_bytes().
hipError_t issue_probe(hipStream_t s, double *out, int n_simd, double clock_ghz, double cycles[2]) {
    hipEvent_t e0, e1;
    hipError_t err = hipEventCreate(&e0);
    if (err != hipSuccess) return err;
    if ((err = hipEventCreate(&e1)) != hipSuccess) { (void)hipEventDestroy(e0); return err; }
    const double wave_ops = (double)kProbeBlocks * kProbeThreads / 64.0 * kProbeIters * kProbeChains;
    for (int mode = 0; mode < 2 && err == hipSuccess; ++mode) {
        float best = 0.f;
        for (int rep = 0; rep < 3 && err == hipSuccess; ++rep) {
            (void)hipEventRecord(e0, s);
            if (mode == 0) k_issue_probe<0><<<kProbeBlocks, kProbeThreads, 0, s>>>(out, 1.5);
            else k_issue_probe<1><<<kProbeBlocks, kProbeThreads, 0, s>>>(out, 1.5);
            (void)hipEventRecord(e1, s);
            if ((err = hipEventSynchronize(e1)) != hipSuccess) break;
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (rep == 0 || ms < best) best = ms;
        }
        cycles[mode] = (double)best * 1e-3 * clock_ghz * 1e9 * (double)n_simd / wave_ops;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return err;
}

}  // namespace mstar
