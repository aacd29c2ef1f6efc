// mstar_force_noalloc: the force evaluation of mstar_force for callers that
// cannot allocate device memory (code under HIP graph capture, serving loops).
// Everything the kernels need beyond the caller's inputs and outputs lives in
// one file-scope device array, `scratch`, of kScratchBytes; each device gets
// its own copy, whose address is looked up once per device with
// hipGetSymbolAddress and kept in g_scratch.  The call only enqueues work on
// the caller's stream: no allocation, no host copy, no synchronisation.
// Invalid trees therefore cannot be reported by the return code; they give
// NaN outputs instead.  Calls that overlap on one device share the array and
// race.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>

#include "../../include/mstar.h"
#include "common.h"

using namespace mstar;

namespace {

constexpr int kNaMaxN = 8192;           // largest N (MSTAR_NOALLOC_MAX_N)
constexpr int kNaSplits = 16;           // j-splits of the pairwise force kernel at most
constexpr int kNaParts = kNaSplits + 1; // plus the close-pair correction partial
constexpr int kNaNib = (kNaMaxN + 63) / 64;
constexpr int kNaMaxDevices = 64;

// Layout of the scratch array (byte offsets, each 256-aligned).
constexpr size_t al(size_t b) { return (b + 255) & ~(size_t)255; }
constexpr size_t kOffP = 0;                                             // d4 [N] positions + mass
constexpr size_t kOffX0 = kOffP + al(sizeof(d4) * kNaMaxN);             // d4 [N] edge vectors
constexpr size_t kOffDX = kOffX0 + al(sizeof(d4) * kNaMaxN);            // d4 [N] zero increments
constexpr size_t kOffA0 = kOffDX + al(sizeof(d4) * kNaMaxN);            // d4 [N] accelerations
constexpr size_t kOffPart = kOffA0 + al(sizeof(d4) * kNaMaxN);          // d4 [parts][N] force partials
constexpr size_t kOffUpart = kOffPart + al(sizeof(d4) * kNaParts * kNaMaxN);   // double [nib][parts]
constexpr size_t kOffInt = kOffUpart + al(sizeof(double) * kNaNib * kNaParts); // int32 arrays below
constexpr size_t kIntN = al(sizeof(int32_t) * (kNaMaxN + 1));
// int32 arrays: parent, level, child_off, child_idx, rkA, rkB, nxtA, nxtB, cnt, fill
constexpr size_t kOffCtl = kOffInt + 10 * kIntN;                        // Ctl, error flag, U
constexpr size_t kScratchBytes = kOffCtl + 256;

struct NaTail {
    Ctl ctl;
    int32_t bad;     // the tree failed a check: outputs are NaN
    int32_t pad;
    double U;
};
static_assert(sizeof(NaTail) <= 256, "scratch tail");

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void *g_scratch[kNaMaxDevices] = {};
int g_cap[kNaMaxDevices] = {};          // resident pairwise force workgroups on the chip, by device

// Address of this device's scratch (looked up on the first call on the
// device, with that device current) and the force kernel's chip capacity.
int scratch_for(int dev, void **out, int *cap) {
    if (dev < 0 || dev >= kNaMaxDevices) return MSTAR_E_UNSUPPORTED;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return MSTAR_E_DEVICE;
        int ncu = 0;
        if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu <= 0)
            return MSTAR_E_DEVICE;
        g_cap[dev] = force_blocks_per_cu(2) * ncu;
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    *cap = g_cap[dev];
    return MSTAR_OK;
}

// Pack the inputs into the scratch layout; parents outside [-1, n) are
// replaced by -1 and flag the call.  One workgroup (n <= kNaMaxN).
__global__ __launch_bounds__(1024) void k_na_prep(int n, const double *m, const double *rho, const int32_t *parent,
                                                  const double *X, d4 *P, d4 *X0, d4 *dX, int32_t *par,
                                                  NaTail *tail) {
    __shared__ int bad;
    if (threadIdx.x == 0) bad = 0;
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        int p = parent[i];
        if (p < -1 || p >= n || p == i) {
            bad = 1;
            p = -1;
        }
        par[i] = p;
        P[i] = d4{rho[3 * i], rho[3 * i + 1], rho[3 * i + 2], m[i]};
        X0[i] = d4{X[3 * i], X[3 * i + 1], X[3 * i + 2], 0.0};
        dX[i] = d4{0.0, 0.0, 0.0, 0.0};
    }
    __syncthreads();
    if (threadIdx.x == 0) tail->bad = bad;
}

// One root, and every level one more than its parent's (no cycles).
__global__ __launch_bounds__(1024) void k_na_check(int n, const int32_t *par, const int32_t *lev, NaTail *tail) {
    __shared__ int roots, bad;
    if (threadIdx.x == 0) { roots = 0; bad = 0; }
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const int p = par[i];
        if (p < 0) {
            atomicAdd(&roots, 1);
            if (lev[i] != 0) bad = 1;
        } else if (lev[i] != lev[p] + 1) {
            bad = 1;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0 && (roots != 1 || bad)) tail->bad = 1;
}

__global__ void k_na_out(int n, const d4 *a0, const NaTail *tail, double *acc, double *U) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const bool bad = tail->bad != 0;
    if (i < n) {
        const d4 a = a0[i];
        acc[3 * i] = bad ? NAN : a.x;
        acc[3 * i + 1] = bad ? NAN : a.y;
        acc[3 * i + 2] = bad ? NAN : a.z;
    }
    if (i == 0) *U = bad ? NAN : tail->U;
}

}  // namespace

extern "C" int mstar_force_noalloc(void *hip_stream, const mstar_params *params, int64_t n, const double *m,
                                   const double *rho, const int32_t *parent, const double *X, double *acc,
                                   double *U) {
    if (!params || params->struct_size != sizeof(mstar_params) || !m || !rho || !parent || !X || !acc || !U)
        return MSTAR_E_INVAL;
    if (n < 2 || n > kNaMaxN) return MSTAR_E_INVAL;   // beyond the scratch array's capacity
    if (!(params->G > 0.0) || !std::isfinite(params->G) || params->n_d < 0) return MSTAR_E_INVAL;
    if (params->n_d > kMaxNd || params->beta != 0.0) return MSTAR_E_UNSUPPORTED;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return MSTAR_E_DEVICE;
    void *base = nullptr;
    int cap = 0;
    int rc = scratch_for(dev, &base, &cap);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)hip_stream;
    unsigned char *b = (unsigned char *)base;
    const int N = (int)n;
    // the workspace view of the scratch array (slot 0 is the only slot)
    Dev d{};
    d.n = N;
    d.nib = (N + 63) / 64;
    d.nfb = (N + 64 * kForceIPL - 1) / (64 * kForceIPL);
    d.kfmax = 1;
    d.nsplit_max = kNaParts;
    d.P = (d4 *)(b + kOffP);
    d.X0 = (d4 *)(b + kOffX0);
    d.dX = (d4 *)(b + kOffDX);
    d.a0 = (d4 *)(b + kOffA0);
    d.part = (d4 *)(b + kOffPart);
    d.Upart = (double *)(b + kOffUpart);
    int32_t *ints[10];
    for (int k = 0; k < 10; ++k) ints[k] = (int32_t *)(b + kOffInt + k * kIntN);
    d.parent = ints[0];
    d.level = ints[1];
    d.child_off = ints[2];
    d.child_idx = ints[3];
    d.rkA = ints[4];
    d.rkB = ints[5];
    d.nxtA = ints[6];
    d.nxtB = ints[7];
    d.cnt = ints[8];
    d.fill = ints[9];
    NaTail *tail = (NaTail *)(b + kOffCtl);
    d.ctl = &tail->ctl;
    // j-splits: enough workgroups to fill the chip, at most kNaSplits, at
    // least 16 j-bodies per wave
    const int hi = std::max(1, std::min(kNaSplits, N / (16 * kForceWaves)));
    const int ns = std::max(1, std::min(hi, (cap + d.nfb - 1) / std::max(1, d.nfb)));
    FLay f{};
    f.mut = 0;
    f.nparts = force_parts(ns, params->n_d);
    SlotList sl{};
    sl.nact = 1;
    sl.slot[0] = 0;
    k_na_prep<<<1, 1024, 0, s>>>(N, m, rho, parent, X, d.P, d.X0, d.dX, d.parent, tail);
    launch_levels_children(d, s);
    k_na_check<<<1, 1024, 0, s>>>(N, d.parent, d.level, tail);
    launch_force(d, s, sl, params->n_d, f, false);
    launch_reduce_start(d, s, 0, params->G, f, d.a0, &tail->U, false, false);
    k_na_out<<<(N + 255) / 256, 256, 0, s>>>(N, d.a0, tail, acc, U);
    return hipGetLastError() == hipSuccess ? MSTAR_OK : MSTAR_E_DEVICE;
}
