// Host side of the C ABI declared in include/mstar.h: context, device
// workspace, validation, and the sequencing of kernel launches that makes up
// the integrator (paper Sec. 2.3 GBS step, Sec. 2.4 driver, Sec. 3.5 MST
// rebuilds, Sec. 4.2 concurrent substep divisions).
//
// All substep divisions of a GBS step advance together: at substep s every
// division that still has a kick left is drifted, has its forces evaluated
// and is kicked in one launch per stage, so the number of dependent launches
// per GBS step is 3 * 2 k_fix + O(1) and the force launches carry up to
// k_fix independent O(N^2) evaluations.  The host reads back one small
// control block per GBS step to decide acceptance and the next step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstddef>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <type_traits>
#include <limits>
#include <vector>

#include "../../include/mstar.h"
#include "adjoint.h"
#include "batch.h"
#include "common.h"
#include "rebuild.h"

using namespace mstar;

// Default accepted steps between re-deriving the carried positions and
// velocities from the MST edges.
constexpr int kResyncEvery = 32;

struct mstar_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::string err;
    Dev d{};
    int cap_n = 0;
    std::vector<void *> allocs;
    double *xin = nullptr, *vin = nullptr, *xout = nullptr;   // staging [3n]
    CtlBlock *h_blk = nullptr;  // pinned host copy of the control block
    Ctl *h_ctl = nullptr;       // its two parts
    SysScal *h_sys = nullptr;
    int32_t *h_flags = nullptr; // [done, rounds]
    int mst_rounds_est = 0;     // Boruvka rounds of the previous build
    // profiling of the force kernel
    bool prof = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
    std::vector<int> ev_kind;          // force kernel of each event pair: 0 pairwise, 1 mutual
    std::vector<double> ev_pairs;      // directed pairs of each launch
    size_t ev_used = 0;
    hipEvent_t prof_ref = nullptr;     // recorded when profiling is enabled: the time origin
    int64_t prof_launches = 0;
    double prof_pairs = 0.0;
    double prof_batch_ms = 0.0;        // batched launches (timed with b_ev)
    // batched small systems (kernels_batch.hip)
    int num_cu = 0;
    int64_t b_cap_sys = 0, b_cap_n = 0;
    std::vector<void *> b_allocs;
    int64_t *b_off = nullptr;
    int32_t *b_order = nullptr, *b_queue = nullptr;
    double *b_m = nullptr, *b_x = nullptr, *b_v = nullptr, *b_x0 = nullptr, *b_v0 = nullptr;
    double *b_t0 = nullptr, *b_te = nullptr;
    BatchStat *b_stat = nullptr;
    BatchStat *h_bstat = nullptr;      // pinned [b_cap_sys]
    BatchArgs *b_args = nullptr;       // device copy of the kernel arguments
    BatchArgs *h_bargs = nullptr;      // pinned staging of the same
    mstar_batch_config bcfg[kBatchMaxKF + 1];
    hipGraphExec_t b_exec = nullptr;   // captured reset + batch kernel
    int b_key_kf = 0, b_key_wl = -1, b_key_nwg = 0;
    hipEvent_t b_ev[2] = {nullptr, nullptr};
    double *b_hrec = nullptr;          // [n_sys][cap] accepted steps of a recording batched call
    size_t b_hrec_cap = 0;
    // one GBS step attempt of mstar_integrate* captured as a graph
    hipGraphExec_t s_exec = nullptr;
    std::string s_key;                 // what the captured launches depend on
    // the rebuild and start-state force after an accepted step, captured likewise
    hipGraphExec_t r_exec = nullptr;
    std::string r_key;
    bool no_graph = false;             // the stream could not be captured: launch eagerly
    int ws_gen = 0;                    // bumped whenever device buffers move
    int mst_spare = 1;                 // Boruvka rounds queued beyond the previous build's count
    int force_cap[3] = {0, 0, 0};      // resident force workgroups per chip, by close-pair kernel kind
    int force_mode = 0;                // 0: mutual kernel where it applies, 1: pairwise only, 2: mutual for any N
    int mut_wps = 3;                   // waves per SIMD the mutual kernel's work is split for
    int mut_waves = 0;                 // resident mutual-kernel waves on the chip (occupancy x CUs)
    int mut_cap_n = 0;                 // N the mutual-kernel buffers are sized for (0: none)
    int div_chains = 1;                // chains of division lanes: 1, 2, or 0 (two at large N)
    int resync_every = kResyncEvery;   // accepted steps between re-deriving the Cartesian caches
    hipStream_t div_s2 = nullptr;      // stream of the second chain
    hipEvent_t div_ev[2] = {nullptr, nullptr};   // fork, join
    DcBuf dc{};                        // divide-and-conquer tree builder buffers
    int dc_cap_n = 0;                  // N they are sized for (0: none)
    bool ext_on = false;               // an external field applies to the running integration
    ExtField h_ext{};                  // host copy of that field
    // frozen-controller replay and adjoint (kernels_adjoint.hip)
    std::vector<void *> a_allocs;
    int a_n = 0, a_kf = 0;
    int64_t a_ncp = 0, a_seg = 0;
    AdjDev ad{};
    d4 *Yr = nullptr, *Yv = nullptr;      // current state
    double *Yt = nullptr;
    d4 *cpr = nullptr, *cpv = nullptr;    // checkpoints
    double *cpt = nullptr;
    d4 *sgr = nullptr, *sgv = nullptr;    // states of one checkpoint segment
    double *sgt = nullptr;
    d4 *brr = nullptr, *brv = nullptr;    // running state of the block recomputation
    double *brt = nullptr;
    // the reverse pass recomputes the next block of steps (keeping every
    // substep state) on a second stream while the current block is reversed
    hipStream_t a_s2 = nullptr;
    hipEvent_t a_ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};   // kept[2], reversed[2], checkpoints
    void *a_store = nullptr;              // two slots of kept substep states
    size_t a_store_cap = 0;               // bytes
    size_t a_store_max = size_t(4) << 30; // limit of both slots together (bytes)
    double *a_m = nullptr, *a_c = nullptr, *a_io[4] = {nullptr, nullptr, nullptr, nullptr};
    double *a_gm = nullptr;               // mass gradient [n]
};

namespace {

constexpr int kNsplitMax = 32;
// The mutual force kernel serves N in [kMutMinN, kMutMaxN] (its j-side
// partials grow as N^2); each of its waves takes at least kMutLmin steps.
constexpr int kMutMinN = 1024;
constexpr int kMutMaxN = 20000;
constexpr int kMutSoloN = 16384;
constexpr long long kMutLmin = 64;     // >= 64: a j-block is never cut into more than two pieces
constexpr int kMutMaxW = 128;          // i-side partials per row and launch (bounds the buffers)

int fail(mstar_ctx *c, int code, const char *fmt, ...) {
    if (c) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        c->err = buf;
    }
    return code;
}

#define HIPCK(x)                                                                          \
    do {                                                                                  \
        hipError_t e_ = (x);                                                              \
        if (e_ != hipSuccess) return fail(ctx, MSTAR_E_DEVICE, "%s: %s", #x, hipGetErrorString(e_)); \
    } while (0)

template <class T>
int dalloc(mstar_ctx *ctx, T **p, size_t count) {
    void *q = nullptr;
    if (hipMalloc(&q, sizeof(T) * (count ? count : 1)) != hipSuccess) {
        *p = nullptr;
        return fail(ctx, MSTAR_E_NOMEM, "device allocation of %zu bytes failed", sizeof(T) * count);
    }
    ctx->allocs.push_back(q);
    *p = (T *)q;
    return MSTAR_OK;
}

// Mutual force kernel geometry for n bodies and the step count L per wave
// (FLay; L is raised to at least Lmin).
FLay mut_geometry(int n, long long total_waves_hint, long long Lmin) {
    FLay f{};
    f.mut = 1;
    f.ipl = kMutIPL;
    f.nb = (n + 63) / 64;
    f.npr = (f.nb + kMutIPL - 1) / kMutIPL;
    f.Ec = mut_rs(f, f.npr);
    // no row (the first is the longest) may span more than kMutMaxW waves
    const long long row0 = mut_rs(f, 1);
    Lmin = std::max(Lmin, (row0 + kMutMaxW - 2) / (kMutMaxW - 1));
    f.L = std::max(Lmin, total_waves_hint > 1 ? (f.Ec + total_waves_hint - 1) / total_waves_hint : Lmin);
    f.maxw = (int)((row0 + f.L - 1) / f.L) + 1;
    return f;
}

void free_workspace(mstar_ctx *ctx) {
    for (void *p : ctx->allocs) (void)hipFree(p);
    ctx->allocs.clear();
    ctx->d = Dev{};
    ctx->cap_n = 0;
    ctx->mut_cap_n = 0;
    ctx->dc = DcBuf{};
    ctx->dc_cap_n = 0;
}

int ensure(mstar_ctx *ctx, int n) {
    if (n <= ctx->cap_n) {
        ctx->d.n = n;
        ctx->d.nib = (n + 63) / 64;
        ctx->d.nkwg = (n + kWG - 1) / kWG;
        ctx->d.nkwg4 = (n + kWG / 4 - 1) / (kWG / 4);
        ctx->d.nfb = (n + 64 * kForceIPL - 1) / (64 * kForceIPL);
        return MSTAR_OK;
    }
    HIPCK(hipStreamSynchronize(ctx->stream));
    free_workspace(ctx);
    ++ctx->ws_gen;
    const int cap = std::max(n, 64);
    const size_t N = (size_t)cap;
    const int nib = (cap + 63) / 64, nkwg = (cap + kWG - 1) / kWG;
    Dev &d = ctx->d;
    int rc = 0;
#define A(ptr, cnt) \
    if ((rc = dalloc(ctx, &(ptr), (cnt))) != MSTAR_OK) { free_workspace(ctx); return rc; }
    A(d.parent, N) A(d.level, N) A(d.parent_new, N) A(d.level_new, N) A(d.child_off, N + 1) A(d.child_idx, N)
    CtlBlock *cb = nullptr;
    int32_t *flags2 = nullptr;
    A(d.root, 1) A(d.X0, N) A(d.V0, N) A(d.a0, N) A(d.m, N) A(cb, 1) A(flags2, 2)
    d.ctl = &cb->ctl;
    d.sys = &cb->sys;
    d.done = flags2;
    d.rounds = flags2 + 1;
    A(d.P, kMaxDiv * N) A(d.Vt, kMaxDiv * N) A(d.dX, kMaxDiv * N) A(d.dV, kMaxDiv * N) A(d.dX1, N) A(d.dV1, N)
    A(d.dP, kMaxDiv * N) A(d.dVt, kMaxDiv * N) A(d.dP1, N) A(d.dVt1, N) A(d.akick, kMaxDiv * N)
    A(d.dscal, kMaxDiv) A(d.dscal1, 1) A(d.part, (size_t)kMaxDiv * kNsplitMax * N)
    A(d.Upart, (size_t)kMaxDiv * nib * kNsplitMax) A(d.Tpart, (size_t)kMaxDiv * (4 * nkwg)) A(d.epspart, (size_t)(nkwg + 1) * kMaxDiv)
    A(d.tsA, N) A(d.tsB, N) A(d.tsC, N) A(d.tsD, N) A(d.tsE, N) A(d.tsF, N) A(d.ancA, N) A(d.ancB, N)
    A(d.bor_w, (size_t)kNsplitMax * N) A(d.bor_j, (size_t)kNsplitMax * N) A(d.comp, N) A(d.ecomp_tmp, N)
    A(d.cw, N) A(d.cidx, N) A(d.tgt, N) A(d.ncomp, 1)
    A(d.deg, N) A(d.off, N + 1) A(d.fill, N) A(d.adj, 2 * N) A(d.arcpos, 2 * N) A(d.nxtA, 2 * N)
    A(d.nxtB, 2 * N) A(d.rkA, 2 * N) A(d.rkB, 2 * N) A(d.cnt, N + 1) A(d.scr, N) A(d.mo, N) A(d.dOm0, N)
    A(ctx->xin, 3 * N) A(ctx->vin, 3 * N) A(ctx->xout, 3 * N)
    ctx->mut_cap_n = 0;
    if (ctx->force_mode == 2 || (ctx->force_mode == 0 && cap >= kMutMinN)) {
        const int mcap = ctx->force_mode == 2 ? cap : std::min(cap, kMutMaxN);
        const FLay g = mut_geometry(mcap, 1, kMutLmin);
        d.mip_s = (size_t)g.npr * kMutMaxW * 64 * kMutIPL;   // every launch has maxw <= kMutMaxW
        d.mjp_s = (size_t)2 * g.npr * mcap;
        d.mup_s = (size_t)g.npr * kMutMaxW + g.nb;
        A(d.mip, kMaxDiv * d.mip_s) A(d.mjp, kMaxDiv * d.mjp_s) A(d.mcp, kMaxDiv * (size_t)mcap)
        A(d.mup, kMaxDiv * d.mup_s)
        ctx->mut_cap_n = mcap;
    }
#undef A
    HIPCK(hipMemsetAsync(d.dX, 0, sizeof(d4) * kMaxDiv * N, ctx->stream));
    HIPCK(hipMemsetAsync(d.dV, 0, sizeof(d4) * kMaxDiv * N, ctx->stream));
    HIPCK(hipMemsetAsync(d.ctl, 0, sizeof(Ctl), ctx->stream));
    HIPCK(hipMemsetAsync(d.sys, 0, sizeof(SysScal), ctx->stream));
    d.kfmax = kMaxDiv;
    d.nsplit_max = kNsplitMax;
    ctx->cap_n = cap;
    d.n = n;
    d.nib = (n + 63) / 64;
    d.nkwg = (n + kWG - 1) / kWG;
    d.nkwg4 = (n + kWG / 4 - 1) / (kWG / 4);
    d.nfb = (n + 64 * kForceIPL - 1) / (64 * kForceIPL);
    return MSTAR_OK;
}

// Buffers of the TTL function Omega, allocated on the first call with
// beta != 0 (they double the force-partial memory) at the current capacity.
int ensure_ttl(mstar_ctx *ctx) {
    Dev &d = ctx->d;
    if (d.opart) return MSTAR_OK;
    const size_t N = (size_t)ctx->cap_n;
    const size_t nib = (N + 63) / 64, nkwg4 = (N + kWG / 4 - 1) / (kWG / 4);
    int rc;
    if ((rc = dalloc(ctx, &d.opart, (size_t)kMaxDiv * kNsplitMax * N)) ||
        (rc = dalloc(ctx, &d.Opart, (size_t)kMaxDiv * nib * kNsplitMax)) ||
        (rc = dalloc(ctx, &d.wpart, (size_t)kMaxDiv * nkwg4))) {
        d.opart = nullptr; d.Opart = nullptr; d.wpart = nullptr;
        return rc;
    }
    ++ctx->ws_gen;
    return MSTAR_OK;
}

// Buffers of the external field, allocated on the first perturbed integration
// at the current capacity.
int ensure_ext(mstar_ctx *ctx) {
    Dev &d = ctx->d;
    if (d.fext) return MSTAR_OK;
    const size_t N = (size_t)ctx->cap_n;
    const size_t nkwg4 = (N + kWG / 4 - 1) / (kWG / 4);
    int rc;
    if ((rc = dalloc(ctx, &d.ext, 1)) || (rc = dalloc(ctx, &d.fext, (size_t)kMaxDiv * N)) ||
        (rc = dalloc(ctx, &d.fpart, (size_t)kMaxDiv * nkwg4)) || (rc = dalloc(ctx, &d.bpart, (size_t)kMaxDiv * nkwg4))) {
        d.ext = nullptr; d.fext = nullptr; d.fpart = nullptr; d.bpart = nullptr;
        return rc;
    }
    ++ctx->ws_gen;
    return MSTAR_OK;
}

// Validate an external field and stage it in ctx->h_ext (G folded into the
// point masses, softening squared).
int stage_ext(mstar_ctx *ctx, const mstar_params *p, const mstar_external *e) {
    if (e->struct_size != sizeof(mstar_external)) return fail(ctx, MSTAR_E_INVAL, "external: bad struct_size");
    if (e->n_point < 0 || e->n_point > MSTAR_MAX_EXT_POINTS)
        return fail(ctx, MSTAR_E_INVAL, "external: n_point must be in [0, %d]", MSTAR_MAX_EXT_POINTS);
    if (e->n_point > 0 && !e->point) return fail(ctx, MSTAR_E_INVAL, "external: point is NULL");
    if (p->beta != 0.0) return fail(ctx, MSTAR_E_UNSUPPORTED, "external: not supported with beta != 0");
    ExtField h{};
    for (int c = 0; c < 3; ++c) {
        if (!std::isfinite(e->g[c])) return fail(ctx, MSTAR_E_INVAL, "external: g must be finite");
        h.g[c] = e->g[c];
    }
    for (int k = 0; k < e->n_point; ++k) {
        const double *q = e->point + 5 * k;
        for (int c = 0; c < 5; ++c)
            if (!std::isfinite(q[c])) return fail(ctx, MSTAR_E_INVAL, "external: point %d is not finite", k);
        if (q[0] < 0.0 || q[4] < 0.0) return fail(ctx, MSTAR_E_INVAL, "external: point %d needs M, b >= 0", k);
        h.pt[k][0] = p->G * q[0];
        h.pt[k][1] = q[1]; h.pt[k][2] = q[2]; h.pt[k][3] = q[3];
        h.pt[k][4] = q[4] * q[4];
    }
    h.np = e->n_point;
    ctx->h_ext = h;
    return MSTAR_OK;
}

Ttl ttl_of(const mstar_params *p) { return Ttl{p->alpha, p->beta, p->gamma}; }
bool ttl_on(const mstar_params *p) { return p->beta != 0.0; }

constexpr int kBase = kBaseSlot;     // slot of the start state

// Resident force workgroups on the whole chip (queried once per N_d kind).
int force_cap(mstar_ctx *ctx, int nd) {
    const int k = nd <= 0 ? 0 : (nd <= 2 ? 1 : 2);
    if (ctx->force_cap[k] <= 0) ctx->force_cap[k] = force_blocks_per_cu(nd) * ctx->num_cu;
    return ctx->force_cap[k];
}

// Layout of one force launch over nact evaluations: the mutual kernel where
// it applies (no TTL function, N_d <= 2, buffers sized for this N), else the
// pairwise kernel with j-splits sized to fill the chip.
FLay plan_force(mstar_ctx *ctx, int nact, int nd, bool om, bool chain = false);

// Bodies from which MSTAR_DIV_CHAINS=0 runs the divisions as two chains.
constexpr int kChainMinN = 4096;

// Number of j-splits of one force launch over `nact` divisions.  The
// workgroups of a launch all take about the same time, so they run in rounds
// of `cap` (resident workgroups of the whole chip); the split count is the
// smallest whose last round is nearly full (within 1% of the best fill over
// all admissible counts), with at least 16 j-bodies per wave.
int nsplit_for(const Dev &d, int nact, int cap) {
    const int per = nact * d.nfb;
    const int hi = std::max(1, std::min(kNsplitMax - 1, d.n / (16 * kForceWaves)));
    double best = 0.0;
    std::vector<double> eff((size_t)hi + 1, 0.0);
    for (int ns = 1; ns <= hi; ++ns) {
        const long w = (long)per * ns;
        const long rounds = (w + cap - 1) / cap;
        eff[ns] = (double)w / (double)(rounds * cap);
        best = std::max(best, eff[ns]);
    }
    for (int ns = 1; ns <= hi; ++ns)
        if (eff[ns] >= best - 0.01) return ns;
    return hi;
}

FLay plan_force(mstar_ctx *ctx, int nact, int nd, bool om, bool chain) {
    const Dev &d = ctx->d;
    // the mutual kernel's waves split the launch's pairs evenly, one range per
    // wave; a single evaluation below kMutSoloN has too few steps to give every
    // SIMD its waves, and the pairwise kernel is faster there
    if (!om && nd <= 2 && ctx->force_mode != 1 && d.n <= ctx->mut_cap_n &&
        (ctx->force_mode == 2 || (d.n >= kMutMinN && (nact > 1 || d.n >= kMutSoloN)))) {
        FLay f = mut_geometry(d.n, 1, kMutLmin);   // L = the shortest allowed
        const long long total = (long long)nact * f.Ec;
        // one of two concurrent chains: one wave per SIMD, so that the two
        // chains' launches leave a slot for the other chain's kicks and drifts
        const long long waves = std::max(1, chain ? 4 * ctx->num_cu : ctx->mut_waves);
        f.L = std::max(f.L, (total + waves - 1) / waves);
        f.maxw = (int)((mut_rs(f, 1) + f.L - 1) / f.L) + 1;
        f.ncorr = nd > 0 ? 1 : 0;
        return f;
    }
    FLay f{};
    f.mut = 0;
    f.nparts = force_parts(nsplit_for(d, nact, force_cap(ctx, nd)), nd);
    return f;
}

int check_params(mstar_ctx *ctx, const mstar_params *p) {
    if (!p || p->struct_size != sizeof(mstar_params)) return fail(ctx, MSTAR_E_INVAL, "params: bad struct_size");
    if (!(p->G > 0.0) || !std::isfinite(p->G)) return fail(ctx, MSTAR_E_INVAL, "params: G must be > 0");
    if (!(p->eta > 0.0)) return fail(ctx, MSTAR_E_INVAL, "params: eta must be > 0");
    if (p->k_fix < 2 || p->k_fix > 16) return fail(ctx, MSTAR_E_INVAL, "params: k_fix must be in [2, 16]");
    if (p->n_d < 0) return fail(ctx, MSTAR_E_INVAL, "params: n_d must be >= 0");
    if (p->n_d > kMaxNd) return fail(ctx, MSTAR_E_UNSUPPORTED, "params: n_d > %d is not implemented on the GPU", kMaxNd);
    if (!std::isfinite(p->alpha) || !std::isfinite(p->beta) || !std::isfinite(p->gamma) || p->alpha < 0.0 ||
        p->beta < 0.0 || p->gamma < 0.0 || (p->alpha == 0.0 && p->beta == 0.0 && p->gamma == 0.0))
        return fail(ctx, MSTAR_E_INVAL, "params: need alpha, beta, gamma >= 0, not all zero");
    if (p->beta != 0.0 && !std::isfinite(p->omega_mass_max))
        return fail(ctx, MSTAR_E_INVAL, "params: omega_mass_max must be finite");
    if (!(p->a_gbs > 0.0) || !(p->f_min > 0.0) || !(p->f_max >= p->f_min) || !(p->q_first > 0.0) ||
        !(p->t_tol >= 0.0) || p->max_steps < 1 || p->max_halvings < 0 || p->max_time_iter < 0 ||
        p->rebuild_every < 0 || !(p->h_init >= 0.0) || p->accept_rule < 0 || p->accept_rule > 1)
        return fail(ctx, MSTAR_E_INVAL, "params: out of range");
    return MSTAR_OK;
}

bool is_dev(uint32_t flags) { return (flags & MSTAR_DEVICE_PTRS) != 0; }

// Bring an input array to the device: copy host memory into `stage`, or use a
// device pointer as is.
int in_dev(mstar_ctx *ctx, uint32_t flags, const void *src, void *stage, size_t bytes, const void **out) {
    if (is_dev(flags)) {
        *out = src;
        return MSTAR_OK;
    }
    HIPCK(hipMemcpyAsync(stage, src, bytes, hipMemcpyHostToDevice, ctx->stream));
    *out = stage;
    return MSTAR_OK;
}

int out_copy(mstar_ctx *ctx, uint32_t flags, void *dst, const void *devsrc, size_t bytes) {
    HIPCK(hipMemcpyAsync(dst, devsrc, bytes, is_dev(flags) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                         ctx->stream));
    return MSTAR_OK;
}

bool finite_host(const double *a, size_t k) {
    for (size_t i = 0; i < k; ++i)
        if (!std::isfinite(a[i])) return false;
    return true;
}

// Validate masses / positions / velocities (host copies) and copy masses.
// With TTL (p->beta != 0) also the Omega masses mo_i = m_i if m_i <=
// omega_mass_max else 0; a time transformation that rests on Omega alone
// needs at least two such bodies.
int load_bodies(mstar_ctx *ctx, uint32_t flags, int64_t n, const double *m, const double *x, const double *v,
                const mstar_params *p) {
    std::vector<double> hm((size_t)n), hx, hv;
    if (is_dev(flags)) {
        HIPCK(hipMemcpy(hm.data(), m, sizeof(double) * n, hipMemcpyDeviceToHost));
        if (x) { hx.resize(3 * (size_t)n); HIPCK(hipMemcpy(hx.data(), x, sizeof(double) * 3 * n, hipMemcpyDeviceToHost)); }
        if (v) { hv.resize(3 * (size_t)n); HIPCK(hipMemcpy(hv.data(), v, sizeof(double) * 3 * n, hipMemcpyDeviceToHost)); }
    } else {
        memcpy(hm.data(), m, sizeof(double) * n);
        if (x) hx.assign(x, x + 3 * n);
        if (v) hv.assign(v, v + 3 * n);
    }
    for (int64_t i = 0; i < n; ++i)
        if (!(hm[i] > 0.0) || !std::isfinite(hm[i])) return fail(ctx, MSTAR_E_INVAL, "mass %lld is not > 0", (long long)i);
    if ((x && !finite_host(hx.data(), hx.size())) || (v && !finite_host(hv.data(), hv.size())))
        return fail(ctx, MSTAR_E_NONFINITE, "non-finite position or velocity");
    HIPCK(hipMemcpyAsync(ctx->d.m, hm.data(), sizeof(double) * n, hipMemcpyHostToDevice, ctx->stream));
    if (p && ttl_on(p)) {
        std::vector<double> mo((size_t)n);
        int64_t light = 0;
        for (int64_t i = 0; i < n; ++i) {
            mo[i] = hm[i] <= p->omega_mass_max ? hm[i] : 0.0;
            light += mo[i] > 0.0;
        }
        if (light < 2 && p->alpha == 0.0 && p->gamma == 0.0)
            return fail(ctx, MSTAR_E_INVAL, "TTL with alpha = gamma = 0 needs two bodies with m <= omega_mass_max");
        int rc = ensure_ttl(ctx);
        if (rc) return rc;
        HIPCK(hipMemcpyAsync(ctx->d.mo, mo.data(), sizeof(double) * n, hipMemcpyHostToDevice, ctx->stream));
    }
    HIPCK(hipStreamSynchronize(ctx->stream));
    return MSTAR_OK;
}

// Check that parent[] is one rooted tree; copy it to the device.
int load_tree(mstar_ctx *ctx, uint32_t flags, int64_t n, const int32_t *parent) {
    std::vector<int32_t> hp((size_t)n);
    if (is_dev(flags)) HIPCK(hipMemcpy(hp.data(), parent, sizeof(int32_t) * n, hipMemcpyDeviceToHost));
    else memcpy(hp.data(), parent, sizeof(int32_t) * n);
    int roots = 0;
    std::vector<int8_t> state((size_t)n, 0);   // 0 unknown, 1 in progress, 2 reaches root
    for (int64_t v = 0; v < n; ++v) {
        if (hp[v] < 0) { ++roots; continue; }
        if (hp[v] >= n || hp[v] == v) return fail(ctx, MSTAR_E_INVAL, "parent[%lld] invalid", (long long)v);
    }
    if (roots != 1) return fail(ctx, MSTAR_E_INVAL, "parent[] must have exactly one root");
    for (int64_t v = 0; v < n; ++v) {
        std::vector<int32_t> path;
        int64_t u = v;
        while (u >= 0 && state[u] == 0) { state[u] = 1; path.push_back((int32_t)u); u = hp[u]; }
        if (u >= 0 && state[u] == 1) return fail(ctx, MSTAR_E_INVAL, "parent[] has a cycle");
        for (int32_t w : path) state[w] = 2;
    }
    HIPCK(hipMemcpyAsync(ctx->d.parent, hp.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, ctx->stream));
    HIPCK(hipStreamSynchronize(ctx->stream));
    return MSTAR_OK;
}

int prof_force(mstar_ctx *ctx, const SlotList &sl, int nd, const FLay &f, bool om, hipStream_t st = nullptr) {
    if (!st) st = ctx->stream;
    if (ctx->prof) {
        if (ctx->ev_used == ctx->ev.size()) {
            hipEvent_t a, b;
            HIPCK(hipEventCreate(&a));
            HIPCK(hipEventCreate(&b));
            ctx->ev.push_back({a, b});
        }
        const size_t k = ctx->ev_used++;
        auto &e = ctx->ev[k];
        HIPCK(hipEventRecord(e.first, st));
        launch_force(ctx->d, st, sl, nd, f, om);
        HIPCK(hipEventRecord(e.second, st));
        const double pairs = (double)sl.nact * (double)ctx->d.n * (double)(ctx->d.n - 1);
        if (ctx->ev_kind.size() < ctx->ev.size()) {
            ctx->ev_kind.resize(ctx->ev.size());
            ctx->ev_pairs.resize(ctx->ev.size());
        }
        ctx->ev_kind[k] = f.mut ? 1 : 0;
        ctx->ev_pairs[k] = pairs;
        ctx->prof_launches++;
        ctx->prof_pairs += pairs;
    } else {
        launch_force(ctx->d, st, sl, nd, f, om);
    }
    HIPCK(hipGetLastError());
    return MSTAR_OK;
}

// The start-state slot has no increments; its dX rows must read as zero for
// the close-pair correction (the slot region moves with n, so clear it).
int zero_base_increments(mstar_ctx *ctx) {
    const Dev &d = ctx->d;
    HIPCK(hipMemsetAsync(d.dX + (size_t)kBase * d.n, 0, sizeof(d4) * d.n, ctx->stream));
    return MSTAR_OK;
}

// Start-of-step quantities.  With `transform`: COM-frame positions and
// velocities of the start state from tree sums of the MST edges (Sec. 2.2
// deconstruction) and T.  With `with_force`: the force at the start state
// (a0, U0) for S'(s0) of eq. gbs-criterion and the end-time clip.
int prepare_start(mstar_ctx *ctx, const mstar_params *p, bool transform, bool with_force, int64_t *nforce) {
    const Dev &d = ctx->d;
    if (transform) {
        // the start slot's edge increments stay zero (only division slots
        // are drifted), so clearing them with each transform is enough
        int rc0 = zero_base_increments(ctx);
        if (rc0) return rc0;
        launch_tree_sums(d, ctx->stream, d.X0, d.V0, d.tsA, d.tsB);
        launch_com_frame(d, ctx->stream, kBase);
    }
    if (with_force) {
        SlotList sl{};
        sl.nact = 1;
        sl.slot[0] = kBase;
        const FLay f = plan_force(ctx, 1, p->n_d, ttl_on(p));
        int rc = prof_force(ctx, sl, p->n_d, f, ttl_on(p));
        if (rc) return rc;
        launch_reduce_start(d, ctx->stream, kBase, p->G, f, d.a0, &d.ctl->U0, ttl_on(p), ttl_on(p));
        if (ctx->ext_on) launch_ext(d, ctx->stream, sl, 1);
        if (nforce) ++*nforce;
    }
    HIPCK(hipGetLastError());
    return MSTAR_OK;
}

// All divisions nlist[k] (slot k) from the start state over the step in
// ctl->H: D(h/2)[K(h)D(h)]^(n-1)K(h)D(h/2) for every division.  Divisions
// are packed into lanes no longer than the longest division (first fit,
// longest first; for n_k = 2k this pairs n with 2 k_fix - n as in the load
// balancing of Sec. 4.2); a lane's next division starts when the previous one
// ends.  Every stage launches the drifts, then one force evaluation and the
// kicks of all divisions active in it: the step takes as many stages as the
// longest division has kicks, with the force evaluations spread evenly over
// them (k_fix = 8: 5 per launch for 8 stages, then 4), which keeps every
// launch large and its j-split partials few.
int run_divisions(mstar_ctx *ctx, const mstar_params *p, const int *nlist, int ndiv, int64_t *nforce) {
    const Dev &d = ctx->d;
    launch_div_init(d, ctx->stream, ndiv, kBase);
    int order[kMaxDiv];
    for (int k = 0; k < ndiv; ++k) order[k] = k;
    std::sort(order, order + ndiv, [&](int a, int b) { return nlist[a] > nlist[b] || (nlist[a] == nlist[b] && a < b); });
    const int cap = ndiv > 0 ? nlist[order[0]] : 0;
    int lane_len[kMaxDiv], nlanes = 0;
    int start[kMaxDiv];   // stage at which each division's first drift runs
    int lane_of[kMaxDiv];
    for (int q = 0; q < ndiv; ++q) {
        const int k = order[q];
        int l = 0;
        while (l < nlanes && lane_len[l] + nlist[k] > cap) ++l;
        if (l == nlanes) lane_len[nlanes++] = 0;
        start[k] = 1 + lane_len[l];
        lane_of[k] = l;
        lane_len[l] += nlist[k];
    }
    // with two chains, lanes go (longest first) to the chain with fewer force
    // evaluations; the chains share no slot, so their launches run on two
    // streams, each one's kicks and drifts beside the other's force launches
    // (measured faster where the mutual kernel runs at N >= kChainMinN, slower
    // below, where an attempt is bound by its launches)
    const bool two = ctx->div_chains == 2 ||
                     (ctx->div_chains == 0 && d.n >= kChainMinN && plan_force(ctx, 2, p->n_d, ttl_on(p), true).mut);
    const int nch = (two && nlanes > 1) ? 2 : 1;
    int chain_of_lane[kMaxDiv];
    long load[2] = {0, 0};
    for (int l = 0; l < nlanes; ++l) {
        const int c = (nch == 2 && load[1] < load[0]) ? 1 : 0;
        chain_of_lane[l] = c;
        load[c] += lane_len[l];
    }
    if (nch == 2) {
        HIPCK(hipEventRecord(ctx->div_ev[0], ctx->stream));
        HIPCK(hipStreamWaitEvent(ctx->div_s2, ctx->div_ev[0], 0));
    }
    const int last = cap;
    // the stages of chain c, launched on its stream
    auto run_chain = [&](int c) -> int {
        hipStream_t st = c ? ctx->div_s2 : ctx->stream;
        for (int t = 1; t <= last + 1; ++t) {
            SlotList dr{}, fk{};
            for (int k = 0; k < ndiv; ++k) {
                if (chain_of_lane[lane_of[k]] != c) continue;
                const int s = t - start[k] + 1;   // local stage of division k
                const int nk = nlist[k];
                if (s < 1 || s > nk + 1) continue;
                dr.slot[dr.nact] = k; dr.nsub[dr.nact] = nk;
                dr.half[dr.nact] = (s == 1 || s == nk + 1) ? 1 : 0;
                dr.first[dr.nact] = (s == 1) ? 1 : 0;
                dr.nact++;
                if (s <= nk) { fk.slot[fk.nact] = k; fk.nsub[fk.nact] = nk; fk.nact++; }
            }
            if (dr.nact) launch_drift(d, st, dr, ttl_of(p), ctx->ext_on);
            if (!fk.nact) continue;
            const FLay f = plan_force(ctx, fk.nact, p->n_d, ttl_on(p), nch == 2);
            int rc = prof_force(ctx, fk, p->n_d, f, ttl_on(p), st);
            if (rc) return rc;
            if (ctx->ext_on) launch_ext(d, st, fk, 0);
            launch_kick(d, st, fk, f, p->G, ttl_of(p), ctx->ext_on);
            if (nforce) *nforce += fk.nact;
        }
        return MSTAR_OK;
    };
    int rc = MSTAR_OK;
    for (int c = 0; c < nch && !rc; ++c) rc = run_chain(c);
    if (nch == 2) {   // join even after an error: a capture must not end with the fork open
        HIPCK(hipEventRecord(ctx->div_ev[1], ctx->div_s2));
        HIPCK(hipStreamWaitEvent(ctx->stream, ctx->div_ev[1], 0));
    }
    if (rc) return rc;
    HIPCK(hipGetLastError());
    return MSTAR_OK;
}

int read_ctl(mstar_ctx *ctx) {
    // one copy: Ctl and SysScal are adjacent in the device control block
    HIPCK(hipMemcpyAsync(ctx->h_blk, ctx->d.ctl, sizeof(CtlBlock), hipMemcpyDeviceToHost, ctx->stream));
    HIPCK(hipStreamSynchronize(ctx->stream));
    return MSTAR_OK;
}

// MST of the complete graph on `pos` (Sec. 3.1-3.4): as many Boruvka rounds
// as the previous build needed, a check of completion on the host, more
// rounds if needed, then rooting.
// j-splits of the Boruvka scan: 16 gives every SIMD enough waves to hide the
// j loads at N ~ 5e3 (8 left the scan latency-bound: 1.5% of the step)
int mst_splits(const Dev &d) { return std::max(1, std::min(16, d.n / 64)); }

// Upper bound on Boruvka rounds (each round at least halves the components).
int mst_max_rounds(const Dev &d) {
    int maxr = 2;
    for (int m = 1; m < d.n; m <<= 1) ++maxr;
    return maxr;
}

// Buffers of the divide-and-conquer builder, sized for the workspace's
// capacity on first use (freed with the workspace).
int ensure_dc(mstar_ctx *ctx) {
    if (ctx->dc_cap_n >= ctx->cap_n && ctx->dc_cap_n > 0) return MSTAR_OK;
    const size_t N = (size_t)ctx->cap_n;
    DcBuf b{};
    int rc = 0;
    if ((rc = dalloc(ctx, &b.key, 2 * N)) || (rc = dalloc(ctx, &b.idx, 2 * N)) || (rc = dalloc(ctx, &b.flag, N + 1)) ||
        (rc = dalloc(ctx, &b.cells, 2 * N)) || (rc = dalloc(ctx, &b.pstart, N + 1)) || (rc = dalloc(ctx, &b.part, N)) ||
        (rc = dalloc(ctx, &b.spos, N)) || (rc = dalloc(ctx, &b.bw, N)) || (rc = dalloc(ctx, &b.bu, N)) ||
        (rc = dalloc(ctx, &b.in, N)) || (rc = dalloc(ctx, &b.np, 1)))
        return rc;
    ctx->dc = b;
    ctx->dc_cap_n = ctx->cap_n;
    return MSTAR_OK;
}

// Groups of the divide-and-conquer builder hold at most ceil(sqrt(N)) bodies.
int dc_mcap(int n) { return (int)std::ceil(std::sqrt((double)n)); }

// The spanning tree on positions pos: the exact MST (Sec. 3.2) or, with dc,
// the divide-and-conquer tree of Sec. 3.3 (its parts are the components the
// Boruvka rounds start from).
int build_mst(mstar_ctx *ctx, const d4 *pos, int root_in, bool dc = false) {
    const Dev &d = ctx->d;
    const int maxr = mst_max_rounds(d);
    const int ns = mst_splits(d);
    if (dc) {
        int rc = ensure_dc(ctx);
        if (rc) return rc;
    }
    launch_mst_init(d, ctx->stream, pos, root_in);
    if (dc) launch_mst_dc(d, ctx->dc, ctx->stream, pos, dc_mcap(d.n));
    int est = ctx->mst_rounds_est > 0 ? std::min(ctx->mst_rounds_est, maxr) : maxr - 2;
    launch_mst_rounds(d, ctx->stream, pos, est, ns);
    for (int extra = 0;; ++extra) {
        HIPCK(hipMemcpyAsync(ctx->h_flags, d.done, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, ctx->stream));  // done, rounds
        HIPCK(hipStreamSynchronize(ctx->stream));
        if (ctx->h_flags[0]) break;
        if (est + extra >= 4 * maxr) return fail(ctx, MSTAR_E_DEVICE, "MST did not complete");
        launch_mst_rounds(d, ctx->stream, pos, 1, ns);
    }
    ctx->mst_rounds_est = ctx->h_flags[1];
    launch_mst_root(d, ctx->stream);
    HIPCK(hipGetLastError());
    return MSTAR_OK;
}

// New MST from the current state (Sec. 3.5), built on the COM-frame positions
// of the start state; far-pair edges of the new tree come from those
// positions and velocities.
int rebuild(mstar_ctx *ctx, const mstar_params *p) {
    const Dev &d = ctx->d;
    const d4 *pos = d.P + (size_t)kBase * d.n;
    const d4 *vel = d.Vt + (size_t)kBase * d.n;
    int rc = build_mst(ctx, pos, -1, (p->flags & MSTAR_MST_DC) != 0);
    if (rc) return rc;
    launch_rebuild_edges(d, ctx->stream, pos, vel, p->n_d);
    HIPCK(hipGetLastError());
    return MSTAR_OK;
}

// The same rebuild queued without waiting for the host: one Boruvka round
// more than the previous build needed, then rooting and the new edge vectors.
// If the rounds did not finish the tree, those kernels leave the old tree in
// place and flag it (ctl->tree_bad), the step that follows is not committed,
// and the driver rebuilds with rebuild() and repeats that step.
int rebuild_queued(mstar_ctx *ctx, const mstar_params *p) {
    const Dev &d = ctx->d;
    const d4 *pos = d.P + (size_t)kBase * d.n;
    const d4 *vel = d.Vt + (size_t)kBase * d.n;
    const int maxr = mst_max_rounds(d);
    const int est = ctx->mst_rounds_est > 0 ? std::min(ctx->mst_rounds_est + ctx->mst_spare, maxr) : maxr;
    launch_mst_init(d, ctx->stream, pos, -1);
    if (p->flags & MSTAR_MST_DC) {
        int rc = ensure_dc(ctx);
        if (rc) return rc;
        launch_mst_dc(d, ctx->dc, ctx->stream, pos, dc_mcap(d.n));
    }
    launch_mst_rounds(d, ctx->stream, pos, est, mst_splits(d));
    launch_mst_root(d, ctx->stream);
    launch_rebuild_edges(d, ctx->stream, pos, vel, p->n_d);
    HIPCK(hipGetLastError());
    return MSTAR_OK;
}

int load_state(mstar_ctx *ctx, const mstar_params *p, int64_t n, const int32_t *parent, const double *X,
               const double *V, const double *scal) {
    const uint32_t flags = p->flags;
    int rc = load_tree(ctx, flags, n, parent);
    if (rc) return rc;
    const void *xd, *vd;
    if ((rc = in_dev(ctx, flags, X, ctx->xin, sizeof(double) * 3 * n, &xd))) return rc;
    if ((rc = in_dev(ctx, flags, V, ctx->vin, sizeof(double) * 3 * n, &vd))) return rc;
    launch_pack3(ctx->stream, (const double *)xd, nullptr, ctx->d.X0, (int)n);
    launch_pack3(ctx->stream, (const double *)vd, nullptr, ctx->d.V0, (int)n);
    double hs[9];
    if (is_dev(flags)) HIPCK(hipMemcpy(hs, scal, sizeof hs, hipMemcpyDeviceToHost));
    else memcpy(hs, scal, sizeof hs);
    if (!finite_host(hs, 9)) return fail(ctx, MSTAR_E_NONFINITE, "non-finite scalars");
    if (hs[2] != 0.0 && !ttl_on(p)) return fail(ctx, MSTAR_E_INVAL, "scal: w != 0 needs beta != 0");
    launch_set_sys(ctx->d, ctx->stream, hs[0], hs[1], hs[2], hs + 3, hs + 6, 1);
    launch_levels_children(ctx->d, ctx->stream);
    HIPCK(hipGetLastError());
    return MSTAR_OK;
}

int store_state(mstar_ctx *ctx, uint32_t flags, int64_t n, double *X, double *V, double *scal) {
    launch_unpack3(ctx->stream, ctx->d.X0, ctx->xout, (int)n);
    int rc = out_copy(ctx, flags, X, ctx->xout, sizeof(double) * 3 * n);
    if (rc) return rc;
    launch_unpack3(ctx->stream, ctx->d.V0, ctx->vin, (int)n);
    if ((rc = out_copy(ctx, flags, V, ctx->vin, sizeof(double) * 3 * n))) return rc;
    if ((rc = read_ctl(ctx))) return rc;
    const SysScal &y = *ctx->h_sys;
    double hs[9] = {y.t, y.B, y.w, y.rcm[0], y.rcm[1], y.rcm[2], y.vcm[0], y.vcm[1], y.vcm[2]};
    if (is_dev(flags)) HIPCK(hipMemcpy(scal, hs, sizeof hs, hipMemcpyHostToDevice));
    else memcpy(scal, hs, sizeof hs);
    HIPCK(hipStreamSynchronize(ctx->stream));
    return MSTAR_OK;
}

// Neville-Aitken extrapolation, error test and step control of one attempt
// (Sec. 2.3, 4.2): judged at k_fix, or (accept_rule 1) at the first order
// whose error passes, whose extrapolation is then the result.
void enqueue_extrapolation(mstar_ctx *ctx, const mstar_params *p, bool ex) {
    const Dev &d = ctx->d;
    const int rule = p->accept_rule == 1 ? 1 : 0;
    launch_extrapolate(d, ctx->stream, p->k_fix, ttl_of(p), kBase, ex, rule);
    launch_control(d, ctx->stream, p->k_fix, p->eta, p->a_gbs, p->f_min, p->f_max, rule);
    if (rule == 1) launch_extrap_pick(d, ctx->stream, p->k_fix, ex);
}

}  // namespace

extern "C" {

int mstar_abi_version(void) { return MSTAR_ABI_VERSION; }

void mstar_params_default(mstar_params *p) {
    if (!p) return;
    memset(p, 0, sizeof *p);
    p->struct_size = sizeof(mstar_params);
    p->G = 1.0;
    p->eta = 1e-12;
    p->alpha = 1.0;
    p->beta = 0.0;
    p->gamma = 0.0;
    p->omega_mass_max = 0.0;
    p->a_gbs = 0.9;
    p->f_min = 0.1;
    p->f_max = 4.0;
    p->q_first = 0.1;
    p->t_tol = 1e-14;
    p->h_init = 0.0;
    p->max_steps = 1000000000LL;
    p->k_fix = 8;
    p->n_d = 2;
    p->max_halvings = 60;
    p->max_time_iter = 8;
    p->rebuild_every = 1;
    p->accept_rule = 0;
}

const char *mstar_strerror(int code) {
    switch (code) {
        case MSTAR_OK: return "ok";
        case MSTAR_E_INVAL: return "invalid argument";
        case MSTAR_E_NOMEM: return "out of memory";
        case MSTAR_E_DEVICE: return "HIP device error";
        case MSTAR_E_NONFINITE: return "non-finite input";
        case MSTAR_E_COINCIDENT: return "coincident bodies";
        case MSTAR_E_NOCONV: return "GBS step did not converge";
        case MSTAR_E_MAXSTEPS: return "maximum number of steps reached";
        case MSTAR_E_UNSUPPORTED: return "not supported by this implementation";
        case MSTAR_W_TIME_TOL: return "end time not met within tolerance";
        default: return "unknown code";
    }
}

int mstar_create(mstar_ctx **out, int hip_device, void *hip_stream) {
    if (!out) return MSTAR_E_INVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return MSTAR_E_DEVICE;
    if (hip_device < 0 || hip_device >= ndev) return MSTAR_E_INVAL;
    mstar_ctx *ctx = new (std::nothrow) mstar_ctx();
    if (!ctx) return MSTAR_E_NOMEM;
    ctx->device = hip_device;
    if (hipSetDevice(hip_device) != hipSuccess) { delete ctx; return MSTAR_E_DEVICE; }
    if (hip_stream) {
        ctx->stream = (hipStream_t)hip_stream;
    } else {
        if (hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking) != hipSuccess) { delete ctx; return MSTAR_E_DEVICE; }
        ctx->own_stream = true;
    }
    // spare Boruvka rounds of a queued rebuild (MSTAR_MST_SPARE_ROUNDS, 0..8;
    // 0 makes the repeat-the-step path of an unfinished rebuild frequent)
    if (const char *e = std::getenv("MSTAR_MST_SPARE_ROUNDS")) {
        const int v = std::atoi(e);
        if (v >= 0 && v <= 8) ctx->mst_spare = v;
    }
    // force kernel choice (MSTAR_FORCE_KERNEL = pairwise | mutual; default:
    // the mutual kernel for N in [kMutMinN, kMutMaxN]) and the waves per SIMD
    // its work is split for (MSTAR_MUT_WPS, 1..8)
    if (const char *e = std::getenv("MSTAR_FORCE_KERNEL")) {
        if (!strcmp(e, "pairwise")) ctx->force_mode = 1;
        else if (!strcmp(e, "mutual")) ctx->force_mode = 2;
    }
    if (const char *e = std::getenv("MSTAR_MUT_WPS")) {
        const int v = std::atoi(e);
        if (v >= 1 && v <= 8) ctx->mut_wps = v;
    }
    // accepted steps between re-deriving the carried Cartesian caches from
    // the MST edges (MSTAR_RESYNC_EVERY, 1..1000)
    if (const char *e = std::getenv("MSTAR_RESYNC_EVERY")) {
        const int v = std::atoi(e);
        if (v >= 1 && v <= 1000) ctx->resync_every = v;
    }
    // division lanes in one chain of launches or two concurrent ones
    // (MSTAR_DIV_CHAINS = 1, the default; 2; or 0: two where the mutual
    // kernel runs at N >= kChainMinN)
    if (const char *e = std::getenv("MSTAR_DIV_CHAINS")) {
        const int v = std::atoi(e);
        if (v == 0 || v == 1 || v == 2) ctx->div_chains = v;
    }
    if (hipStreamCreateWithFlags(&ctx->div_s2, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->div_ev[0], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->div_ev[1], hipEventDisableTiming) != hipSuccess) {
        mstar_destroy(ctx);
        return MSTAR_E_DEVICE;
    }
    if (hipHostMalloc((void **)&ctx->h_blk, sizeof(CtlBlock), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&ctx->h_flags, 2 * sizeof(int32_t), hipHostMallocDefault) != hipSuccess) {
        mstar_destroy(ctx);
        return MSTAR_E_NOMEM;
    }
    ctx->h_ctl = &ctx->h_blk->ctl;
    ctx->h_sys = &ctx->h_blk->sys;
    if (hipDeviceGetAttribute(&ctx->num_cu, hipDeviceAttributeMultiprocessorCount, hip_device) != hipSuccess ||
        ctx->num_cu <= 0 || hipEventCreate(&ctx->b_ev[0]) != hipSuccess ||
        hipEventCreate(&ctx->b_ev[1]) != hipSuccess) {
        mstar_destroy(ctx);
        return MSTAR_E_DEVICE;
    }
    // resident waves of the mutual kernel: mut_wps per SIMD (4 per CU), the same
    // number on every SIMD, within the kernel's occupancy
    ctx->mut_waves = std::max(1, std::min(force_mut_blocks_per_cu() / 4, ctx->mut_wps)) * 4 * ctx->num_cu;
    for (auto &c : ctx->bcfg) {
        memset(&c, 0, sizeof c);
        c.struct_size = sizeof(mstar_batch_config);
        c.wave_lanes = 16;
        c.wave_max_n = 16;
        c.wgs_per_cu = 0;
        c.use_graph = 1;
    }
    *out = ctx;
    return MSTAR_OK;
}

void mstar_destroy(mstar_ctx *ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    free_workspace(ctx);
    if (ctx->a_s2) (void)hipStreamSynchronize(ctx->a_s2);
    for (void *p : ctx->a_allocs) (void)hipFree(p);
    if (ctx->a_store) (void)hipFree(ctx->a_store);
    for (hipEvent_t e : ctx->a_ev)
        if (e) (void)hipEventDestroy(e);
    if (ctx->a_s2) (void)hipStreamDestroy(ctx->a_s2);
    if (ctx->div_s2) {
        (void)hipStreamSynchronize(ctx->div_s2);
        (void)hipStreamDestroy(ctx->div_s2);
    }
    for (hipEvent_t e : ctx->div_ev)
        if (e) (void)hipEventDestroy(e);
    for (void *p : ctx->b_allocs) (void)hipFree(p);
    if (ctx->h_bstat) (void)hipHostFree(ctx->h_bstat);
    if (ctx->b_hrec) (void)hipFree(ctx->b_hrec);
    if (ctx->h_bargs) (void)hipHostFree(ctx->h_bargs);
    if (ctx->b_exec) (void)hipGraphExecDestroy(ctx->b_exec);
    if (ctx->s_exec) (void)hipGraphExecDestroy(ctx->s_exec);
    if (ctx->r_exec) (void)hipGraphExecDestroy(ctx->r_exec);
    for (hipEvent_t e : ctx->b_ev)
        if (e) (void)hipEventDestroy(e);
    for (auto &e : ctx->ev) { (void)hipEventDestroy(e.first); (void)hipEventDestroy(e.second); }
    if (ctx->prof_ref) (void)hipEventDestroy(ctx->prof_ref);
    if (ctx->h_blk) (void)hipHostFree(ctx->h_blk);
    if (ctx->h_flags) (void)hipHostFree(ctx->h_flags);
    if (ctx->own_stream && ctx->stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
}

const char *mstar_last_error(const mstar_ctx *ctx) { return ctx ? ctx->err.c_str() : "no context"; }

int mstar_profile_enable(mstar_ctx *ctx, int enable) {
    if (!ctx) return MSTAR_E_INVAL;
    (void)hipSetDevice(ctx->device);
    HIPCK(hipStreamSynchronize(ctx->stream));
    if (ctx->div_s2) HIPCK(hipStreamSynchronize(ctx->div_s2));
    ctx->prof = enable != 0;
    ctx->ev_used = 0;
    ctx->prof_launches = 0;
    ctx->prof_pairs = 0.0;
    ctx->prof_batch_ms = 0.0;
    if (ctx->prof) {
        if (!ctx->prof_ref) HIPCK(hipEventCreate(&ctx->prof_ref));
        HIPCK(hipEventRecord(ctx->prof_ref, ctx->stream));
    }
    return MSTAR_OK;
}

// Time during which force launches of `kind` (-1: any) ran: the union of
// their intervals, placed on one time line by their offsets from the event
// recorded when profiling was enabled (the two division chains' launches
// overlap; launches on one stream do not, and then this is the sum of their
// durations).  Offsets are float milliseconds: about 1e-7 of the profiling
// window.
static int prof_busy(mstar_ctx *ctx, int kind, int64_t *nl, double *ms, double *pairs) {
    HIPCK(hipStreamSynchronize(ctx->stream));
    if (ctx->div_s2) HIPCK(hipStreamSynchronize(ctx->div_s2));
    std::vector<std::pair<double, double>> iv;
    double pr = 0.0;
    for (size_t k = 0; k < ctx->ev_used; ++k) {
        if (kind >= 0 && ctx->ev_kind[k] != kind) continue;
        float a = 0.f, dur = 0.f;
        HIPCK(hipEventElapsedTime(&a, ctx->prof_ref, ctx->ev[k].first));
        HIPCK(hipEventElapsedTime(&dur, ctx->ev[k].first, ctx->ev[k].second));
        iv.emplace_back((double)a, (double)a + (double)dur);
        pr += ctx->ev_pairs[k];
    }
    std::sort(iv.begin(), iv.end());
    double tot = 0.0, lo = 0.0, hi = -1.0;
    for (const auto &q : iv) {
        if (q.first > hi) {
            if (hi > lo) tot += hi - lo;
            lo = q.first;
            hi = q.second;
        } else {
            hi = std::max(hi, q.second);
        }
    }
    if (hi > lo) tot += hi - lo;
    if (nl) *nl = (int64_t)iv.size();
    if (ms) *ms = tot;
    if (pairs) *pairs = pr;
    return MSTAR_OK;
}

int mstar_profile_read(mstar_ctx *ctx, int64_t *launches, double *kernel_ms, double *pairs) {
    if (!ctx) return MSTAR_E_INVAL;
    (void)hipSetDevice(ctx->device);
    double ms = 0.0;
    int rc = prof_busy(ctx, -1, nullptr, &ms, nullptr);
    if (rc) return rc;
    if (launches) *launches = ctx->prof_launches;
    if (kernel_ms) *kernel_ms = ms + ctx->prof_batch_ms;
    if (pairs) *pairs = ctx->prof_pairs;
    return MSTAR_OK;
}

int mstar_profile_read_kernel(mstar_ctx *ctx, int32_t kind, int64_t *launches, double *kernel_ms, double *pairs) {
    if (!ctx || kind < 0 || kind > 1) return MSTAR_E_INVAL;
    (void)hipSetDevice(ctx->device);
    return prof_busy(ctx, kind, launches, kernel_ms, pairs);
}

int mstar_issue_rates(mstar_ctx *ctx, double *fma_cycles, double *rsq_cycles) {
    if (!ctx || !fma_cycles || !rsq_cycles) return fail(ctx, MSTAR_E_INVAL, "issue_rates: bad arguments");
    (void)hipSetDevice(ctx->device);
    double *buf = nullptr;
    HIPCK(hipMalloc((void **)&buf, issue_probe_bytes()));
    double cyc[2] = {0.0, 0.0};
    const hipError_t e = issue_probe(ctx->stream, buf, 4 * ctx->num_cu, 2.4, cyc);
    (void)hipFree(buf);
    if (e != hipSuccess) return fail(ctx, MSTAR_E_DEVICE, "issue_rates: %s", hipGetErrorString(e));
    *fma_cycles = cyc[0];
    *rsq_cycles = cyc[1];
    return MSTAR_OK;
}

int mstar_mst_build(mstar_ctx *ctx, uint32_t flags, int64_t n, const double *m, const double *x, int32_t root_in,
                    int32_t *parent, int32_t *level, int32_t *root_out) {
    if (!ctx) return MSTAR_E_INVAL;
    if (n < 2 || n > (1 << 24) || !m || !x || !parent || !level || !root_out)
        return fail(ctx, MSTAR_E_INVAL, "mst_build: bad arguments");
    (void)hipSetDevice(ctx->device);
    int rc = ensure(ctx, (int)n);
    if (rc) return rc;
    if ((rc = load_bodies(ctx, flags, n, m, x, nullptr, nullptr))) return rc;
    const void *xd;
    if ((rc = in_dev(ctx, flags, x, ctx->xin, sizeof(double) * 3 * n, &xd))) return rc;
    const Dev &d = ctx->d;
    launch_pack3(ctx->stream, (const double *)xd, nullptr, d.tsA, (int)n);
    if ((rc = build_mst(ctx, d.tsA, (root_in >= 0 && root_in < n) ? root_in : -1, (flags & MSTAR_MST_DC) != 0)))
        return rc;
    launch_tree_finish(d, ctx->stream);
    HIPCK(hipGetLastError());
    if ((rc = out_copy(ctx, flags, parent, d.parent, sizeof(int32_t) * n))) return rc;
    if ((rc = out_copy(ctx, flags, level, d.level, sizeof(int32_t) * n))) return rc;
    if ((rc = out_copy(ctx, flags, root_out, d.root, sizeof(int32_t)))) return rc;
    HIPCK(hipStreamSynchronize(ctx->stream));
    return MSTAR_OK;
}

int mstar_force(mstar_ctx *ctx, const mstar_params *params, int64_t n, const double *m, const double *rho,
                const int32_t *parent, const double *X, double *acc, double *U, double *Omega, double *dOmega) {
    if (!ctx) return MSTAR_E_INVAL;
    int rc = check_params(ctx, params);
    if (rc) return rc;
    if (n < 2 || n > (1 << 24) || !m || !rho || !parent || !X || !acc || !U)
        return fail(ctx, MSTAR_E_INVAL, "force: bad arguments");
    (void)hipSetDevice(ctx->device);
    const uint32_t flags = params->flags;
    if ((rc = ensure(ctx, (int)n))) return rc;
    if ((rc = load_bodies(ctx, flags, n, m, rho, nullptr, params))) return rc;
    if ((rc = load_tree(ctx, flags, n, parent))) return rc;
    const Dev &d = ctx->d;
    const void *rd, *xd;
    if ((rc = in_dev(ctx, flags, rho, ctx->xin, sizeof(double) * 3 * n, &rd))) return rc;
    if ((rc = in_dev(ctx, flags, X, ctx->vin, sizeof(double) * 3 * n, &xd))) return rc;
    launch_pack3(ctx->stream, (const double *)rd, d.m, d.P + (size_t)kBase * n, (int)n);
    launch_pack3(ctx->stream, (const double *)xd, nullptr, d.X0, (int)n);
    launch_levels_children(d, ctx->stream);
    if ((rc = zero_base_increments(ctx))) return rc;
    SlotList sl{};
    sl.nact = 1;
    sl.slot[0] = kBase;
    const bool om = ttl_on(params);
    const FLay f = plan_force(ctx, 1, params->n_d, om);
    if ((rc = prof_force(ctx, sl, params->n_d, f, om))) return rc;
    launch_reduce_start(d, ctx->stream, kBase, params->G, f, d.a0, &d.ctl->U0, om, false);
    launch_unpack3(ctx->stream, d.a0, ctx->xout, (int)n);
    HIPCK(hipGetLastError());
    if ((rc = out_copy(ctx, flags, acc, ctx->xout, sizeof(double) * 3 * n))) return rc;
    if ((rc = out_copy(ctx, flags, U, &d.ctl->U0, sizeof(double)))) return rc;
    if (Omega && (rc = out_copy(ctx, flags, Omega, &d.ctl->Om0, sizeof(double)))) return rc;
    if (dOmega) {
        HIPCK(hipStreamSynchronize(ctx->stream));   // xin is reused below
        if (om) launch_unpack3(ctx->stream, d.dOm0, ctx->xin, (int)n);
        else HIPCK(hipMemsetAsync(ctx->xin, 0, sizeof(double) * 3 * n, ctx->stream));
        if ((rc = out_copy(ctx, flags, dOmega, ctx->xin, sizeof(double) * 3 * n))) return rc;
    }
    HIPCK(hipStreamSynchronize(ctx->stream));
    return MSTAR_OK;
}

int mstar_leapfrog(mstar_ctx *ctx, const mstar_params *params, int64_t n, const double *m, const int32_t *parent,
                   double *X, double *V, double *scal, double H, int32_t nsub) {
    if (!ctx) return MSTAR_E_INVAL;
    int rc = check_params(ctx, params);
    if (rc) return rc;
    if (n < 2 || n > (1 << 24) || !m || !parent || !X || !V || !scal || nsub < 1 || nsub > 4096 ||
        !std::isfinite(H))
        return fail(ctx, MSTAR_E_INVAL, "leapfrog: bad arguments");
    (void)hipSetDevice(ctx->device);
    const uint32_t flags = params->flags;
    if ((rc = ensure(ctx, (int)n))) return rc;
    if ((rc = load_bodies(ctx, flags, n, m, nullptr, nullptr, params))) return rc;
    if ((rc = load_state(ctx, params, n, parent, X, V, scal))) return rc;
    if ((rc = prepare_start(ctx, params, true, false, nullptr))) return rc;
    launch_set_h(ctx->d, ctx->stream, H, 0.0, 0, ttl_of(params), 0);
    const int nl[1] = {nsub};
    if ((rc = run_divisions(ctx, params, nl, 1, nullptr))) return rc;
    launch_commit(ctx->d, ctx->stream, 0, 0);
    return store_state(ctx, flags, n, X, V, scal);
}

int mstar_gbs_step(mstar_ctx *ctx, const mstar_params *params, int64_t n, const double *m, const int32_t *parent,
                   double *X, double *V, double *scal, double H, int32_t *accepted, double *eps, double *h_next) {
    if (!ctx) return MSTAR_E_INVAL;
    int rc = check_params(ctx, params);
    if (rc) return rc;
    if (n < 2 || n > (1 << 24) || !m || !parent || !X || !V || !scal || !accepted || !eps || !h_next ||
        !std::isfinite(H) || H == 0.0)
        return fail(ctx, MSTAR_E_INVAL, "gbs_step: bad arguments");
    (void)hipSetDevice(ctx->device);
    const uint32_t flags = params->flags;
    if ((rc = ensure(ctx, (int)n))) return rc;
    if ((rc = load_bodies(ctx, flags, n, m, nullptr, nullptr, params))) return rc;
    if ((rc = load_state(ctx, params, n, parent, X, V, scal))) return rc;
    if ((rc = prepare_start(ctx, params, true, true, nullptr))) return rc;
    launch_set_h(ctx->d, ctx->stream, H, 0.0, 0, ttl_of(params), 0);
    int nl[16];
    for (int k = 0; k < params->k_fix; ++k) nl[k] = 2 * (k + 1);
    if ((rc = run_divisions(ctx, params, nl, params->k_fix, nullptr))) return rc;
    enqueue_extrapolation(ctx, params, false);
    launch_commit(ctx->d, ctx->stream, 1, 0);
    HIPCK(hipGetLastError());
    if ((rc = store_state(ctx, flags, n, X, V, scal))) return rc;
    *accepted = ctx->h_ctl->accepted;
    *eps = ctx->h_ctl->eps;
    *h_next = ctx->h_ctl->h_next;
    return MSTAR_OK;
}

}  // extern "C"

// One GBS step attempt after the start state is prepared: the step length
// (from ctl->h_next, clipped to t_end), all divisions, extrapolation, the
// accept decision and the commit.
int enqueue_attempt(mstar_ctx *ctx, const mstar_params *p, double t_end, const int *nl, int64_t *nforce) {
    const Dev &d = ctx->d;
    launch_set_h(d, ctx->stream, 0.0, t_end, 1, ttl_of(p), 1);
    int rc = run_divisions(ctx, p, nl, p->k_fix, nforce);
    if (rc) return rc;
    enqueue_extrapolation(ctx, p, ctx->ext_on);
    launch_commit(d, ctx->stream, 1, 0);
    HIPCK(hipGetLastError());
    return MSTAR_OK;
}

// The same attempt replayed from a captured graph (about 60 kernel launches
// become one), recaptured when anything its launches depend on changes: the
// parameters, t_end, N, the external-field switch or the device buffers.
// MSTAR_EAGER, or force-kernel profiling, launches it from the host instead.
// Capture `enqueue` once per key and replay it.  A stream that cannot be
// captured (the caller's stream is given to mstar_create) makes the context
// launch eagerly from then on: the graph is an optimisation only.
template <class F>
int replay_graph(mstar_ctx *ctx, hipGraphExec_t &exec, std::string &have, const std::string &key, F enqueue) {
    if (ctx->no_graph) return enqueue();
    if (!exec || key != have) {
        if (exec) (void)hipGraphExecDestroy(exec);
        exec = nullptr;
        have.clear();
        prepare_tree_launches();
        hipGraph_t graph = nullptr;
        if (hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
            (void)hipGetLastError();
            ctx->no_graph = true;
            return enqueue();
        }
        const int lrc = enqueue();
        const hipError_t ec = hipStreamEndCapture(ctx->stream, &graph);
        hipError_t ei = hipErrorUnknown;
        if (!lrc && ec == hipSuccess) ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (graph) (void)hipGraphDestroy(graph);
        if (lrc) return lrc;
        if (ei != hipSuccess) {   // nothing ran: launch the same work eagerly
            exec = nullptr;
            (void)hipGetLastError();
            ctx->no_graph = true;
            return enqueue();
        }
        have = key;
    }
    HIPCK(hipGraphLaunch(exec, ctx->stream));
    return MSTAR_OK;
}

int run_attempt(mstar_ctx *ctx, const mstar_params *p, double t_end, const int *nl, int64_t *nforce) {
    if ((p->flags & MSTAR_EAGER) || ctx->prof) return enqueue_attempt(ctx, p, t_end, nl, nforce);
    // everything the captured kernel arguments are made of
    const double kd[] = {p->G, p->eta, p->alpha, p->beta, p->gamma, p->a_gbs, p->f_min, p->f_max, t_end};
    const int ki[] = {p->k_fix, p->n_d, ctx->d.n, ctx->ws_gen, ctx->ext_on ? 1 : 0, p->accept_rule};
    std::string key((const char *)kd, sizeof kd);
    key.append((const char *)ki, sizeof ki);
    (void)force_cap(ctx, p->n_d);   // occupancy query outside any capture
    int rc = replay_graph(ctx, ctx->s_exec, ctx->s_key, key,
                          [&]() { return enqueue_attempt(ctx, p, t_end, nl, nullptr); });
    if (rc) return rc;
    if (nforce)
        for (int k = 0; k < p->k_fix; ++k) *nforce += nl[k];
    return MSTAR_OK;
}

// Start of a step after an accepted one: the queued MST rebuild (when due)
// and the start-state force.  Replayed from a graph when no re-derivation of
// the Cartesian caches is due (that one clears memory, which stays out of
// graphs), keyed like the attempt plus the queued round count.
int prepare_step(mstar_ctx *ctx, const mstar_params *p, bool rebuild_due, bool resync, int64_t *nforce) {
    if ((p->flags & MSTAR_EAGER) || ctx->prof || resync || !rebuild_due) {
        if (rebuild_due) {
            int rc = rebuild_queued(ctx, p);
            if (rc) return rc;
        }
        return prepare_start(ctx, p, resync, true, nforce);
    }
    const double kd[] = {p->G, p->alpha, p->beta, p->gamma};
    const int ki[] = {p->n_d, ctx->d.n, ctx->ws_gen, ctx->ext_on ? 1 : 0, ctx->mst_rounds_est, ctx->mst_spare,
                      (p->flags & MSTAR_MST_DC) ? 1 : 0};
    std::string key((const char *)kd, sizeof kd);
    key.append((const char *)ki, sizeof ki);
    (void)force_cap(ctx, p->n_d);
    if (p->flags & MSTAR_MST_DC) {   // allocate outside the capture
        int rc = ensure_dc(ctx);
        if (rc) return rc;
    }
    int rc = replay_graph(ctx, ctx->r_exec, ctx->r_key, key, [&]() {
        int r = rebuild_queued(ctx, p);
        return r ? r : prepare_start(ctx, p, false, true, nullptr);
    });
    if (rc) return rc;
    if (nforce) ++*nforce;
    return MSTAR_OK;
}

// Receiver of the accepted steps while the driver runs (the host side of an
// adjoint that replays the record as it grows); called outside any graph
// capture, after the step's control block has been read back.
struct StepFeed {
    virtual int accepted(double H) = 0;
    virtual ~StepFeed() = default;
};

// The driver (Sec. 2.4); with rec_H, the fictitious step of every accepted
// step is recorded and the run stops after max_acc accepted steps.
static int integrate_run(mstar_ctx *ctx, const mstar_params *params, int64_t n, const double *m, double *x,
                         double *v, double t0, double t_end, mstar_stats *stats, int64_t max_acc, double *rec_H,
                         int64_t *n_rec, const mstar_external *ext, StepFeed *feed);

// The external field applies for the duration of one integration only.
static int integrate_impl(mstar_ctx *ctx, const mstar_params *params, int64_t n, const double *m, double *x,
                          double *v, double t0, double t_end, mstar_stats *stats, int64_t max_acc, double *rec_H,
                          int64_t *n_rec, const mstar_external *ext = nullptr, StepFeed *feed = nullptr) {
    if (!ctx) return MSTAR_E_INVAL;
    const int rc = integrate_run(ctx, params, n, m, x, v, t0, t_end, stats, max_acc, rec_H, n_rec, ext, feed);
    ctx->ext_on = false;
    return rc;
}

static int integrate_run(mstar_ctx *ctx, const mstar_params *params, int64_t n, const double *m, double *x,
                         double *v, double t0, double t_end, mstar_stats *stats, int64_t max_acc, double *rec_H,
                         int64_t *n_rec, const mstar_external *ext, StepFeed *feed) {
    ctx->ext_on = false;
    if (n_rec) *n_rec = 0;
    int rc = check_params(ctx, params);
    if (rc) return rc;
    if (n < 2 || n > (1 << 24) || !m || !x || !v || !stats || stats->struct_size != sizeof(mstar_stats))
        return fail(ctx, MSTAR_E_INVAL, "integrate: bad arguments");
    if (!std::isfinite(t0) || !std::isfinite(t_end) || t0 == t_end)
        return fail(ctx, MSTAR_E_INVAL, "integrate: need finite t0 != t_end");
    mstar_stats st{};
    st.struct_size = sizeof(mstar_stats);
    st.t_reached = t0;
    (void)hipSetDevice(ctx->device);
    const uint32_t flags = params->flags;
    const mstar_params &p = *params;
    if (ext && (rc = stage_ext(ctx, params, ext))) return rc;
    if ((rc = ensure(ctx, (int)n))) return rc;
    if ((rc = load_bodies(ctx, flags, n, m, x, v, params))) return rc;
    if (ext) {
        if ((rc = ensure_ext(ctx))) return rc;
        HIPCK(hipMemcpyAsync(ctx->d.ext, &ctx->h_ext, sizeof(ExtField), hipMemcpyHostToDevice, ctx->stream));
        launch_ext_minv(ctx->d, ctx->stream);
        ctx->ext_on = true;
    }
    const Dev &d = ctx->d;
    const void *xd, *vd;
    if ((rc = in_dev(ctx, flags, x, ctx->xin, sizeof(double) * 3 * n, &xd))) return rc;
    if ((rc = in_dev(ctx, flags, v, ctx->vin, sizeof(double) * 3 * n, &vd))) return rc;
    // initial MST on the Cartesian positions, edge vectors, COM
    launch_pack3(ctx->stream, (const double *)xd, nullptr, d.tsA, (int)n);
    if ((rc = build_mst(ctx, d.tsA, -1, (flags & MSTAR_MST_DC) != 0))) return rc;
    launch_tree_finish(d, ctx->stream);
    launch_set_sys(d, ctx->stream, t0, 0.0, 0.0, nullptr, nullptr, 0);
    launch_state_from_cartesian(d, ctx->stream, (const double *)xd, (const double *)vd);
    launch_check_coincident(d, ctx->stream);
    if ((rc = prepare_start(ctx, &p, true, true, &st.force_evals))) return rc;
    launch_set_B(d, ctx->stream);
    if ((rc = read_ctl(ctx))) return rc;
    if (ctx->h_ctl->coincident) return fail(ctx, MSTAR_E_COINCIDENT, "two bodies share a position");
    const double gk0 = (p.alpha * ctx->h_ctl->U0 + p.beta * ctx->h_ctl->Om0) + p.gamma;
    double H = p.h_init > 0.0 ? p.h_init : p.q_first * gk0 * (t_end - t0);
    const double span = std::fabs(t_end - t0);
    int halvings = 0, since_rebuild = 0, since_resync = 0;
    bool fresh = false;   // the start state was just prepared
    bool just_rebuilt = false;
    bool h_on_dev = false;   // ctl->h_next already holds H
    bool last_resync = false;   // the current step's start re-derived the Cartesian caches
    int nl[16];
    for (int k = 0; k < p.k_fix; ++k) nl[k] = 2 * (k + 1);
    double t_now = t0;
    for (;;) {
        if (st.steps_accepted + st.steps_rejected >= p.max_steps) { rc = MSTAR_E_MAXSTEPS; break; }
        if (fresh) {
            const bool due = since_rebuild >= p.rebuild_every;
            if (due) {
                st.mst_rebuilds++;
                since_rebuild = 0;
                just_rebuilt = true;
            }
            const bool resync = since_resync >= ctx->resync_every;
            if (resync) since_resync = 0;
            last_resync = resync;
            if ((rc = prepare_step(ctx, &p, due, resync, &st.force_evals))) break;
            fresh = false;
        }
        if (!h_on_dev) launch_put_hnext(d, ctx->stream, H);
        if ((rc = run_attempt(ctx, &p, t_end, nl, &st.force_evals))) break;
        if ((rc = read_ctl(ctx))) break;
        h_on_dev = true;   // every branch below continues with H = ctl->h_next
        const Ctl &c = *ctx->h_ctl;
        if (just_rebuilt && c.tree_bad) {
            // the queued Boruvka rounds did not finish the new tree, so the
            // step ran on the old one and was not committed: rebuild with the
            // host check and repeat the step with the same H
            if ((rc = rebuild(ctx, &p))) break;
            if ((rc = prepare_start(ctx, &p, last_resync, true, &st.force_evals))) break;
            h_on_dev = false;   // control overwrote h_next; the repeat uses H
            continue;
        }
        if (just_rebuilt) {
            st.topo_changes += c.topo;
            just_rebuilt = false;
            ctx->mst_rounds_est = c.mst_rounds;
        }
        st.eps_last = c.eps;
        H = c.H;
        if (!c.accepted) {
            st.steps_rejected++;
            if (++halvings > p.max_halvings) { rc = MSTAR_E_NOCONV; break; }
            H = c.h_next;
            continue;
        }
        if (rec_H && *n_rec < max_acc) rec_H[(*n_rec)++] = H;
        if (feed && (rc = feed->accepted(H))) break;
        st.steps_accepted++;
        st.h_last = H;
        halvings = 0;
        since_rebuild++;
        since_resync++;
        fresh = true;
        if (c.clipped) st.time_iters++;
        H = c.h_next;
        st.h_next = H;
        t_now = ctx->h_sys->t;
        if (std::fabs(t_end - t_now) <= p.t_tol * span) { rc = MSTAR_OK; break; }
        if (st.time_iters > p.max_time_iter) { rc = MSTAR_W_TIME_TOL; break; }
        if (rec_H && st.steps_accepted >= max_acc) { rc = MSTAR_OK; break; }
    }
    st.t_reached = ctx->h_sys->t;
    if (rc == MSTAR_OK || rc == MSTAR_W_TIME_TOL || rc == MSTAR_E_NOCONV || rc == MSTAR_E_MAXSTEPS) {
        launch_tree_sums(d, ctx->stream, d.X0, d.V0, d.tsA, d.tsB);
        launch_output_cartesian(d, ctx->stream, ctx->xout, ctx->vin);
        int rc2;
        if ((rc2 = out_copy(ctx, flags, x, ctx->xout, sizeof(double) * 3 * n))) return rc2;
        if ((rc2 = out_copy(ctx, flags, v, ctx->vin, sizeof(double) * 3 * n))) return rc2;
        if (hipStreamSynchronize(ctx->stream) != hipSuccess) return fail(ctx, MSTAR_E_DEVICE, "sync failed");
    }
    *stats = st;
    if (rc < 0 && ctx->err.empty()) fail(ctx, rc, "%s", mstar_strerror(rc));
    return rc;
}

extern "C" {

int mstar_integrate(mstar_ctx *ctx, const mstar_params *params, int64_t n, const double *m, double *x, double *v,
                    double t0, double t_end, mstar_stats *stats) {
    return integrate_impl(ctx, params, n, m, x, v, t0, t_end, stats, -1, nullptr, nullptr);
}

int mstar_integrate_ext(mstar_ctx *ctx, const mstar_params *params, int64_t n, const double *m, double *x, double *v,
                        double t0, double t_end, const mstar_external *ext, mstar_stats *stats) {
    if (!ctx) return MSTAR_E_INVAL;
    if (!ext) return fail(ctx, MSTAR_E_INVAL, "integrate_ext: ext is NULL");
    return integrate_impl(ctx, params, n, m, x, v, t0, t_end, stats, -1, nullptr, nullptr, ext);
}

int mstar_integrate_record(mstar_ctx *ctx, const mstar_params *params, int64_t n, const double *m, double *x,
                           double *v, double t0, double t_end, int64_t max_accepted, double *H,
                           int64_t *n_accepted, mstar_stats *stats) {
    if (!ctx) return MSTAR_E_INVAL;
    if (max_accepted < 1 || !H || !n_accepted) return fail(ctx, MSTAR_E_INVAL, "integrate_record: bad arguments");
    return integrate_impl(ctx, params, n, m, x, v, t0, t_end, stats, max_accepted, H, n_accepted);
}

}  // extern "C"

// ------------------------------------------------------------------------
// Batched small systems: validation, device buffers, launch shape, graph.

static_assert(sizeof(BatchStat) == sizeof(mstar_batch_stats), "BatchStat must mirror mstar_batch_stats");
static_assert(offsetof(BatchStat, t_reached) == offsetof(mstar_batch_stats, t_reached), "layout");

namespace {

int ensure_batch(mstar_ctx *ctx, int64_t n_sys, int64_t n_tot) {
    if (n_sys <= ctx->b_cap_sys && n_tot <= ctx->b_cap_n) return MSTAR_OK;
    HIPCK(hipStreamSynchronize(ctx->stream));
    for (void *p : ctx->b_allocs) (void)hipFree(p);
    ctx->b_allocs.clear();
    if (ctx->h_bstat) (void)hipHostFree(ctx->h_bstat);
    ctx->h_bstat = nullptr;
    if (ctx->b_exec) (void)hipGraphExecDestroy(ctx->b_exec);
    ctx->b_exec = nullptr;
    ctx->b_key_wl = -1;
    ctx->b_cap_sys = ctx->b_cap_n = 0;
    const int64_t S = std::max<int64_t>(n_sys, 64), N = std::max<int64_t>(n_tot, 256);
    auto A = [&](auto **p, size_t bytes) -> int {
        void *q = nullptr;
        if (hipMalloc(&q, bytes) != hipSuccess) return fail(ctx, MSTAR_E_NOMEM, "device allocation of %zu bytes failed", bytes);
        ctx->b_allocs.push_back(q);
        *p = (std::remove_reference_t<decltype(*p)>)q;
        return MSTAR_OK;
    };
    int rc = 0;
    if ((rc = A(&ctx->b_off, sizeof(int64_t) * (S + 1))) || (rc = A(&ctx->b_order, sizeof(int32_t) * S)) ||
        (rc = A(&ctx->b_queue, sizeof(int32_t) * 2)) || (rc = A(&ctx->b_m, sizeof(double) * N)) ||
        (rc = A(&ctx->b_x, sizeof(double) * 3 * N)) || (rc = A(&ctx->b_v, sizeof(double) * 3 * N)) ||
        (rc = A(&ctx->b_x0, sizeof(double) * 3 * N)) || (rc = A(&ctx->b_v0, sizeof(double) * 3 * N)) ||
        (rc = A(&ctx->b_t0, sizeof(double) * S)) || (rc = A(&ctx->b_te, sizeof(double) * S)) ||
        (rc = A(&ctx->b_stat, sizeof(BatchStat) * S)) || (rc = A(&ctx->b_args, sizeof(BatchArgs))))
        return rc;
    if (!ctx->h_bargs && hipHostMalloc((void **)&ctx->h_bargs, sizeof(BatchArgs), hipHostMallocDefault) != hipSuccess) {
        ctx->h_bargs = nullptr;
        return fail(ctx, MSTAR_E_NOMEM, "pinned allocation failed");
    }
    if (hipHostMalloc((void **)&ctx->h_bstat, sizeof(BatchStat) * S, hipHostMallocDefault) != hipSuccess) {
        ctx->h_bstat = nullptr;
        return fail(ctx, MSTAR_E_NOMEM, "pinned allocation failed");
    }
    ctx->b_cap_sys = S;
    ctx->b_cap_n = N;
    return MSTAR_OK;
}

// Parameters, offsets and times of a batched call; *n_tot = offsets[n_sys].
// The parameter sets the batched kernel implements; others go through the
// single-system driver (mstar_integrate_batch) or are refused (autotune).
const char *batch_kernel_gap(const mstar_params *p) {
    if (ttl_on(p)) return "beta != 0 (TTL)";
    if (p->n_d > 2) return "n_d > 2";
    if (p->accept_rule != 0) return "accept_rule 1";
    if (p->k_fix > kBatchMaxKF) return "k_fix > 8";
    return nullptr;
}

int batch_validate(mstar_ctx *ctx, const mstar_params *p, int32_t n_sys, const int64_t *off, const double *t0,
                   const double *t_end, int64_t *n_tot, bool kernel_only) {
    int rc = check_params(ctx, p);
    if (rc) return rc;
    if (kernel_only)
        if (const char *g = batch_kernel_gap(p))
            return fail(ctx, MSTAR_E_UNSUPPORTED, "batch kernel: %s is not implemented", g);
    if (n_sys < 1 || !off || !t_end) return fail(ctx, MSTAR_E_INVAL, "batch: need n_sys >= 1, offsets and t_end");
    if (off[0] != 0) return fail(ctx, MSTAR_E_INVAL, "batch: offsets[0] must be 0");
    for (int32_t s = 0; s < n_sys; ++s) {
        const int64_t n = off[s + 1] - off[s];
        if (n < 2) return fail(ctx, MSTAR_E_INVAL, "batch: system %d has %lld < 2 bodies", s, (long long)n);
        if (n > (1 << 24)) return fail(ctx, MSTAR_E_INVAL, "batch: system %d has %lld bodies", s, (long long)n);
        const double a = t0 ? t0[s] : 0.0;
        if (!std::isfinite(a) || !std::isfinite(t_end[s]) || a == t_end[s])
            return fail(ctx, MSTAR_E_INVAL, "batch: system %d needs finite t0 != t_end", s);
    }
    *n_tot = off[n_sys];
    return MSTAR_OK;
}

int check_config(mstar_ctx *ctx, const mstar_batch_config *c) {
    if (!c || c->struct_size != sizeof(mstar_batch_config)) return fail(ctx, MSTAR_E_INVAL, "batch config: bad struct_size");
    if (c->wave_lanes != 0 && c->wave_lanes != 16 && c->wave_lanes != 32 && c->wave_lanes != 64)
        return fail(ctx, MSTAR_E_INVAL, "batch config: wave_lanes must be 0, 16, 32 or 64");
    if (c->wave_max_n < 0 || c->wave_max_n > c->wave_lanes)
        return fail(ctx, MSTAR_E_INVAL, "batch config: need 0 <= wave_max_n <= wave_lanes");
    if (c->wgs_per_cu < 0 || c->wgs_per_cu > 64) return fail(ctx, MSTAR_E_INVAL, "batch config: wgs_per_cu out of range");
    return MSTAR_OK;
}

// One batched launch on device arrays md, xd, vd (x, v overwritten); per-
// system results to ctx->h_bstat; kernel time (reset + persistent kernel).
int batch_run(mstar_ctx *ctx, const mstar_params *p, const mstar_batch_config &cfg, int32_t n_sys,
              const int64_t *off, const double *md, double *xd, double *vd, const double *t0, const double *t_end,
              double *kernel_ms, double *hrec = nullptr, int64_t hrec_cap = 0) {
    const int kf = p->k_fix;
    const int wl = cfg.wave_lanes;
    const int wmax = wl > 0 ? cfg.wave_max_n : 0;
    // two queues (whole-workgroup systems, single-wave systems), each by
    // decreasing cost estimate N^2 (ties by index)
    std::vector<int32_t> coop, wave;
    for (int32_t s = 0; s < n_sys; ++s) {
        const int64_t n = off[s + 1] - off[s];
        if (n > kBatchMaxN) continue;   // integrated by the single-system driver after the launch
        ((n > wmax) ? coop : wave).push_back(s);
    }
    auto by_cost = [&](int32_t a, int32_t b) {
        const int64_t na = off[a + 1] - off[a], nb = off[b + 1] - off[b];
        return na != nb ? na > nb : a < b;
    };
    std::sort(coop.begin(), coop.end(), by_cost);
    std::sort(wave.begin(), wave.end(), by_cost);
    std::vector<int32_t> order(coop);
    order.insert(order.end(), wave.begin(), wave.end());
    if (order.empty()) {   // every system is left to the single-system driver
        if (kernel_ms) *kernel_ms = 0.0;
        return MSTAR_OK;
    }
    std::vector<double> h0;
    if (t0) h0.assign(t0, t0 + n_sys);
    HIPCK(hipMemcpyAsync(ctx->b_off, off, sizeof(int64_t) * (n_sys + 1), hipMemcpyHostToDevice, ctx->stream));
    HIPCK(hipMemcpyAsync(ctx->b_order, order.data(), sizeof(int32_t) * order.size(), hipMemcpyHostToDevice,
                         ctx->stream));
    HIPCK(hipMemcpyAsync(ctx->b_te, t_end, sizeof(double) * n_sys, hipMemcpyHostToDevice, ctx->stream));
    if (t0) HIPCK(hipMemcpyAsync(ctx->b_t0, h0.data(), sizeof(double) * n_sys, hipMemcpyHostToDevice, ctx->stream));

    BatchArgs &a = *ctx->h_bargs;
    memset(&a, 0, sizeof a);
    a.n_coop = (int32_t)coop.size();
    a.n_wave = (int32_t)wave.size();
    a.order = ctx->b_order;
    a.queue = ctx->b_queue;
    a.off = ctx->b_off;
    a.m = md;
    a.x = xd;
    a.v = vd;
    a.t0 = t0 ? ctx->b_t0 : nullptr;
    a.t_end = ctx->b_te;
    a.stat = ctx->b_stat;
    a.hrec = hrec;
    a.hrec_cap = hrec ? hrec_cap : 0;
    a.p.G = p->G;
    a.p.eta = p->eta;
    a.p.alpha = p->alpha;
    a.p.gamma = p->gamma;
    a.p.a_gbs = p->a_gbs;
    a.p.f_min = p->f_min;
    a.p.f_max = p->f_max;
    a.p.q_first = p->q_first;
    a.p.t_tol = p->t_tol;
    a.p.h_init = p->h_init;
    a.p.max_steps = p->max_steps;
    a.p.k_fix = kf;
    a.p.n_d = p->n_d;
    a.p.max_halvings = p->max_halvings;
    a.p.max_time_iter = p->max_time_iter;
    a.p.rebuild_every = p->rebuild_every;

    const int fit = batch_blocks_per_cu(kf, wl);   // also sets the kernel's LDS limit
    if (fit < 1) return fail(ctx, MSTAR_E_DEVICE, "batch kernel (k_fix %d, wave_lanes %d) cannot be launched", kf, wl);
    const int per = cfg.wgs_per_cu > 0 ? std::min(cfg.wgs_per_cu, fit) : fit;
    const int64_t need = std::max<int64_t>(a.n_coop, (a.n_wave + 3) / 4);
    const int nwg = (int)std::max<int64_t>(1, std::min<int64_t>((int64_t)per * ctx->num_cu, need));

    HIPCK(hipMemcpyAsync(ctx->b_args, &a, sizeof a, hipMemcpyHostToDevice, ctx->stream));
    HIPCK(hipEventRecord(ctx->b_ev[0], ctx->stream));
    if (cfg.use_graph) {
        const bool same = ctx->b_exec && ctx->b_key_kf == kf && ctx->b_key_wl == wl && ctx->b_key_nwg == nwg;
        if (!same) {
            if (ctx->b_exec) (void)hipGraphExecDestroy(ctx->b_exec);
            ctx->b_exec = nullptr;
            ctx->b_key_wl = -1;
            hipGraph_t graph = nullptr;
            HIPCK(hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
            const int lrc = launch_batch(ctx->stream, ctx->b_args, ctx->b_queue, kf, wl, nwg);
            const hipError_t ec = hipStreamEndCapture(ctx->stream, &graph);
            if (lrc || ec != hipSuccess) {
                if (graph) (void)hipGraphDestroy(graph);
                return fail(ctx, MSTAR_E_DEVICE, "batch graph capture failed: %s", hipGetErrorString(ec));
            }
            const hipError_t ei = hipGraphInstantiate(&ctx->b_exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (ei != hipSuccess) {
                ctx->b_exec = nullptr;
                return fail(ctx, MSTAR_E_DEVICE, "batch graph instantiation failed: %s", hipGetErrorString(ei));
            }
            ctx->b_key_kf = kf;
            ctx->b_key_wl = wl;
            ctx->b_key_nwg = nwg;
        }
        HIPCK(hipGraphLaunch(ctx->b_exec, ctx->stream));
    } else {
        if (launch_batch(ctx->stream, ctx->b_args, ctx->b_queue, kf, wl, nwg))
            return fail(ctx, MSTAR_E_DEVICE, "batch launch failed");
    }
    HIPCK(hipGetLastError());
    HIPCK(hipEventRecord(ctx->b_ev[1], ctx->stream));
    HIPCK(hipMemcpyAsync(ctx->h_bstat, ctx->b_stat, sizeof(BatchStat) * n_sys, hipMemcpyDeviceToHost, ctx->stream));
    HIPCK(hipStreamSynchronize(ctx->stream));
    float ms = 0.f;
    HIPCK(hipEventElapsedTime(&ms, ctx->b_ev[0], ctx->b_ev[1]));
    if (kernel_ms) *kernel_ms = ms;
    return MSTAR_OK;
}

}  // namespace

extern "C" {

static int integrate_batch_impl(mstar_ctx *ctx, const mstar_params *params, int32_t n_sys, const int64_t *offsets,
                                const double *m, double *x, double *v, const double *t0, const double *t_end,
                                mstar_batch_stats *stats, int64_t rec_cap, double *H) {
    if (!ctx) return MSTAR_E_INVAL;
    ctx->err.clear();
    int64_t n_tot = 0;
    int rc = batch_validate(ctx, params, n_sys, offsets, t0, t_end, &n_tot, false);
    if (rc) return rc;
    if (!m || !x || !v || !stats) return fail(ctx, MSTAR_E_INVAL, "batch: null array");
    if (H && (rec_cap < 1 || rec_cap > ((int64_t)1 << 40) / n_sys))
        return fail(ctx, MSTAR_E_INVAL, "batch_record: bad record capacity");
    (void)hipSetDevice(ctx->device);
    // parameters the batched kernel does not implement: every system takes
    // the single-system driver below
    const bool in_kernel = batch_kernel_gap(params) == nullptr;
    double ms = 0.0;
    if (in_kernel) {
        if ((rc = ensure_batch(ctx, n_sys, n_tot))) return rc;
        double *hrec = nullptr;
        if (H) {   // device record of the accepted steps, kept in the context
            const size_t need = (size_t)n_sys * (size_t)rec_cap;
            if (need > ctx->b_hrec_cap) {
                if (ctx->b_hrec) (void)hipFree(ctx->b_hrec);
                ctx->b_hrec = nullptr;
                ctx->b_hrec_cap = 0;
                if (hipMalloc((void **)&ctx->b_hrec, sizeof(double) * need) != hipSuccess) {
                    ctx->b_hrec = nullptr;
                    return fail(ctx, MSTAR_E_NOMEM, "batch_record: device allocation failed");
                }
                ctx->b_hrec_cap = need;
            }
            hrec = ctx->b_hrec;
        }
        const uint32_t flags = params->flags;
        const double *md = m;
        double *xd = x, *vd = v;
        if (!is_dev(flags)) {
            HIPCK(hipMemcpyAsync(ctx->b_m, m, sizeof(double) * n_tot, hipMemcpyHostToDevice, ctx->stream));
            HIPCK(hipMemcpyAsync(ctx->b_x, x, sizeof(double) * 3 * n_tot, hipMemcpyHostToDevice, ctx->stream));
            HIPCK(hipMemcpyAsync(ctx->b_v, v, sizeof(double) * 3 * n_tot, hipMemcpyHostToDevice, ctx->stream));
            md = ctx->b_m;
            xd = ctx->b_x;
            vd = ctx->b_v;
        }
        if ((rc = batch_run(ctx, params, ctx->bcfg[params->k_fix], n_sys, offsets, md, xd, vd, t0, t_end, &ms, hrec,
                            rec_cap)))
            return rc;
        if (!is_dev(flags)) {
            HIPCK(hipMemcpyAsync(x, ctx->b_x, sizeof(double) * 3 * n_tot, hipMemcpyDeviceToHost, ctx->stream));
            HIPCK(hipMemcpyAsync(v, ctx->b_v, sizeof(double) * 3 * n_tot, hipMemcpyDeviceToHost, ctx->stream));
            HIPCK(hipStreamSynchronize(ctx->stream));
        }
        if (H) {
            HIPCK(hipMemcpyAsync(H, hrec, sizeof(double) * (size_t)n_sys * (size_t)rec_cap, hipMemcpyDeviceToHost,
                                 ctx->stream));
            HIPCK(hipStreamSynchronize(ctx->stream));
        }
        memcpy(stats, ctx->h_bstat, sizeof(BatchStat) * n_sys);
    }
    // systems beyond the kernel's kBatchMaxN bodies, or all of them when the
    // kernel does not implement the parameters: mstar_integrate's driver, one
    // after the other, in place, each with its own status
    struct RowFeed final : StepFeed {
        double *row = nullptr;
        int64_t cap = 0, k = 0;
        int accepted(double h) override {
            if (row && k < cap) row[k] = h;
            ++k;
            return MSTAR_OK;
        }
    };
    for (int32_t s = 0; s < n_sys; ++s) {
        const int64_t o = offsets[s], n = offsets[s + 1] - o;
        if (in_kernel && n <= kBatchMaxN) continue;
        mstar_stats st{};
        st.struct_size = sizeof(mstar_stats);
        RowFeed feed;
        if (H) {
            feed.row = H + (size_t)s * (size_t)rec_cap;
            feed.cap = rec_cap;
        }
        const int r = integrate_impl(ctx, params, n, m + o, x + 3 * o, v + 3 * o, t0 ? t0[s] : 0.0, t_end[s], &st, -1,
                                     nullptr, nullptr, nullptr, H ? &feed : nullptr);
        mstar_batch_stats &b = stats[s];
        b.status = r;
        b.reserved = 0;
        b.steps_accepted = st.steps_accepted;
        b.steps_rejected = st.steps_rejected;
        b.force_evals = st.force_evals;
        b.mst_rebuilds = st.mst_rebuilds;
        b.topo_changes = st.topo_changes;
        b.time_iters = st.time_iters;
        b.t_reached = st.t_reached;
        b.eps_last = st.eps_last;
        b.h_next = st.h_next;
        b.h_last = st.h_last;
    }
    if (H) {   // the slots past a system's recorded steps were never written: NaN, not stale memory
        for (int32_t s = 0; s < n_sys; ++s)
            for (int64_t k = std::max<int64_t>(0, std::min<int64_t>(stats[s].steps_accepted, rec_cap)); k < rec_cap; ++k)
                H[(size_t)s * (size_t)rec_cap + (size_t)k] = std::numeric_limits<double>::quiet_NaN();
    }
    if (ctx->prof && in_kernel) {   // the batched launch only
        double pairs = 0.0;
        for (int32_t s = 0; s < n_sys; ++s) {
            const double n = (double)(offsets[s + 1] - offsets[s]);
            if (n <= kBatchMaxN) pairs += (double)stats[s].force_evals * n * (n - 1.0);
        }
        ctx->prof_launches += 1;
        ctx->prof_pairs += pairs;
        ctx->prof_batch_ms += ms;
    }
    return MSTAR_OK;
}

int mstar_integrate_batch(mstar_ctx *ctx, const mstar_params *params, int32_t n_sys, const int64_t *offsets,
                          const double *m, double *x, double *v, const double *t0, const double *t_end,
                          mstar_batch_stats *stats) {
    return integrate_batch_impl(ctx, params, n_sys, offsets, m, x, v, t0, t_end, stats, 0, nullptr);
}

int mstar_integrate_batch_record(mstar_ctx *ctx, const mstar_params *params, int32_t n_sys, const int64_t *offsets,
                                 const double *m, double *x, double *v, const double *t0, const double *t_end,
                                 mstar_batch_stats *stats, int64_t rec_cap, double *H) {
    if (!H) return fail(ctx, MSTAR_E_INVAL, "batch_record: H is NULL");
    return integrate_batch_impl(ctx, params, n_sys, offsets, m, x, v, t0, t_end, stats, rec_cap, H);
}

int mstar_batch_get_config(mstar_ctx *ctx, int32_t k_fix, mstar_batch_config *cfg) {
    if (!ctx) return MSTAR_E_INVAL;
    if (!cfg || k_fix < 2 || k_fix > kBatchMaxKF) return fail(ctx, MSTAR_E_INVAL, "batch config: bad arguments");
    *cfg = ctx->bcfg[k_fix];
    return MSTAR_OK;
}

int mstar_batch_set_config(mstar_ctx *ctx, int32_t k_fix, const mstar_batch_config *cfg) {
    if (!ctx) return MSTAR_E_INVAL;
    if (k_fix < 2 || k_fix > kBatchMaxKF) return fail(ctx, MSTAR_E_INVAL, "batch config: k_fix out of range");
    int rc = check_config(ctx, cfg);
    if (rc) return rc;
    ctx->bcfg[k_fix] = *cfg;
    return MSTAR_OK;
}

int mstar_batch_autotune(mstar_ctx *ctx, const mstar_params *params, int32_t n_sys, const int64_t *offsets,
                         const double *m, const double *x, const double *v, const double *t0,
                         const double *t_end, mstar_batch_config *best) {
    if (!ctx) return MSTAR_E_INVAL;
    ctx->err.clear();
    int64_t n_tot = 0;
    int rc = batch_validate(ctx, params, n_sys, offsets, t0, t_end, &n_tot, true);
    if (rc) return rc;
    if (!m || !x || !v || !best) return fail(ctx, MSTAR_E_INVAL, "autotune: null argument");
    bool any = false;
    for (int32_t s = 0; s < n_sys && !any; ++s) any = offsets[s + 1] - offsets[s] <= kBatchMaxN;
    if (!any) return fail(ctx, MSTAR_E_INVAL, "autotune: no system of at most %d bodies to time", kBatchMaxN);
    (void)hipSetDevice(ctx->device);
    if ((rc = ensure_batch(ctx, n_sys, n_tot))) return rc;
    const hipMemcpyKind k = is_dev(params->flags) ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    HIPCK(hipMemcpyAsync(ctx->b_m, m, sizeof(double) * n_tot, k, ctx->stream));
    HIPCK(hipMemcpyAsync(ctx->b_x0, x, sizeof(double) * 3 * n_tot, k, ctx->stream));
    HIPCK(hipMemcpyAsync(ctx->b_v0, v, sizeof(double) * 3 * n_tot, k, ctx->stream));
    const int kf = params->k_fix;
    // candidate shapes: tile width for single-wave systems, the N cut between
    // the two tile kinds, and persistent workgroups per CU
    const int shapes[][2] = {{0, 0}, {16, 16}, {32, 16}, {32, 32}, {64, 32}, {64, 64}};
    mstar_batch_config top{};
    double top_ms = 0.0;
    bool have = false;
    for (const auto &sh : shapes) {
        const int fit = batch_blocks_per_cu(kf, sh[0]);
        for (int per = 1; per <= fit; ++per) {
            mstar_batch_config c{};
            c.struct_size = sizeof c;
            c.wave_lanes = sh[0];
            c.wave_max_n = sh[1];
            c.wgs_per_cu = per;
            c.use_graph = 0;
            HIPCK(hipMemcpyAsync(ctx->b_x, ctx->b_x0, sizeof(double) * 3 * n_tot, hipMemcpyDeviceToDevice, ctx->stream));
            HIPCK(hipMemcpyAsync(ctx->b_v, ctx->b_v0, sizeof(double) * 3 * n_tot, hipMemcpyDeviceToDevice, ctx->stream));
            double ms = 0.0;
            if ((rc = batch_run(ctx, params, c, n_sys, offsets, ctx->b_m, ctx->b_x, ctx->b_v, t0, t_end, &ms)))
                return rc;
            if (!have || ms < top_ms) {
                top = c;
                top_ms = ms;
                have = true;
            }
        }
    }
    if (!have) return fail(ctx, MSTAR_E_DEVICE, "autotune: no launchable shape");
    top.use_graph = 1;
    top.kernel_ms = top_ms;
    ctx->bcfg[kf] = top;
    *best = top;
    return MSTAR_OK;
}

}  // extern "C"

// ------------------------------------------------------------------------
// Frozen-controller replay and its adjoint.

namespace {

// Threads per body of the division kernels: up to 4, and one more for as many
// bodies as fit in 1024 threads.
void adj_threads(AdjDev &d, int n) {
    d.tpb = std::max(1, std::min(4, kAdjMaxN / n));
    d.ext = d.tpb < 4 ? std::min(n, kAdjMaxN - d.tpb * n) : 0;
}

int ensure_adj(mstar_ctx *ctx, int n, int kf, int64_t ncp, int64_t seg) {
    if (n <= ctx->a_n && kf <= ctx->a_kf && ncp <= ctx->a_ncp && seg <= ctx->a_seg) {
        ctx->ad.n = n;
        ctx->ad.kf = kf;
        adj_threads(ctx->ad, n);
        return MSTAR_OK;
    }
    HIPCK(hipStreamSynchronize(ctx->stream));
    if (ctx->a_s2) HIPCK(hipStreamSynchronize(ctx->a_s2));
    const size_t N = (size_t)std::max(n, ctx->a_n), K = (size_t)std::max(std::max(kf, 2), ctx->a_kf);
    const size_t CP = (size_t)std::max<int64_t>(std::max<int64_t>(ncp, 1), ctx->a_ncp);
    const size_t SG = (size_t)std::max<int64_t>(std::max<int64_t>(seg, 1), ctx->a_seg);
    for (void *p : ctx->a_allocs) (void)hipFree(p);
    ctx->a_allocs.clear();
    ctx->a_n = ctx->a_kf = 0;
    ctx->a_ncp = ctx->a_seg = 0;
    AdjDev &d = ctx->ad;
    auto A = [&](auto **p, size_t count) -> int {
        void *q = nullptr;
        const size_t bytes = sizeof(**p) * std::max<size_t>(count, 1);
        if (hipMalloc(&q, bytes) != hipSuccess) return fail(ctx, MSTAR_E_NOMEM, "device allocation of %zu bytes failed", bytes);
        ctx->a_allocs.push_back(q);
        *p = (std::remove_reference_t<decltype(*p)>)q;
        return MSTAR_OK;
    };
    double *m_ = nullptr, *c_ = nullptr;
    int rc = 0;
    if ((rc = A(&m_, N)) || (rc = A(&c_, K)) || (rc = A(&d.B, 1)) || (rc = A(&d.Er, K * N)) || (rc = A(&d.Ev, K * N)) ||
        (rc = A(&d.Et, K)) || (rc = A(&d.Lr, N)) || (rc = A(&d.Lv, N)) || (rc = A(&d.Lt, 1)) || (rc = A(&d.LB, 1)) ||
        (rc = A(&d.Sr, K * N)) || (rc = A(&d.Sv, K * N)) || (rc = A(&d.St, K)) || (rc = A(&d.SB, K)) ||
        (rc = A(&d.Sm, K * N)) || (rc = A(&d.Lm, N)) || (rc = A(&ctx->a_gm, N)) ||
        (rc = A(&ctx->brr, N)) || (rc = A(&ctx->brv, N)) || (rc = A(&ctx->brt, 1)) || (rc = A(&ctx->Yr, N)) || (rc = A(&ctx->Yv, N)) || (rc = A(&ctx->Yt, 1)) || (rc = A(&ctx->cpr, CP * N)) ||
        (rc = A(&ctx->cpv, CP * N)) || (rc = A(&ctx->cpt, CP)) || (rc = A(&ctx->sgr, SG * N)) ||
        (rc = A(&ctx->sgv, SG * N)) || (rc = A(&ctx->sgt, SG)))
        return rc;
    for (auto &io : ctx->a_io)
        if ((rc = A(&io, 3 * N))) return rc;
    ctx->a_m = m_;
    ctx->a_c = c_;
    d.m = m_;
    d.c = c_;
    ctx->a_n = (int)N;
    ctx->a_kf = (int)K;
    ctx->a_ncp = (int64_t)CP;
    ctx->a_seg = (int64_t)SG;
    d.n = n;
    d.kf = kf;
    adj_threads(d, n);
    return MSTAR_OK;
}

// Common set-up of a replay: parameters, sizes, steps; masses, extrapolation
// weights and the initial state (r0, v0, t0) on the device.
int adj_setup(mstar_ctx *ctx, const mstar_params *p, int64_t n, const double *m, const double *x, const double *v,
              double t0, int64_t nsteps, const double *H, int64_t ncp, int64_t seg) {
    int rc = check_params(ctx, p);
    if (rc) return rc;
    if (n < 2 || !m || !x || !v || nsteps < 0 || (nsteps > 0 && !H) || !std::isfinite(t0))
        return fail(ctx, MSTAR_E_INVAL, "replay: bad arguments");
    if (n > kAdjMaxN) return fail(ctx, MSTAR_E_UNSUPPORTED, "replay: n > %d is not implemented", kAdjMaxN);
    if (ttl_on(p)) return fail(ctx, MSTAR_E_UNSUPPORTED, "replay: beta != 0 (TTL) is not implemented");
    for (int64_t k = 0; k < nsteps; ++k)
        if (!std::isfinite(H[k]) || H[k] == 0.0) return fail(ctx, MSTAR_E_INVAL, "replay: H[%lld] invalid", (long long)k);
    (void)hipSetDevice(ctx->device);
    // work a failed adjoint call left on the second stream shares the division buffers
    if (ctx->a_s2) HIPCK(hipStreamSynchronize(ctx->a_s2));
    const uint32_t flags = p->flags;
    std::vector<double> hm((size_t)n), hx(3 * (size_t)n), hv(3 * (size_t)n);
    const hipMemcpyKind k = is_dev(flags) ? hipMemcpyDeviceToHost : hipMemcpyHostToHost;
    HIPCK(hipMemcpy(hm.data(), m, sizeof(double) * n, k));
    HIPCK(hipMemcpy(hx.data(), x, sizeof(double) * 3 * n, k));
    HIPCK(hipMemcpy(hv.data(), v, sizeof(double) * 3 * n, k));
    for (int64_t i = 0; i < n; ++i)
        if (!(hm[i] > 0.0) || !std::isfinite(hm[i])) return fail(ctx, MSTAR_E_INVAL, "mass %lld is not > 0", (long long)i);
    if (!finite_host(hx.data(), hx.size()) || !finite_host(hv.data(), hv.size()))
        return fail(ctx, MSTAR_E_NONFINITE, "non-finite position or velocity");
    if ((rc = ensure_adj(ctx, (int)n, p->k_fix, ncp, seg))) return rc;
    AdjDev &d = ctx->ad;
    d.G = p->G;
    d.alpha = p->alpha;
    d.gamma = p->gamma;
    // weights of the extrapolation to h = 0 in h^2, nodes h = H/n_k, n_k = 2k
    double c[kAdjMaxKF];
    for (int a = 0; a < p->k_fix; ++a) {
        const double na = (double)(2 * (a + 1)) * (double)(2 * (a + 1));
        double w = 1.0;
        for (int b = 0; b < p->k_fix; ++b)
            if (b != a) {
                const double nb = (double)(2 * (b + 1)) * (double)(2 * (b + 1));
                w = w * (na / (na - nb));
            }
        c[a] = w;
    }
    HIPCK(hipMemcpyAsync(ctx->a_m, hm.data(), sizeof(double) * n, hipMemcpyHostToDevice, ctx->stream));
    HIPCK(hipMemcpyAsync(ctx->a_c, c, sizeof(double) * p->k_fix, hipMemcpyHostToDevice, ctx->stream));
    HIPCK(hipMemcpyAsync(ctx->a_io[0], hx.data(), sizeof(double) * 3 * n, hipMemcpyHostToDevice, ctx->stream));
    HIPCK(hipMemcpyAsync(ctx->a_io[1], hv.data(), sizeof(double) * 3 * n, hipMemcpyHostToDevice, ctx->stream));
    launch_adj_pack(ctx->stream, (int)n, ctx->a_io[0], ctx->Yr, t0, ctx->Yt);
    launch_adj_pack(ctx->stream, (int)n, ctx->a_io[1], ctx->Yv, 0.0, nullptr);
    launch_adj_init(d, ctx->stream, ctx->Yr, ctx->Yv);
    HIPCK(hipGetLastError());
    HIPCK(hipStreamSynchronize(ctx->stream));   // host copies above are locals
    return MSTAR_OK;
}

// One replayed GBS step from (r, v, t) into (or, ov, ot) (may alias).
void adj_step(mstar_ctx *ctx, hipStream_t s, const d4 *r, const d4 *v, const double *t, double H, d4 *or_, d4 *ov,
              double *ot) {
    launch_adj_fwd(ctx->ad, s, r, v, t, H, false);
    launch_adj_combine(ctx->ad, s, r, v, t, or_, ov, ot);
}

// Kept substep states of one GBS step: every kick's positions, every drift's
// velocities and the op scalars of the k_fix divisions, 256-byte aligned.
size_t adj_step_bytes(int n, int kf) {
    const size_t kicks = (size_t)kf * (kf + 1), drifts = kicks + kf, ops = 2 * kicks + kf;
    const size_t b = sizeof(d4) * (kicks + drifts) * (size_t)n + sizeof(double) * kAdjOpScal * ops;
    return (b + 255) & ~size_t(255);
}
// AdjDev whose store pointers address step a of slot z (Q steps per slot).
AdjDev adj_slot(const mstar_ctx *ctx, int z, int64_t Q, int64_t a) {
    AdjDev d = ctx->ad;
    const size_t kicks = (size_t)d.kf * (d.kf + 1), drifts = kicks + d.kf;
    char *base = (char *)ctx->a_store + (size_t)(z * Q + a) * adj_step_bytes(d.n, d.kf);
    d.rst = (d4 *)base;
    d.vst = d.rst + kicks * (size_t)d.n;
    d.sc = (double *)(d.vst + drifts * (size_t)d.n);
    return d;
}
int ensure_adj_pipe(mstar_ctx *ctx, size_t bytes) {
    if (!ctx->a_s2) HIPCK(hipStreamCreateWithFlags(&ctx->a_s2, hipStreamNonBlocking));
    for (hipEvent_t &e : ctx->a_ev)
        if (!e) HIPCK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    if (bytes > ctx->a_store_cap) {
        HIPCK(hipStreamSynchronize(ctx->stream));
        HIPCK(hipStreamSynchronize(ctx->a_s2));
        if (ctx->a_store) (void)hipFree(ctx->a_store);
        ctx->a_store = nullptr;
        ctx->a_store_cap = 0;
        if (hipMalloc(&ctx->a_store, bytes) != hipSuccess)
            return fail(ctx, MSTAR_E_NOMEM, "device allocation of %zu bytes failed", bytes);
        ctx->a_store_cap = bytes;
    }
    return MSTAR_OK;
}

int adj_out(mstar_ctx *ctx, uint32_t flags, int64_t n, const d4 *a, double *dst, int io) {
    launch_adj_unpack(ctx->stream, (int)n, a, ctx->a_io[io]);
    return out_copy(ctx, flags, dst, ctx->a_io[io], sizeof(double) * 3 * n);
}

// Step k of the forward pass of the adjoint on stream st: the state goes to
// checkpoint k / C first when k is a multiple of C; H = 0 only stores the
// checkpoint (a record without steps).
void adj_forward_step(mstar_ctx *ctx, hipStream_t st, int64_t k, int64_t C, double H) {
    const size_t N = (size_t)ctx->ad.n;
    if (k % C == 0)
        launch_adj_copy(st, (int)N, ctx->Yr, ctx->Yv, ctx->Yt, ctx->cpr + (size_t)(k / C) * N,
                        ctx->cpv + (size_t)(k / C) * N, ctx->cpt + k / C);
    if (H != 0.0) adj_step(ctx, st, ctx->Yr, ctx->Yv, ctx->Yt, H, ctx->Yr, ctx->Yv, ctx->Yt);
}

// Forward pass of an adjoint fed by the driver: each accepted step is
// replayed on the second stream as soon as the driver has accepted it, so the
// pass runs alongside the integration instead of after it.
struct AdjFeed final : StepFeed {
    mstar_ctx *ctx;
    int64_t C, k = 0;
    AdjFeed(mstar_ctx *c, int64_t every) : ctx(c), C(every) {}
    int accepted(double H) override {
        adj_forward_step(ctx, ctx->a_s2, k++, C, H);
        const hipError_t e = hipGetLastError();
        return e == hipSuccess ? MSTAR_OK : fail(ctx, MSTAR_E_DEVICE, "adjoint replay launch: %s", hipGetErrorString(e));
    }
};

// Reverse pass of the adjoint over the n_steps recorded steps H, once the
// checkpoints are in place (the second stream must already be ordered after
// the forward pass): seeds, the pipelined reverse, the chain through B and
// the outputs.
int adj_reverse(mstar_ctx *ctx, const mstar_params *params, int64_t n, int64_t n_steps, const double *H, int64_t C,
                const double *gx, const double *gv, double gt, double *gx0, double *gv0, double *gm) {
    // seeds: cotangent of the end state
    const uint32_t flags = params->flags;
    const AdjDev &d = ctx->ad;
    const size_t N = (size_t)n;
    hipStream_t s = ctx->stream;
    const int64_t ncp = n_steps > 0 ? (n_steps + C - 1) / C : 1;
    int rc = 0;
    const void *gxd, *gvd;
    if ((rc = in_dev(ctx, flags, gx, ctx->a_io[0], sizeof(double) * 3 * n, &gxd))) return rc;
    if ((rc = in_dev(ctx, flags, gv, ctx->a_io[1], sizeof(double) * 3 * n, &gvd))) return rc;
    launch_adj_pack(s, (int)n, (const double *)gxd, d.Lr, gt, d.Lt);
    launch_adj_pack(s, (int)n, (const double *)gvd, d.Lv, 0.0, nullptr);
    launch_adj_zero(s, d.LB);
    launch_adj_zero_n(s, (int)n, d.Lm);
    // Reverse pass in blocks of at most Q steps, the last block first.  A
    // block is recomputed from its start state on the second stream, keeping
    // the substep states of all its steps in one of two slots, and then
    // reversed on the context's stream; the recomputation of the next block
    // runs while the current one is reversed.  A block is a whole checkpoint
    // segment when two segments' states fit the store (Q = C); otherwise the
    // segment's step states are first recomputed into sgr and its blocks
    // start there.  The kernels and their order per step are those of a
    // serial pass, so the result does not depend on C or Q.
    if (n_steps > 0) {
        const size_t sb = adj_step_bytes((int)n, d.kf);
        const int64_t Q = std::max<int64_t>(1, std::min<int64_t>(C, (int64_t)(ctx->a_store_max / (2 * sb))));
        if ((rc = ensure_adj_pipe(ctx, 2 * (size_t)Q * sb))) return rc;
        hipStream_t s2 = ctx->a_s2;
        hipEvent_t *kept = ctx->a_ev, *done = ctx->a_ev + 2;
        struct Blk { int64_t seg, b0, b1; };
        std::vector<Blk> blocks;   // in the order they are reversed
        for (int64_t seg = ncp - 1; seg >= 0; --seg) {
            const int64_t j0 = seg * C, j1 = std::min(n_steps, j0 + C);
            for (int64_t b1 = j1; b1 > j0; b1 -= Q) blocks.push_back(Blk{seg, std::max(j0, b1 - Q), b1});
        }
        auto recompute = [&](size_t i) -> int {
            const Blk &B = blocks[i];
            const int z = (int)(i & 1);
            const int64_t j0 = B.seg * C, j1 = std::min(n_steps, j0 + C);
            const d4 *sr = ctx->cpr + (size_t)B.seg * N, *sv = ctx->cpv + (size_t)B.seg * N;
            const double *st = ctx->cpt + B.seg;
            if (j1 - j0 > Q) {
                // the segment's step states, once per segment (its last block comes first)
                if (B.b1 == j1) {
                    launch_adj_copy(s2, (int)n, sr, sv, st, ctx->sgr, ctx->sgv, ctx->sgt);
                    for (int64_t j = j0; j < B.b0; ++j) {   // states up to the latest block start
                        const size_t a = (size_t)(j - j0), b = a + 1;
                        adj_step(ctx, s2, ctx->sgr + a * N, ctx->sgv + a * N, ctx->sgt + a, H[j], ctx->sgr + b * N,
                                 ctx->sgv + b * N, ctx->sgt + b);
                    }
                }
                const size_t a = (size_t)(B.b0 - j0);
                sr = ctx->sgr + a * N;
                sv = ctx->sgv + a * N;
                st = ctx->sgt + a;
            }
            if (i >= 2) HIPCK(hipStreamWaitEvent(s2, done[z], 0));   // the slot's previous block is reversed
            launch_adj_copy(s2, (int)n, sr, sv, st, ctx->brr, ctx->brv, ctx->brt);
            for (int64_t j = B.b0; j < B.b1; ++j) {
                launch_adj_fwd(adj_slot(ctx, z, Q, j - B.b0), s2, ctx->brr, ctx->brv, ctx->brt, H[j], true);
                if (j + 1 < B.b1) launch_adj_combine(d, s2, ctx->brr, ctx->brv, ctx->brt, ctx->brr, ctx->brv, ctx->brt);
            }
            HIPCK(hipEventRecord(kept[z], s2));
            return MSTAR_OK;
        };
        if ((rc = recompute(0))) return rc;
        for (size_t i = 0; i < blocks.size(); ++i) {
            if (i + 1 < blocks.size() && (rc = recompute(i + 1))) return rc;
            const Blk &B = blocks[i];
            const int z = (int)(i & 1);
            HIPCK(hipStreamWaitEvent(s, kept[z], 0));
            for (int64_t j = B.b1 - 1; j >= B.b0; --j) {
                launch_adj_rev(adj_slot(ctx, z, Q, j - B.b0), s);
                launch_adj_combine_rev(d, s);
            }
            HIPCK(hipEventRecord(done[z], s));
        }
    }
    launch_adj_finish(d, s, ctx->cpr, ctx->cpv, ctx->a_io[2], ctx->a_io[3], gm ? ctx->a_gm : nullptr);
    HIPCK(hipGetLastError());
    if ((rc = out_copy(ctx, flags, gx0, ctx->a_io[2], sizeof(double) * 3 * n))) return rc;
    if ((rc = out_copy(ctx, flags, gv0, ctx->a_io[3], sizeof(double) * 3 * n))) return rc;
    if (gm && (rc = out_copy(ctx, flags, gm, ctx->a_gm, sizeof(double) * n))) return rc;
    HIPCK(hipStreamSynchronize(s));
    return MSTAR_OK;
}


}  // namespace

extern "C" {

int mstar_replay(mstar_ctx *ctx, const mstar_params *params, int64_t n, const double *m, double *x, double *v,
                 double t0, int64_t n_steps, const double *H, double *t_out) {
    if (!ctx) return MSTAR_E_INVAL;
    ctx->err.clear();
    int rc = adj_setup(ctx, params, n, m, x, v, t0, n_steps, H, 1, 1);
    if (rc) return rc;
    for (int64_t k = 0; k < n_steps; ++k)
        adj_step(ctx, ctx->stream, ctx->Yr, ctx->Yv, ctx->Yt, H[k], ctx->Yr, ctx->Yv, ctx->Yt);
    HIPCK(hipGetLastError());
    const uint32_t flags = params->flags;
    if ((rc = adj_out(ctx, flags, n, ctx->Yr, x, 2))) return rc;
    if ((rc = adj_out(ctx, flags, n, ctx->Yv, v, 3))) return rc;
    double t = 0.0;
    HIPCK(hipMemcpyAsync(&t, ctx->Yt, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HIPCK(hipStreamSynchronize(ctx->stream));
    if (t_out) *t_out = t;
    return MSTAR_OK;
}

int mstar_replay_adjoint(mstar_ctx *ctx, const mstar_params *params, int64_t n, const double *m, const double *x0,
                         const double *v0, double t0, int64_t n_steps, const double *H, int32_t checkpoint_every,
                         const double *gx, const double *gv, double gt, double *gx0, double *gv0, double *gm) {
    if (!ctx) return MSTAR_E_INVAL;
    ctx->err.clear();
    if (checkpoint_every < 1 || !gx || !gv || !gx0 || !gv0 || !std::isfinite(gt))
        return fail(ctx, MSTAR_E_INVAL, "replay_adjoint: bad arguments");
    const int64_t C = checkpoint_every;
    const int64_t ncp = n_steps > 0 ? (n_steps + C - 1) / C : 1;
    int rc = adj_setup(ctx, params, n, m, x0, v0, t0, n_steps, H, ncp, C);
    if (rc) return rc;
    hipStream_t s = ctx->stream;
    // forward pass, keeping the state at every C-th step
    for (int64_t k = 0; k < n_steps; ++k) adj_forward_step(ctx, s, k, C, H[k]);
    if (n_steps == 0) adj_forward_step(ctx, s, 0, C, 0.0);
    if ((rc = ensure_adj_pipe(ctx, 0))) return rc;
    HIPCK(hipEventRecord(ctx->a_ev[4], s));   // checkpoints in place: the recomputation may start
    HIPCK(hipStreamWaitEvent(ctx->a_s2, ctx->a_ev[4], 0));
    return adj_reverse(ctx, params, n, n_steps, H, C, gx, gv, gt, gx0, gv0, gm);
}

int mstar_adjoint_store_limit(mstar_ctx *ctx, int64_t bytes) {
    if (!ctx) return MSTAR_E_INVAL;
    ctx->err.clear();
    if (bytes < 0) return fail(ctx, MSTAR_E_INVAL, "adjoint_store_limit: bytes < 0");
    ctx->a_store_max = bytes == 0 ? size_t(4) << 30 : (size_t)bytes;
    return MSTAR_OK;
}

int mstar_integrate_adjoint(mstar_ctx *ctx, const mstar_params *params, int64_t n, const double *m, const double *x0,
                            const double *v0, double t0, double t_end, int64_t n_steps, int32_t checkpoint_every,
                            const double *gxT, const double *gvT, double gtT, double *gx0, double *gv0, double *gm,
                            mstar_stats *stats) {
    if (!ctx) return MSTAR_E_INVAL;
    ctx->err.clear();
    if (!params || n < 2 || n > kAdjMaxN || !m || !x0 || !v0 || n_steps < 1 || checkpoint_every < 1 || !gxT ||
        !gvT || !gx0 || !gv0 || !std::isfinite(gtT))
        return fail(ctx, n > kAdjMaxN ? MSTAR_E_UNSUPPORTED : MSTAR_E_INVAL, "integrate_adjoint: bad arguments");
    if (ttl_on(params)) return fail(ctx, MSTAR_E_UNSUPPORTED, "integrate_adjoint: beta != 0 (TTL) is not implemented");
    (void)hipSetDevice(ctx->device);
    // the adjoint's start state and B from the caller's x0, v0; the driver
    // then feeds every accepted step to its forward pass on the second stream
    const int64_t C = checkpoint_every;
    int rc = adj_setup(ctx, params, n, m, x0, v0, t0, 0, nullptr, (n_steps + C - 1) / C, C);
    if (rc) return rc;
    if ((rc = ensure_adj_pipe(ctx, 0))) return rc;   // adj_setup has synchronised ctx->stream
    // forward: the integrator, recording the accepted steps, on copies of x0, v0
    const size_t b3 = sizeof(double) * 3 * (size_t)n;
    std::vector<double> hx(3 * (size_t)n), hv(3 * (size_t)n), hm((size_t)n);
    const hipMemcpyKind k = is_dev(params->flags) ? hipMemcpyDeviceToHost : hipMemcpyHostToHost;
    HIPCK(hipMemcpy(hx.data(), x0, b3, k));
    HIPCK(hipMemcpy(hv.data(), v0, b3, k));
    HIPCK(hipMemcpy(hm.data(), m, sizeof(double) * n, k));
    mstar_params ph = *params;
    ph.flags &= ~MSTAR_DEVICE_PTRS;
    std::vector<double> H((size_t)n_steps);
    int64_t nrec = 0;
    mstar_stats st{};
    st.struct_size = sizeof(mstar_stats);
    AdjFeed feed(ctx, C);
    rc = integrate_impl(ctx, &ph, n, hm.data(), hx.data(), hv.data(), t0, t_end, &st, n_steps, H.data(), &nrec,
                        nullptr, &feed);
    if (stats) *stats = st;
    if (rc < 0) return rc;
    if (nrec == 0) adj_forward_step(ctx, ctx->a_s2, 0, C, 0.0);   // the checkpoint of the start state only
    HIPCK(hipEventRecord(ctx->a_ev[4], ctx->a_s2));   // the forward pass is complete: reverse on ctx->stream
    HIPCK(hipStreamWaitEvent(ctx->stream, ctx->a_ev[4], 0));
    // reverse: the adjoint of the recorded steps
    const int rc2 = adj_reverse(ctx, params, n, nrec, H.data(), C, gxT, gvT, gtT, gx0, gv0, gm);
    return rc2 ? rc2 : rc;
}

int mstar_force_hvp(mstar_ctx *ctx, const mstar_params *params, int64_t n, const double *m, const double *x,
                    const double *w, double *out) {
    if (!ctx) return MSTAR_E_INVAL;
    int rc = check_params(ctx, params);
    if (rc) return rc;
    if (n < 2 || n > (1 << 24) || !m || !x || !w || !out) return fail(ctx, MSTAR_E_INVAL, "force_hvp: bad arguments");
    (void)hipSetDevice(ctx->device);
    const uint32_t flags = params->flags;
    if ((rc = ensure(ctx, (int)n))) return rc;
    if ((rc = load_bodies(ctx, flags, n, m, x, nullptr, nullptr))) return rc;
    const void *xd, *wd;
    if ((rc = in_dev(ctx, flags, x, ctx->xin, sizeof(double) * 3 * n, &xd))) return rc;
    if ((rc = in_dev(ctx, flags, w, ctx->vin, sizeof(double) * 3 * n, &wd))) return rc;
    launch_force_hvp(ctx->stream, (int)n, params->G, ctx->d.m, (const double *)xd, (const double *)wd, ctx->xout);
    HIPCK(hipGetLastError());
    if ((rc = out_copy(ctx, flags, out, ctx->xout, sizeof(double) * 3 * n))) return rc;
    HIPCK(hipStreamSynchronize(ctx->stream));
    return MSTAR_OK;
}

}  // extern "C"

// ------------------------------------------------------------------------
// Coordinate round trips (kernels_rebuild.hip).

extern "C" int mstar_rebuild_cycles(mstar_ctx *ctx, uint32_t flags, int32_t n_sys, const int64_t *offsets,
                                    const int32_t *kinds, const double *m, const double *x, const double *v,
                                    int64_t n_cycles, int32_t n_out, double *x_out, double *v_out,
                                    double *mean_level) {
    if (!ctx) return MSTAR_E_INVAL;
    ctx->err.clear();
    if (n_sys < 1 || !offsets || !kinds || !m || !x || !v || n_cycles < 0 || n_out < 0 ||
        (n_out > 0 && (!x_out || !v_out)))
        return fail(ctx, MSTAR_E_INVAL, "rebuild_cycles: bad arguments");
    (void)hipSetDevice(ctx->device);
    std::vector<int64_t> off((size_t)n_sys + 1);
    std::vector<int32_t> kd((size_t)n_sys);
    if (is_dev(flags)) {
        HIPCK(hipMemcpy(off.data(), offsets, sizeof(int64_t) * (n_sys + 1), hipMemcpyDeviceToHost));
        HIPCK(hipMemcpy(kd.data(), kinds, sizeof(int32_t) * n_sys, hipMemcpyDeviceToHost));
    } else {
        memcpy(off.data(), offsets, sizeof(int64_t) * (n_sys + 1));
        memcpy(kd.data(), kinds, sizeof(int32_t) * n_sys);
    }
    if (off[0] != 0) return fail(ctx, MSTAR_E_INVAL, "rebuild_cycles: offsets[0] must be 0");
    for (int32_t s = 0; s < n_sys; ++s) {
        const int64_t n = off[s + 1] - off[s];
        if (n < 2 || n > kRebuildMaxN)
            return fail(ctx, MSTAR_E_INVAL, "rebuild_cycles: system %d has %lld bodies (need 2..%d)", s, (long long)n,
                        kRebuildMaxN);
        if (kd[s] < 0 || kd[s] > 3) return fail(ctx, MSTAR_E_INVAL, "rebuild_cycles: kind must be 0..3");
    }
    const int64_t n_tot = off[n_sys];
    // device buffers for this call (freed before returning)
    std::vector<void *> bufs;
    auto alloc = [&](size_t bytes, void **p) -> int {
        if (hipMalloc(p, bytes ? bytes : 1) != hipSuccess) return fail(ctx, MSTAR_E_NOMEM, "rebuild_cycles: allocation failed");
        bufs.push_back(*p);
        return MSTAR_OK;
    };
    auto release = [&]() { for (void *p : bufs) (void)hipFree(p); };
    RebuildArgs a{};
    int64_t *d_off; int32_t *d_kind, *d_next; double *d_m, *d_x, *d_v, *d_xo, *d_vo, *d_ls; RebuildArgs *d_args;
    int rc = 0;
    if ((rc = alloc(sizeof(int64_t) * (n_sys + 1), (void **)&d_off)) || (rc = alloc(sizeof(int32_t) * n_sys, (void **)&d_kind)) ||
        (rc = alloc(sizeof(int32_t) * n_sys, (void **)&d_next)) || (rc = alloc(sizeof(double) * n_tot, (void **)&d_m)) ||
        (rc = alloc(sizeof(double) * 3 * n_tot, (void **)&d_x)) || (rc = alloc(sizeof(double) * 3 * n_tot, (void **)&d_v)) ||
        (rc = alloc(sizeof(double) * 3 * n_tot * (size_t)n_out, (void **)&d_xo)) ||
        (rc = alloc(sizeof(double) * 3 * n_tot * (size_t)n_out, (void **)&d_vo)) ||
        (rc = alloc(sizeof(double) * n_sys, (void **)&d_ls)) || (rc = alloc(sizeof(RebuildArgs), (void **)&d_args))) {
        release();
        return rc;
    }
    const hipMemcpyKind k = is_dev(flags) ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    hipError_t e = hipSuccess;
    auto ck = [&](hipError_t r) { if (e == hipSuccess) e = r; };
    ck(hipMemcpyAsync(d_off, off.data(), sizeof(int64_t) * (n_sys + 1), hipMemcpyHostToDevice, ctx->stream));
    ck(hipMemcpyAsync(d_kind, kd.data(), sizeof(int32_t) * n_sys, hipMemcpyHostToDevice, ctx->stream));
    ck(hipMemcpyAsync(d_m, m, sizeof(double) * n_tot, k, ctx->stream));
    ck(hipMemcpyAsync(d_x, x, sizeof(double) * 3 * n_tot, k, ctx->stream));
    ck(hipMemcpyAsync(d_v, v, sizeof(double) * 3 * n_tot, k, ctx->stream));
    ck(hipMemsetAsync(d_ls, 0, sizeof(double) * n_sys, ctx->stream));
    ck(hipMemsetAsync(d_next, 0, sizeof(int32_t) * n_sys, ctx->stream));
    a.off = d_off; a.kind = d_kind; a.m = d_m; a.x = d_x; a.v = d_v;
    a.n_cycles = n_cycles; a.n_tot = n_tot; a.n_out = n_out;
    a.x_out = d_xo; a.v_out = d_vo; a.level_sum = d_ls; a.next_out = d_next;
    ck(hipMemcpyAsync(d_args, &a, sizeof a, hipMemcpyHostToDevice, ctx->stream));
    // launches of at most kChunk cycles keep every kernel short
    constexpr int64_t kChunk = 500;
    for (int64_t c0 = 0; c0 < n_cycles && e == hipSuccess; c0 += kChunk) {
        launch_rebuild(ctx->stream, d_args, n_sys, c0, std::min(n_cycles, c0 + kChunk));
        ck(hipGetLastError());
    }
    std::vector<double> ls((size_t)n_sys);
    if (n_out > 0) {
        const hipMemcpyKind ko = is_dev(flags) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
        ck(hipMemcpyAsync(x_out, d_xo, sizeof(double) * 3 * n_tot * n_out, ko, ctx->stream));
        ck(hipMemcpyAsync(v_out, d_vo, sizeof(double) * 3 * n_tot * n_out, ko, ctx->stream));
    }
    ck(hipMemcpyAsync(ls.data(), d_ls, sizeof(double) * n_sys, hipMemcpyDeviceToHost, ctx->stream));
    ck(hipStreamSynchronize(ctx->stream));
    release();
    if (e != hipSuccess) return fail(ctx, MSTAR_E_DEVICE, "rebuild_cycles: %s", hipGetErrorString(e));
    if (mean_level)
        for (int32_t s = 0; s < n_sys; ++s) mean_level[s] = n_cycles > 0 ? ls[s] / (double)n_cycles : 0.0;
    return MSTAR_OK;
}
