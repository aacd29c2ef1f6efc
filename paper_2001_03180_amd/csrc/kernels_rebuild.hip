// Coordinate round trips (paper Sec. 3.5): the coordinate structure -- the
// minimum spanning tree of Sec. 3.1-3.4 or the chain of Sec. 2.2 -- is built
// from the Cartesian state, its edge vectors formed and the state rebuilt from
// them (Sec. 2.2 deconstruction), many times over; the physical state does not
// change, so whatever the state drifts by is the rounding these transforms
// accumulate, and its size follows the mean depth of the structure.
//
// One wave per system (N <= kRebuildMaxN, bodies i = lane + 64 k), the state
// in LDS for the cycles of one launch:
//  * MST: Prim's algorithm under the strict edge order (w, min index, max
//    index), rooted at the body nearest the centre of mass, with each step's
//    minimum found in two levels (weight, then the packed index pair) across
//    the wave.
//  * chain: the two ends of the shortest edge start it; the body nearest to
//    either end (same strict order) joins at that end; the tree is rooted at
//    the final tail.
//  * edge vectors X_v = x_v - x_parent(v); root-relative positions rho by
//    levels, parents first (rho_v = rho_parent + X_v, so each rho_v is the
//    top-down sum along its path); x = r_cm + (rho - rho_bar), velocities alike.
//  * centre-of-mass sums are compensated (Neumaier) per lane, the lanes'
//    sums and corrections combined in a fixed order; or (kind bit 2) plain
//    sums in index order, as in the paper's test, which then repeats the
//    oracle's round trips bit for bit.
#include "common.h"
#include "rebuild.h"

namespace mstar {

namespace {

constexpr int kPer = kRebuildMaxN / 64;   // bodies per lane

__device__ __forceinline__ double wmin64(double w) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) w = fmin(w, __shfl_xor(w, o, 64));
    return w;
}
__device__ __forceinline__ uint32_t umin64(uint32_t k) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) k = min(k, (uint32_t)__shfl_xor((int)k, o, 64));
    return k;
}
__device__ __forceinline__ int imax64(int k) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) k = max(k, __shfl_xor(k, o, 64));
    return k;
}
__device__ __forceinline__ void lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Neumaier accumulation and the combination of two partial sums.
struct Comp {
    double s, c;
};
__device__ __forceinline__ void comp_add(Comp &a, double x) {
    const double t = a.s + x;
    if (fabs(a.s) >= fabs(x)) a.c = a.c + ((a.s - t) + x);
    else a.c = a.c + ((x - t) + a.s);
    a.s = t;
}
// Sum over the wave of the lanes' compensated sums: lane sums added with
// compensation in a fixed butterfly order, the corrections summed alongside.
__device__ __forceinline__ double comp_wave(Comp a) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double s2 = __shfl_xor(a.s, o, 64), c2 = __shfl_xor(a.c, o, 64);
        const int lane = __lane_id();
        // both partners form the same sum: the lower lane's value first
        const double lo_s = (lane & o) ? s2 : a.s, hi_s = (lane & o) ? a.s : s2;
        const double lo_c = (lane & o) ? c2 : a.c, hi_c = (lane & o) ? a.c : c2;
        Comp r{lo_s, lo_c + hi_c};
        comp_add(r, hi_s);
        a = r;
    }
    return a.s + a.c;
}

struct RebLDS {
    double x[3][kRebuildMaxN], v[3][kRebuildMaxN], rho[3][kRebuildMaxN];
    double m[kRebuildMaxN];
    int parent[kRebuildMaxN], level[kRebuildMaxN];
    int in[kRebuildMaxN];
};

__device__ __forceinline__ double sqd(const RebLDS &S, int i, int j) {
    const double dx = S.x[0][j] - S.x[0][i], dy = S.x[1][j] - S.x[1][i], dz = S.x[2][j] - S.x[2][i];
    return (dx * dx + dy * dy) + dz * dz;   // -ffp-contract=off: no fusion
}

// Strict edge order (w, min index, max index).
__device__ __forceinline__ bool key_lt(double w1, int a1, int b1, double w2, int a2, int b2) {
    const int lo1 = min(a1, b1), hi1 = max(a1, b1), lo2 = min(a2, b2), hi2 = max(a2, b2);
    if (w1 != w2) return w1 < w2;
    if (lo1 != lo2) return lo1 < lo2;
    return hi1 < hi2;
}

// Wave minimum of per-lane candidate keys (w, a, b) under the strict order;
// returns the packed (min, max) indices of the minimum edge.
__device__ __forceinline__ uint32_t wave_key_min(double w, int a, int b, bool valid) {
    const double wm = wmin64(valid ? w : INFINITY);
    const uint32_t k = (valid && w == wm) ? (((uint32_t)min(a, b) << 16) | (uint32_t)max(a, b)) : 0xffffffffu;
    return umin64(k);
}

// Centre of mass: compensated lane sums combined in a fixed order, or (plain)
// one lane's plain sums in index order, the order of the paper's test.
__device__ __forceinline__ void com_of(const RebLDS &S, const double (&arr)[3][kRebuildMaxN], int n, double out[3],
                                       bool plain) {
    const int lane = __lane_id();
    if (plain) {
        double M = 0.0, s0 = 0.0, s1 = 0.0, s2 = 0.0;
        if (lane == 0)
            for (int i = 0; i < n; ++i) {
                M = M + S.m[i];
                s0 = s0 + S.m[i] * arr[0][i];
                s1 = s1 + S.m[i] * arr[1][i];
                s2 = s2 + S.m[i] * arr[2][i];
            }
        out[0] = __shfl(s0 / M, 0, 64);
        out[1] = __shfl(s1 / M, 0, 64);
        out[2] = __shfl(s2 / M, 0, 64);
        return;
    }
    Comp M{0.0, 0.0}, s[3] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
    for (int k = 0; k < kPer; ++k) {
        const int i = lane + 64 * k;
        if (i < n) {
            comp_add(M, S.m[i]);
            for (int c = 0; c < 3; ++c) comp_add(s[c], S.m[i] * arr[c][i]);
        }
    }
    const double Mt = comp_wave(M);
    for (int c = 0; c < 3; ++c) out[c] = comp_wave(s[c]) / Mt;
}

// MST (kind 0) or chain (kind 1) on the positions in S.x: parent[], level[].
__device__ void build(RebLDS &S, int n, int kind, const double rcm[3]) {
    const int lane = __lane_id();
    for (int k = 0; k < kPer; ++k) {
        const int i = lane + 64 * k;
        if (i < n) S.in[i] = 0;
    }
    lds_sync();
    double bw[kPer];
    int bu[kPer];
    int head = -1, tail = -1;
    if (kind == 0) {
        // root: nearest to the centre of mass, ties to the lowest index
        double w = INFINITY;
        int r = 0x7fffffff;
        for (int k = 0; k < kPer; ++k) {
            const int i = lane + 64 * k;
            if (i < n) {
                const double dx = S.x[0][i] - rcm[0], dy = S.x[1][i] - rcm[1], dz = S.x[2][i] - rcm[2];
                const double wi = (dx * dx + dy * dy) + dz * dz;
                if (wi < w || (wi == w && i < r)) { w = wi; r = i; }
            }
        }
        const double wm = wmin64(w);
        const int root = (int)umin64(w == wm ? (uint32_t)r : 0xffffffffu);
        if (lane == 0) {
            S.in[root] = 1;
            S.parent[root] = -1;
            S.level[root] = 0;
        }
        lds_sync();
        for (int k = 0; k < kPer; ++k) {
            const int i = lane + 64 * k;
            bw[k] = (i < n && i != root) ? sqd(S, root, i) : INFINITY;
            bu[k] = root;
        }
        for (int step = 1; step < n; ++step) {
            double w1 = INFINITY;
            int a1 = 0, b1 = 0;
            bool any = false;
            for (int k = 0; k < kPer; ++k) {
                const int i = lane + 64 * k;
                if (i < n && !S.in[i] && (!any || key_lt(bw[k], bu[k], i, w1, a1, b1))) {
                    w1 = bw[k]; a1 = bu[k]; b1 = i; any = true;
                }
            }
            const uint32_t km = wave_key_min(w1, a1, b1, any);
            if (km == 0xffffffffu) break;   // no candidate left (cannot happen for step < n)
            const int lo = (int)(km >> 16), hi = (int)(km & 0xffffu);
            const int pick = S.in[lo] ? hi : lo;
            const int pu = pick == lo ? hi : lo;
            if (lane == 0) {
                S.in[pick] = 1;
                S.parent[pick] = pu;
                S.level[pick] = S.level[pu] + 1;
            }
            lds_sync();
            for (int k = 0; k < kPer; ++k) {
                const int i = lane + 64 * k;
                if (i < n && !S.in[i]) {
                    const double w = sqd(S, pick, i);
                    if (key_lt(w, pick, i, bw[k], bu[k], i)) { bw[k] = w; bu[k] = pick; }
                }
            }
        }
        return;
    }
    // chain: the shortest edge over all pairs
    {
        double w1 = INFINITY;
        int a1 = 0, b1 = 0;
        bool any = false;
        for (int k = 0; k < kPer; ++k) {
            const int i = lane + 64 * k;
            if (i >= n) continue;
            for (int j = i + 1; j < n; ++j) {
                const double w = sqd(S, i, j);
                if (!any || key_lt(w, i, j, w1, a1, b1)) { w1 = w; a1 = i; b1 = j; any = true; }
            }
        }
        const uint32_t km = wave_key_min(w1, a1, b1, any);
        tail = (int)(km >> 16);
        head = (int)(km & 0xffffu);
    }
    // the chain grows at both ends; positions along it are kept relative to
    // the first tail (pos), so levels are pos - (final tail's pos)
    if (lane == 0) {
        S.in[tail] = 1;
        S.in[head] = 1;
        S.parent[tail] = -1;     // fixed below once the final tail is known
        S.parent[head] = tail;
        S.level[tail] = 0;
        S.level[head] = 1;
    }
    lds_sync();
    int tpos = 0;                // position of the current tail
    for (int added = 2; added < n; ++added) {
        double w1 = INFINITY;
        int e1 = 0, u1 = 0;
        bool any = false;
        for (int k = 0; k < kPer; ++k) {
            const int u = lane + 64 * k;
            if (u >= n || S.in[u]) continue;
            const double wt = sqd(S, tail, u), wh = sqd(S, head, u);
            int e = tail;
            double w = wt;
            if (key_lt(wh, head, u, wt, tail, u)) { e = head; w = wh; }
            if (!any || key_lt(w, e, u, w1, e1, u1)) { w1 = w; e1 = e; u1 = u; any = true; }
        }
        const uint32_t km = wave_key_min(w1, e1, u1, any);
        if (km == 0xffffffffu) break;       // no body left outside the chain (cannot happen)
        const int lo = (int)(km >> 16), hi = (int)(km & 0xffffu);
        const int pick = S.in[lo] ? hi : lo;
        const int end = pick == lo ? hi : lo;
        if (lane == 0) {
            S.in[pick] = 1;
            if (end == tail) {       // new tail: the old tail now hangs from it
                S.parent[tail] = pick;
                S.parent[pick] = -1;
                S.level[pick] = tpos - 1;
            } else {
                S.parent[pick] = head;
                S.level[pick] = S.level[head] + 1;
            }
        }
        if (end == tail) { tail = pick; --tpos; }
        else head = pick;
        lds_sync();
    }
    // levels relative to the final tail
    for (int k = 0; k < kPer; ++k) {
        const int i = lane + 64 * k;
        if (i < n) S.level[i] = S.level[i] - tpos;
    }
    lds_sync();
}

// rho_v = rho_parent + (a_v - a_parent) by levels; then out = base + (rho - rho_bar).
__device__ void rebuild_one(RebLDS &S, int n, int maxl, double (&a)[3][kRebuildMaxN], const double base[3],
                            bool plain) {
    const int lane = __lane_id();
    for (int k = 0; k < kPer; ++k) {
        const int i = lane + 64 * k;
        if (i < n && S.parent[i] < 0) S.rho[0][i] = S.rho[1][i] = S.rho[2][i] = 0.0;
    }
    lds_sync();
    for (int L = 1; L <= maxl; ++L) {
        for (int k = 0; k < kPer; ++k) {
            const int i = lane + 64 * k;
            if (i < n && S.level[i] == L) {
                const int q = S.parent[i];
                for (int c = 0; c < 3; ++c) S.rho[c][i] = S.rho[c][q] + (a[c][i] - a[c][q]);
            }
        }
        lds_sync();
    }
    double cb[3];
    com_of(S, S.rho, n, cb, plain);
    lds_sync();
    for (int k = 0; k < kPer; ++k) {
        const int i = lane + 64 * k;
        if (i < n)
            for (int c = 0; c < 3; ++c) a[c][i] = base[c] + (S.rho[c][i] - cb[c]);
    }
    lds_sync();
}

__global__ __launch_bounds__(64) void k_rebuild(const RebuildArgs *__restrict__ args, int64_t c0, int64_t c1) {
    __shared__ RebLDS S;
    const RebuildArgs &A = *args;
    const int sys = blockIdx.x;
    const int lane = threadIdx.x;
    const int64_t o = A.off[sys];
    const int n = (int)(A.off[sys + 1] - o);
    const int kind = A.kind[sys];
    const bool plain = (kind & 2) != 0;
    for (int k = 0; k < kPer; ++k) {
        const int i = lane + 64 * k;
        if (i < n) {
            S.m[i] = A.m[o + i];
            for (int c = 0; c < 3; ++c) {
                S.x[c][i] = A.x[3 * (o + i) + c];
                S.v[c][i] = A.v[3 * (o + i) + c];
            }
        }
    }
    lds_sync();
    double lsum = 0.0;
    int kout = (int)A.next_out[sys];
    for (int64_t cyc = c0 + 1; cyc <= c1; ++cyc) {
        double rcm[3], vcm[3];
        com_of(S, S.x, n, rcm, plain);
        com_of(S, S.v, n, vcm, plain);
        build(S, n, kind & 1, rcm);
        int ml = 0;
        long ls = 0;
        for (int k = 0; k < kPer; ++k) {
            const int i = lane + 64 * k;
            if (i < n) {
                ml = max(ml, S.level[i]);
                ls += S.level[i];
            }
        }
        const int maxl = imax64(ml);
        double lsd = (double)ls;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) lsd = lsd + __shfl_xor(lsd, off, 64);
        lsum = lsum + lsd / n;
        rebuild_one(S, n, maxl, S.x, rcm, plain);
        rebuild_one(S, n, maxl, S.v, vcm, plain);
        while (kout < A.n_out && cyc == ((int64_t)(kout + 1) * A.n_cycles) / A.n_out) {
            double *xo = A.x_out + ((size_t)kout * A.n_tot + o) * 3, *vo = A.v_out + ((size_t)kout * A.n_tot + o) * 3;
            for (int k = 0; k < kPer; ++k) {
                const int i = lane + 64 * k;
                if (i < n)
                    for (int c = 0; c < 3; ++c) {
                        xo[3 * i + c] = S.x[c][i];
                        vo[3 * i + c] = S.v[c][i];
                    }
            }
            ++kout;
        }
    }
    // carry the state to the next launch
    for (int k = 0; k < kPer; ++k) {
        const int i = lane + 64 * k;
        if (i < n)
            for (int c = 0; c < 3; ++c) {
                A.x[3 * (o + i) + c] = S.x[c][i];
                A.v[3 * (o + i) + c] = S.v[c][i];
            }
    }
    if (lane == 0) {
        A.level_sum[sys] = A.level_sum[sys] + lsum;
        A.next_out[sys] = kout;
    }
}

}  // namespace

void launch_rebuild(hipStream_t s, const RebuildArgs *a, int n_sys, int64_t c0, int64_t c1) {
    k_rebuild<<<n_sys, 64, 0, s>>>(a, c0, c1);
}

}  // namespace mstar
