// Many small independent systems integrated in one persistent launch (the
// paper notes in Sec. 4.2 that the method extends to several independent
// N-body systems at once).
//
// Each system is integrated start to end on the device: MST by Prim's
// algorithm (Sec. 3.2), GBS steps (Sec. 2.3) whose k_fix substep divisions
// run concurrently, the error test and step control (eq. gbs-criterion,
// eq. hnext), MST rebuilds (Sec. 3.5) and the end-time iteration (Sec. 2.4),
// following the same arithmetic as the single-system path.
//
// Tiles: a system's bodies map to the lanes of a lane group of width L
// (L >= N).  Group g runs the division pairs (n, 2 k_fix + 2 - n) starting at
// n = 2(g + 1) (the balanced grouping of Sec. 4.2: every pair costs
// 2 k_fix + 2 kicks), so the groups need no synchronisation inside a step.
//  - cooperative tile: 4 groups of 64 lanes = the 4 waves of a workgroup;
//  - wave tile: 64 / L groups of L lanes inside one wave, one system per
//    wave, each wave of the workgroup working on its own system.
// Systems are pulled from two queues (cooperative first), each ordered by
// decreasing estimated cost, so the persistent grid stays balanced.  Within a
// group the MST transforms are pointer jumping over the parents with lane
// shuffles, the force loop reads j-positions from LDS, and U, T and the
// centre-of-mass sums are butterfly reductions (identical in every lane).
#include "../../include/mstar.h"
#include "batch.h"

namespace mstar {
namespace {

constexpr int kBatchWG = 256;

// ---------------------------------------------------------------- lane groups
template <int L>
__device__ __forceinline__ int glane() { return (int)(threadIdx.x & (L - 1)); }

// Sums over a lane group without LDS traffic: DPP moves inside 16-lane rows
// (quad swaps, then the mirrored half-row and row) and the gfx950 row-swap
// instructions across rows.  Every step pairs lanes that hold equal partial
// sums, so all lanes end with the same bits; lanes past the group's bodies
// hold zeros, so the result does not depend on the group width.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    return __builtin_amdgcn_update_dpp(0.0, v, CTRL, 0xF, 0xF, false);
}
__device__ __forceinline__ double row_swap_sum(double v, bool wide) {
    const uint64_t u = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = (uint32_t)u, hi = (uint32_t)(u >> 32);
    uint32_t a0, a1, b0, b1;
    if (wide) {   // rows (0,1) <-> rows (2,3)
        const auto l = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
        const auto h = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
        a0 = l[0]; b0 = l[1]; a1 = h[0]; b1 = h[1];
    } else {      // row 0 <-> row 1, row 2 <-> row 3
        const auto l = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
        const auto h = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
        a0 = l[0]; b0 = l[1]; a1 = h[0]; b1 = h[1];
    }
    const double a = __longlong_as_double((long long)(((uint64_t)a1 << 32) | a0));
    const double b = __longlong_as_double((long long)(((uint64_t)b1 << 32) | b0));
    return a + b;
}
template <int L>
__device__ __forceinline__ double gsum(double v) {
    static_assert(L == 16 || L == 32 || L == 64, "lane groups of 16, 32 or 64");
    v = v + dpp_f64<0xB1>(v);     // quad_perm [1,0,3,2]
    v = v + dpp_f64<0x4E>(v);     // quad_perm [2,3,0,1]
    v = v + dpp_f64<0x141>(v);    // row_half_mirror
    v = v + dpp_f64<0x140>(v);    // row_mirror
    if (L >= 32) v = row_swap_sum(v, false);
    if (L >= 64) v = row_swap_sum(v, true);
    return v;
}
template <int L>
__device__ __forceinline__ void gsum3(double &a, double &b, double &c) {
    static_assert(L == 16 || L == 32 || L == 64, "lane groups of 16, 32 or 64");
    a = a + dpp_f64<0xB1>(a); b = b + dpp_f64<0xB1>(b); c = c + dpp_f64<0xB1>(c);
    a = a + dpp_f64<0x4E>(a); b = b + dpp_f64<0x4E>(b); c = c + dpp_f64<0x4E>(c);
    a = a + dpp_f64<0x141>(a); b = b + dpp_f64<0x141>(b); c = c + dpp_f64<0x141>(c);
    a = a + dpp_f64<0x140>(a); b = b + dpp_f64<0x140>(b); c = c + dpp_f64<0x140>(c);
    if (L >= 32) { a = row_swap_sum(a, false); b = row_swap_sum(b, false); c = row_swap_sum(c, false); }
    if (L >= 64) { a = row_swap_sum(a, true); b = row_swap_sum(b, true); c = row_swap_sum(c, true); }
}
// Value of the butterfly partner at step q (the pairing used by gsum):
// quad swaps, mirrored half-row and row, then the row swaps.
template <int CTRL>
__device__ __forceinline__ int dpp_i32(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}
__device__ __forceinline__ uint32_t swap_partner_u32(uint32_t v, bool wide) {
    const int lane = __lane_id();
    if (wide) {
        const auto l = __builtin_amdgcn_permlane32_swap(v, v, false, false);
        return ((lane >> 5) & 1) ? l[0] : l[1];
    }
    const auto l = __builtin_amdgcn_permlane16_swap(v, v, false, false);
    return ((lane >> 4) & 1) ? l[0] : l[1];
}
template <int Q>
__device__ __forceinline__ double partner_f64(double v) {
    if constexpr (Q == 0) return dpp_f64<0xB1>(v);
    else if constexpr (Q == 1) return dpp_f64<0x4E>(v);
    else if constexpr (Q == 2) return dpp_f64<0x141>(v);
    else if constexpr (Q == 3) return dpp_f64<0x140>(v);
    else {
        const uint64_t u = (uint64_t)__double_as_longlong(v);
        const uint32_t lo = swap_partner_u32((uint32_t)u, Q == 5), hi = swap_partner_u32((uint32_t)(u >> 32), Q == 5);
        return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
    }
}
template <int Q>
__device__ __forceinline__ int partner_i32(int v) {
    if constexpr (Q == 0) return dpp_i32<0xB1>(v);
    else if constexpr (Q == 1) return dpp_i32<0x4E>(v);
    else if constexpr (Q == 2) return dpp_i32<0x141>(v);
    else if constexpr (Q == 3) return dpp_i32<0x140>(v);
    else return (int)swap_partner_u32((uint32_t)v, Q == 5);
}
// Minimum over a lane group of the key (w, a, b, c), lexicographic; every
// lane ends with the group minimum (keys are distinct or equal in full).
template <int Q>
__device__ __forceinline__ void argmin_step(double &w, int &a, int &b, int &c) {
    const double w2 = partner_f64<Q>(w);
    const int a2 = partner_i32<Q>(a), b2 = partner_i32<Q>(b), c2 = partner_i32<Q>(c);
    const bool take = (w2 < w) || (w2 == w && (a2 < a || (a2 == a && (b2 < b || (b2 == b && c2 < c)))));
    if (take) { w = w2; a = a2; b = b2; c = c2; }
}
template <int L>
__device__ __forceinline__ void gargmin(double &w, int &a, int &b, int &c) {
    static_assert(L == 16 || L == 32 || L == 64, "lane groups of 16, 32 or 64");
    argmin_step<0>(w, a, b, c);
    argmin_step<1>(w, a, b, c);
    argmin_step<2>(w, a, b, c);
    argmin_step<3>(w, a, b, c);
    if constexpr (L >= 32) argmin_step<4>(w, a, b, c);
    if constexpr (L >= 64) argmin_step<5>(w, a, b, c);
}
// Minimum over a lane group of a double without NaNs, and of a uint32; every
// lane ends with the group minimum.
template <int L>
__device__ __forceinline__ double gmin_f64(double w) {
    w = fmin(w, partner_f64<0>(w));
    w = fmin(w, partner_f64<1>(w));
    w = fmin(w, partner_f64<2>(w));
    w = fmin(w, partner_f64<3>(w));
    if constexpr (L >= 32) w = fmin(w, partner_f64<4>(w));
    if constexpr (L >= 64) w = fmin(w, partner_f64<5>(w));
    return w;
}
template <int L>
__device__ __forceinline__ uint32_t gmin_u32(uint32_t k) {
    k = min(k, (uint32_t)partner_i32<0>((int)k));
    k = min(k, (uint32_t)partner_i32<1>((int)k));
    k = min(k, (uint32_t)partner_i32<2>((int)k));
    k = min(k, (uint32_t)partner_i32<3>((int)k));
    if constexpr (L >= 32) k = min(k, (uint32_t)partner_i32<4>((int)k));
    if constexpr (L >= 64) k = min(k, (uint32_t)partner_i32<5>((int)k));
    return k;
}
// Lane k's value in every lane (k uniform; group 0 starts at lane 0).
__device__ __forceinline__ int lane_i32(int v, int k) {
    return __builtin_amdgcn_readlane(v, __builtin_amdgcn_readfirstlane(k));
}
__device__ __forceinline__ double lane_f64(double v, int k) {
    const int kk = __builtin_amdgcn_readfirstlane(k);
    const uint64_t u = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, kk);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), kk);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

template <int L>
__device__ __forceinline__ int gor(int p) {
#pragma unroll
    for (int o = 1; o < L; o <<= 1) p |= __shfl_xor(p, o, L);
    return p;
}
template <int L>
__device__ __forceinline__ int gmaxi(int p) {
#pragma unroll
    for (int o = 1; o < L; o <<= 1) p = max(p, __shfl_xor(p, o, L));
    return p;
}
// max over the wave, NaN -> +inf
__device__ __forceinline__ double wave_max_inf(double v) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const double u = __shfl_xor(v, o, 64);
        v = (isnan(v) || isnan(u)) ? INFINITY : (u > v ? u : v);
    }
    return v;
}

// Orders the LDS traffic of one wave around a point where lanes read what
// other lanes of the same wave wrote (LDS operations of a wave complete in
// order; this keeps the compiler from moving them across).
__device__ __forceinline__ void wsync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ double w3(double ax, double ay, double az, double bx, double by, double bz) {
    const double dx = bx - ax, dy = by - ay, dz = bz - az;
    return (dx * dx + dy * dy) + dz * dz;   // built with -ffp-contract=off
}

// Strict edge order (w, min index, max index).
__device__ __forceinline__ bool key_less(double w1, int a1, int b1, double w2, int a2, int b2) {
    const int lo1 = min(a1, b1), hi1 = max(a1, b1), lo2 = min(a2, b2), hi2 = max(a2, b2);
    if (w1 != w2) return w1 < w2;
    if (lo1 != lo2) return lo1 < lo2;
    return hi1 < hi2;
}

// Root-relative tree sums by pointer jumping (Sec. 2.2 deconstruction):
// a[r] is the 2^r-th ancestor of the lane's body, R rounds cover every path.
template <int L>
struct Jumps {
    int a[6];
    int R;
    __device__ __forceinline__ void init(int par, int rounds) {
        R = rounds;
        a[0] = par;
#pragma unroll
        for (int r = 1; r < 6; ++r) {
            a[r] = -1;
            if (r < R) {
                const int p = a[r - 1];
                const int q = __shfl(p, p < 0 ? glane<L>() : p, L);
                a[r] = p < 0 ? -1 : q;
            }
        }
    }
    __device__ __forceinline__ d4 sum(const d4 &X) const {
        d4 s = a[0] < 0 ? d4{0.0, 0.0, 0.0, 0.0} : d4{X.x, X.y, X.z, 0.0};
#pragma unroll
        for (int r = 0; r < 6; ++r) {
            if (r < R) {
                const int p = a[r];
                const int src = p < 0 ? glane<L>() : p;
                const double sx = __shfl(s.x, src, L), sy = __shfl(s.y, src, L), sz = __shfl(s.z, src, L);
                if (p >= 0) {
                    s.x = s.x + sx;
                    s.y = s.y + sy;
                    s.z = s.z + sz;
                }
            }
        }
        return s;
    }
};

// ---------------------------------------------------------------- LDS state
template <int KF, int L, int G>
struct SysLDS {
    d4 X0[L], V0[L], a0[L];        // start-of-step MST edges (X, V) and accelerations
    d4 pos[G][L];                  // per group: current root-relative positions + mass
    d4 dXw[G][L];                  // per group: current edge increments (close pairs)
    double E[KF][6][L];            // per division: end increments of X, V; row 0 later holds the extrapolation
    double m[L];
    double tau[KF], drcm[KF][3];
    double t, B, H, U0, T0, M, rcm[3], vcm[3], t0, t_end, eps, h_next, h_last, epsw[4];
    int par[L], lev[L], opar[L], olev[L], coff[L + 1], cidx[L];
    int n, R, root, fresh, since_rebuild, halvings, approach, done, status, accepted;
    int64_t acc, rej, nforce, nrebuild, ntopo, time_iters;
};

// ---------------------------------------------------------------- MST (Prim)
// Prim's algorithm in one lane group on positions p (Sec. 3.2): root = body
// nearest the centre of mass (ties to the lower index), then repeatedly the
// smallest edge from the tree to a body outside it under the strict order.
// Writes par, lev, the children lists and the jump-round count R.
template <int KF, int L, int G>
__device__ __forceinline__ void group_prim(SysLDS<KF, L, G> &S, const d4 &p, int n) {
    // Runs in group 0 (lanes 0 .. L-1 of the first wave) only.
    const int i = glane<L>();
    const bool live = i < n;
    const double mi = live ? S.m[i] : 0.0;
    const double M = gsum<L>(mi);
    double cx = mi * p.x, cy = mi * p.y, cz = mi * p.z;
    gsum3<L>(cx, cy, cz);
    cx = cx / M;
    cy = cy / M;
    cz = cz / M;
    double wr = live ? w3(cx, cy, cz, p.x, p.y, p.z) : INFINITY;
    int root = live ? i : 0x7fffffff, z0 = 0, z1 = 0;
    gargmin<L>(wr, root, z0, z1);
    bool in = (i == root);
    int mypar = -1, mylev = 0;
    const double rx = lane_f64(p.x, root), ry = lane_f64(p.y, root), rz = lane_f64(p.z, root);
    double bw = (live && !in) ? w3(rx, ry, rz, p.x, p.y, p.z) : INFINITY;
    int bu = root;
    for (int step = 1; step < n; ++step) {
        // the smallest candidate edge under the strict order: first the
        // weight, then (min, max index) among the edges of that weight; the
        // edge's end outside the tree is the body added
        const bool cand = live && !in;
        const double wmin = gmin_f64<L>(cand ? bw : INFINITY);
        const uint32_t kk = (cand && bw == wmin) ? (((uint32_t)min(bu, i) << 16) | (uint32_t)max(bu, i)) : 0xffffffffu;
        const uint32_t kmin = gmin_u32<L>(kk);
        const int lo = (int)(kmin >> 16), hi = (int)(kmin & 0xffffu);
        const uint64_t inmask = __ballot(in ? 1 : 0);   // group 0 occupies lanes 0 .. L-1
        const int pick = ((inmask >> lo) & 1ull) ? hi : lo;
        const int pu = pick == lo ? hi : lo;
        const int plev = lane_i32(mylev, pu);
        if (i == pick) {
            in = true;
            mypar = pu;
            mylev = plev + 1;
        }
        const double qx = lane_f64(p.x, pick), qy = lane_f64(p.y, pick), qz = lane_f64(p.z, pick);
        if (live && !in) {
            const double w = w3(qx, qy, qz, p.x, p.y, p.z);
            if (key_less(w, pick, i, bw, bu, i)) { bw = w; bu = pick; }
        }
    }
    // children lists in ascending order
    int nchild = 0;
    for (int k = 0; k < n; ++k) nchild += (lane_i32(mypar, k) == i) ? 1 : 0;
    int incl = live ? nchild : 0;
#pragma unroll
    for (int o = 1; o < L; o <<= 1) {
        const int t = __shfl_up(incl, o, L);
        if (i >= o) incl += t;
    }
    int w = incl - nchild;
    for (int k = 0; k < n; ++k) {
        const bool mine = live && lane_i32(mypar, k) == i;
        if (mine) S.cidx[w++] = k;
    }
    const int maxlev = gmaxi<L>(live ? mylev : 0);
    if (live) {
        S.par[i] = mypar;
        S.lev[i] = mylev;
        S.coff[i] = incl - nchild;
    }
    if (i == n - 1) S.coff[n] = incl;
    if (i == 0) {
        int R = 0;
        while ((1 << R) < maxlev) ++R;
        S.R = R;
        S.root = root;
    }
}

// Separation of (i, j) under the close-pair rule of the tree (par, lev):
// MST path sum S_j - S_i (each accumulated top-down from the lowest common
// ancestor) within nd tree edges, else rj - ri (Sec. 3.4).
__device__ __forceinline__ d4 sep_rule(int i, int j, const int *par, const int *lev, const d4 *X, const d4 &ri, const d4 &rj, int nd) {
    if (i != j && nd > 0 && abs(lev[i] - lev[j]) <= nd) {
        int anc[4];
        int na = 0, u = i;
        for (int a = 0; a <= nd; ++a) {
            anc[na++] = u;
            if (par[u] < 0) break;
            u = par[u];
        }
        int w = j, fa = -1, fb = -1;
        for (int b = 0; b <= nd && fa < 0; ++b) {
            for (int a = 0; a < na && a + b <= nd; ++a)
                if (anc[a] == w) { fa = a; fb = b; break; }
            if (fa >= 0 || par[w] < 0) break;
            w = par[w];
        }
        if (fa >= 0) {
            d4 si{0.0, 0.0, 0.0, 0.0}, sj{0.0, 0.0, 0.0, 0.0};
            int pth[4];
            u = i;
            for (int s = 0; s < fa; ++s) { pth[s] = u; u = par[u]; }
            for (int s = fa - 1; s >= 0; --s) {
                const d4 x = X[pth[s]];
                si = d4{si.x + x.x, si.y + x.y, si.z + x.z, 0.0};
            }
            u = j;
            for (int s = 0; s < fb; ++s) { pth[s] = u; u = par[u]; }
            for (int s = fb - 1; s >= 0; --s) {
                const d4 x = X[pth[s]];
                sj = d4{sj.x + x.x, sj.y + x.y, sj.z + x.z, 0.0};
            }
            return d4{sj.x - si.x, sj.y - si.y, sj.z - si.z, 0.0};
        }
    }
    return d4{rj.x - ri.x, rj.y - ri.y, rj.z - ri.z, 0.0};
}

// ---------------------------------------------------------------- force
// Accelerations (without G) and phi of the lane's body from the group's
// positions pos[g][] (Sec. 2.1); pairs within nd <= 2 tree edges use the MST
// path sums of the current edges X0 + dXw[g] (Sec. 3.4).
template <int KF, int L, int G>
__device__ __forceinline__ void group_force(const SysLDS<KF, L, G> &S, int g, int n, int nd, const d4 &pi,
                                            double &ax, double &ay, double &az, double &ph) {
    const int i = glane<L>();
    const d4 *pos = S.pos[g];
    ax = ay = az = ph = 0.0;
    for (int j = 0; j < n; ++j) {
        const d4 pj = pos[j];
        const double dx = pj.x - pi.x, dy = pj.y - pi.y, dz = pj.z - pi.z;
        double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
        const bool self = (j == i);
        r2 = self ? 1.0 : r2;
        const double mj = self ? 0.0 : pj.w;
        const double y = rsqrt_f64(r2);
        const double mr = mj * y;
        const double s = mr * (y * y);
        ph = ph + mr;
        ax = fma(s, dx, ax);
        ay = fma(s, dy, ay);
        az = fma(s, dz, az);
    }
    if (nd <= 0 || i >= n) return;
    auto Xc = [&](int u) {
        const d4 a = S.X0[u], b = S.dXw[g][u];
        return d4{a.x + b.x, a.y + b.y, a.z + b.z, 0.0};
    };
    // replace the Cartesian term of a close pair by its path-sum term
    auto add = [&](double px, double py, double pz, int j) {
        const d4 pj = pos[j];
        double s1, mr1, s0, mr0;
        pair_terms(px, py, pz, pj.w, s1, mr1);
        const double cx = pj.x - pi.x, cy = pj.y - pi.y, cz = pj.z - pi.z;
        pair_terms(cx, cy, cz, pj.w, s0, mr0);
        ax = ax + fma(s1, px, -(s0 * cx));
        ay = ay + fma(s1, py, -(s0 * cy));
        az = az + fma(s1, pz, -(s0 * cz));
        ph = ph + (mr1 - mr0);
    };
    const int p = S.par[i];
    const d4 Xi = Xc(i);
    if (p >= 0) {
        add(-Xi.x, -Xi.y, -Xi.z, p);                                      // parent
        if (nd >= 2) {
            const int gp = S.par[p];
            if (gp >= 0) {
                const d4 Xp = Xc(p);
                add(-(Xp.x + Xi.x), -(Xp.y + Xi.y), -(Xp.z + Xi.z), gp);  // grandparent
            }
            for (int k = S.coff[p]; k < S.coff[p + 1]; ++k) {             // siblings
                const int c = S.cidx[k];
                if (c == i) continue;
                const d4 Xs = Xc(c);
                add(Xs.x - Xi.x, Xs.y - Xi.y, Xs.z - Xi.z, c);
            }
        }
    }
    for (int k = S.coff[i]; k < S.coff[i + 1]; ++k) {                     // children
        const int c = S.cidx[k];
        const d4 Xcc = Xc(c);
        add(Xcc.x, Xcc.y, Xcc.z, c);
        if (nd >= 2) {
            for (int q = S.coff[c]; q < S.coff[c + 1]; ++q) {             // grandchildren
                const int gc = S.cidx[q];
                const d4 Xg = Xc(gc);
                add(Xcc.x + Xg.x, Xcc.y + Xg.y, Xcc.z + Xg.z, gc);
            }
        }
    }
}

// Kinetic energy in the centre-of-mass frame of root-relative velocities u
// (Sec. 2.2: velocities are transformed back to the original frame).
template <int L>
__device__ __forceinline__ double group_T(const d4 &u, double mi, double M) {
    double bx = mi * u.x, by = mi * u.y, bz = mi * u.z;
    gsum3<L>(bx, by, bz);
    bx = bx / M;
    by = by / M;
    bz = bz / M;
    const double vx = u.x - bx, vy = u.y - by, vz = u.z - bz;
    return 0.5 * gsum<L>(mi * ((vx * vx + vy * vy) + vz * vz));
}

// Force at the start state by group 0: a0 (for S'(s0) of eq. gbs-criterion),
// U0 (end-time clip, Sec. 2.4) and T0.
template <int KF, int L, int G>
__device__ __forceinline__ void group_start(SysLDS<KF, L, G> &S, const BatchParams &P, int n) {
    const int i = glane<L>();
    const bool live = i < n;
    const int par = live ? S.par[i] : -1;
    const double mi = live ? S.m[i] : 0.0;
    Jumps<L> J;
    J.init(par, S.R);
    const d4 X0 = live ? S.X0[i] : d4{0.0, 0.0, 0.0, 0.0}, V0 = live ? S.V0[i] : d4{0.0, 0.0, 0.0, 0.0};
    const d4 rho = J.sum(X0);
    if (live) {
        S.pos[0][i] = d4{rho.x, rho.y, rho.z, mi};
        S.dXw[0][i] = d4{0.0, 0.0, 0.0, 0.0};
    }
    wsync();
    double ax, ay, az, ph;
    group_force(S, 0, n, P.n_d, d4{rho.x, rho.y, rho.z, mi}, ax, ay, az, ph);
    const double U = 0.5 * P.G * gsum<L>(live ? mi * ph : 0.0);
    if (live) S.a0[i] = d4{P.G * ax, P.G * ay, P.G * az, 0.0};
    const double T = group_T<L>(J.sum(V0), mi, S.M);
    wsync();
    if (i == 0) {
        S.U0 = U;
        S.T0 = T;
        S.nforce += 1;
    }
}

// New MST on the current positions (Sec. 3.5).  If the tree changed, the
// edge vector of each new edge is the separation the old tree gives for that
// pair under the close-pair rule.  Group 0.
template <int KF, int L, int G>
__device__ __forceinline__ void group_rebuild(SysLDS<KF, L, G> &S, const BatchParams &P, int n) {
    const int i = glane<L>();
    const bool live = i < n;
    const int par = live ? S.par[i] : -1;
    Jumps<L> J;
    J.init(par, S.R);
    const d4 X0 = live ? S.X0[i] : d4{0.0, 0.0, 0.0, 0.0}, V0 = live ? S.V0[i] : d4{0.0, 0.0, 0.0, 0.0};
    const d4 rho = J.sum(X0), ups = J.sum(V0);
    if (live) {
        S.opar[i] = par;
        S.olev[i] = S.lev[i];
        S.pos[0][i] = rho;    // old positions and velocities (group 0's buffers are free here)
        S.dXw[0][i] = ups;
    }
    wsync();
    group_prim(S, rho, n);
    wsync();
    const int changed = gor<L>((live && S.par[i] != par) ? 1 : 0);
    if (changed) {
        d4 nX{0.0, 0.0, 0.0, 0.0}, nV{0.0, 0.0, 0.0, 0.0};
        if (live) {
            const int q = S.par[i];
            if (q >= 0) {
                nX = sep_rule(q, i, S.opar, S.olev, S.X0, S.pos[0][q], S.pos[0][i], P.n_d);
                nV = sep_rule(q, i, S.opar, S.olev, S.V0, S.dXw[0][q], S.dXw[0][i], P.n_d);
            }
        }
        wsync();
        if (live) {
            S.X0[i] = nX;
            S.V0[i] = nV;
        }
    }
    wsync();
    if (i == 0) {
        S.nrebuild += 1;
        S.ntopo += changed ? 1 : 0;
    }
}

// Kicks of the pairs group g runs in one GBS step.
template <int KF, int G>
__device__ __forceinline__ int group_kicks(int g) {
    constexpr int NP = (KF + 1) / 2;
    int k = 0;
    for (int p = g; p < NP; p += G) k += 2 * (p + 1) + ((KF - 1 - p != p) ? 2 * (KF - p) : 0);
    return k;
}

// The divisions of group g over the step S.H: for each division n,
// D(h/2)[K(h)D(h)]^(n-1)K(h)D(h/2) with h = H/n from the start state
// (Sec. 2.3), as increments; end increments go to E[k], tau[k], drcm[k].
// The divisions of a group run as one flat loop of kicks so that all groups
// of a wave stay converged.
//
// Positions and velocities relative to the root are carried along with the
// edge increments instead of being re-summed from the edges at every
// substep: a drift adds dt V_e to every edge on a body's path, so the body
// moves by dt u (u = root-relative velocity), and a kick adds
// dt (a_v - a_parent) along the path, so u changes by dt (a - a_root).  They
// start each step from tree sums of the start state's edges.
template <int KF, int L, int G, bool COOP>
__device__ __forceinline__ void group_divisions(SysLDS<KF, L, G> &S, const BatchParams &P, int g, int n) {
    constexpr int NP = (KF + 1) / 2;
    const int i = glane<L>();
    const bool live = i < n;
    const int par = live ? S.par[i] : -1;
    const int root = S.root;
    const double mi = live ? S.m[i] : 0.0;
    const d4 X0 = live ? S.X0[i] : d4{0.0, 0.0, 0.0, 0.0}, V0 = live ? S.V0[i] : d4{0.0, 0.0, 0.0, 0.0};
    d4 r0, u0;
    {
        Jumps<L> J;
        J.init(par, S.R);
        r0 = J.sum(X0);
        u0 = J.sum(V0);
    }
    const double H = S.H, B = S.B, T0 = S.T0, M = S.M;
    const double vc0 = S.vcm[0], vc1 = S.vcm[1], vc2 = S.vcm[2];
    const double gd0 = P.alpha * (T0 + B) + P.gamma;
    const int kg = group_kicks<KF, G>(g);
    int kloop = kg;
    if (!COOP) {
        for (int gg = 0; gg < G; ++gg) kloop = max(kloop, group_kicks<KF, G>(gg));
    }
    int p = g, second = 0, k = g;
    int nsub = 2 * (k + 1), s = 0;
    double h = H / (double)nsub;
    d4 dX{0.0, 0.0, 0.0, 0.0}, dV{0.0, 0.0, 0.0, 0.0}, dr{0.0, 0.0, 0.0, 0.0}, du{0.0, 0.0, 0.0, 0.0};
    double tau = 0.0, dr0 = 0.0, dr1 = 0.0, dr2 = 0.0;
    // first half drift of a division: V = V0, so T = T0
    auto start = [&]() {
        const double dt = (0.5 * h) / gd0;
        dV = d4{0.0, 0.0, 0.0, 0.0};
        du = d4{0.0, 0.0, 0.0, 0.0};
        dX = par >= 0 ? d4{dt * V0.x, dt * V0.y, dt * V0.z, 0.0} : d4{0.0, 0.0, 0.0, 0.0};
        dr = d4{dt * u0.x, dt * u0.y, dt * u0.z, 0.0};
        tau = dt;
        dr0 = dt * vc0;
        dr1 = dt * vc1;
        dr2 = dt * vc2;
    };
    if (p < NP) start();
    for (int q = 0; q < kloop; ++q) {
        if (q < kg) {
            // kick K(h): forces at the current positions, U, velocity updates
            const d4 rho{r0.x + dr.x, r0.y + dr.y, r0.z + dr.z, 0.0};
            if (live) {
                S.pos[g][i] = d4{rho.x, rho.y, rho.z, mi};
                S.dXw[g][i] = dX;
            }
            wsync();
            double ax, ay, az, ph;
            group_force(S, g, n, P.n_d, d4{rho.x, rho.y, rho.z, mi}, ax, ay, az, ph);
            const double U = 0.5 * P.G * gsum<L>(live ? mi * ph : 0.0);
            ax = P.G * ax;
            ay = P.G * ay;
            az = P.G * az;
            const double dtk = h / (P.alpha * U + P.gamma);
            const int src = par < 0 ? i : par;
            const double bx = __shfl(ax, src, L), by = __shfl(ay, src, L), bz = __shfl(az, src, L);
            const double cx = __shfl(ax, root, L), cy = __shfl(ay, root, L), cz = __shfl(az, root, L);
            if (par >= 0) {
                dV = d4{dV.x + dtk * (ax - bx), dV.y + dtk * (ay - by), dV.z + dtk * (az - bz), 0.0};
                du = d4{du.x + dtk * (ax - cx), du.y + dtk * (ay - cy), du.z + dtk * (az - cz), 0.0};
            }
            wsync();
            ++s;
            const bool last = (s == nsub);
            // drift D(h) (D(h/2) at the end of the division)
            const d4 u{u0.x + du.x, u0.y + du.y, u0.z + du.z, 0.0};
            const double T = group_T<L>(live ? u : d4{0.0, 0.0, 0.0, 0.0}, mi, M);
            const double dtd = (last ? 0.5 * h : h) / (P.alpha * (T + B) + P.gamma);
            if (par >= 0) {
                dX = d4{dX.x + dtd * (V0.x + dV.x), dX.y + dtd * (V0.y + dV.y), dX.z + dtd * (V0.z + dV.z), 0.0};
                dr = d4{dr.x + dtd * u.x, dr.y + dtd * u.y, dr.z + dtd * u.z, 0.0};
            }
            tau = tau + dtd;
            dr0 = dr0 + dtd * vc0;
            dr1 = dr1 + dtd * vc1;
            dr2 = dr2 + dtd * vc2;
            if (last) {
                if (live) {
                    S.E[k][0][i] = dX.x;
                    S.E[k][1][i] = dX.y;
                    S.E[k][2][i] = dX.z;
                    S.E[k][3][i] = dV.x;
                    S.E[k][4][i] = dV.y;
                    S.E[k][5][i] = dV.z;
                }
                if (i == 0) {
                    S.tau[k] = tau;
                    S.drcm[k][0] = dr0;
                    S.drcm[k][1] = dr1;
                    S.drcm[k][2] = dr2;
                }
                if (second == 0 && KF - 1 - p != p) {
                    second = 1;
                    k = KF - 1 - p;
                } else {
                    second = 0;
                    p += G;
                    k = p;
                }
                if (p < NP) {
                    nsub = 2 * (k + 1);
                    s = 0;
                    h = H / (double)nsub;
                    start();
                }
            }
        }
    }
}

template <int KF>
__device__ __forceinline__ void neville(double (&p)[KF]) {
#pragma unroll
    for (int j = 1; j < KF; ++j) {
#pragma unroll
        for (int k = KF - 1; k >= j; --k) {
            const double r = (double)(2 * (k + 1)) / (double)(2 * (k - j + 1));
            const double den = r * r - 1.0;
            p[k] = p[k] + (p[k] - p[k - 1]) / den;
        }
    }
}

// |num| / |den| of one variable group (eq. gbs-criterion); non-finite -> inf.
__device__ __forceinline__ double gerr(double nx, double ny, double nz, double dx, double dy, double dz) {
    if (!isfinite(nx) || !isfinite(ny) || !isfinite(nz)) return INFINITY;
    const double dd = sqrt((dx * dx + dy * dy) + dz * dz);
    if (!(dd > 0.0)) return 0.0;
    const double e = sqrt((nx * nx + ny * ny) + nz * nz) / dd;
    return isnan(e) ? INFINITY : e;
}

// The same with the larger of two denominators (the centre-of-mass group: its
// value can start at the rounding level, so the end value is a scale too).
__device__ __forceinline__ double gerr2(double nx, double ny, double nz, double dx, double dy, double dz, double ex,
                                        double ey, double ez) {
    if (!isfinite(nx) || !isfinite(ny) || !isfinite(nz)) return INFINITY;
    double dd = sqrt((dx * dx + dy * dy) + dz * dz);
    const double de = sqrt((ex * ex + ey * ey) + ez * ez);
    if (de > dd) dd = de;
    if (!(dd > 0.0)) return 0.0;
    const double e = sqrt((nx * nx + ny * ny) + nz * nz) / dd;
    return isnan(e) ? INFINITY : e;
}

// Neville-Aitken extrapolation in h^2 of row b of E component c (or of the
// scalars t, r_cm when c < 0): returns T_{k,k} and sets *prev = T_{k-1,k-1}.
template <int KF>
__device__ __forceinline__ double extrap_one(const double *src, int stride, double *prev) {
    double p[KF];
#pragma unroll
    for (int k = 0; k < KF; ++k) p[k] = src[k * stride];
    neville<KF>(p);
    *prev = p[KF - 2];
    return p[KF - 1];
}

// Extrapolation of item `it` (X or V of one body, or the scalars t, r_cm);
// result to row 0 of E (or tau[0], drcm[0]); returns its error measure.
template <int KF, int L, int G>
__device__ __forceinline__ double extrap_item(SysLDS<KF, L, G> &S, int it, int n, double gd, double gk, double hn) {
    if (it < 2 * L) {
        const int b = it % L, c0 = it < L ? 0 : 3;
        if (b >= n) return 0.0;
        constexpr int stride = 6 * L;   // E[k][c][b] -> E[k+1][c][b]
        double qx, qy, qz;
        const double ex = extrap_one<KF>(&S.E[0][c0][b], stride, &qx);
        const double ey = extrap_one<KF>(&S.E[0][c0 + 1][b], stride, &qy);
        const double ez = extrap_one<KF>(&S.E[0][c0 + 2][b], stride, &qz);
        S.E[0][c0][b] = ex;
        S.E[0][c0 + 1][b] = ey;
        S.E[0][c0 + 2][b] = ez;
        const int q = S.par[b];
        if (q < 0) return 0.0;
        const double nx = ex - qx, ny = ey - qy, nz = ez - qz;
        if (c0 == 0) {
            const d4 X0 = S.X0[b], V0 = S.V0[b];
            return gerr(nx, ny, nz, X0.x + hn * (V0.x / gd), X0.y + hn * (V0.y / gd), X0.z + hn * (V0.z / gd));
        }
        const d4 V0 = S.V0[b], av = S.a0[b], ap = S.a0[q];
        return gerr(nx, ny, nz, V0.x + hn * ((av.x - ap.x) / gk), V0.y + hn * ((av.y - ap.y) / gk),
                    V0.z + hn * ((av.z - ap.z) / gk));
    }
    if (it == 2 * L) {
        double qt, q0, q1, q2;
        const double et_ = extrap_one<KF>(&S.tau[0], 1, &qt);
        const double e0 = extrap_one<KF>(&S.drcm[0][0], 3, &q0);
        const double e1 = extrap_one<KF>(&S.drcm[0][1], 3, &q1);
        const double e2 = extrap_one<KF>(&S.drcm[0][2], 3, &q2);
        const double et = gerr(et_ - qt, 0.0, 0.0, S.t + hn * (1.0 / gd), 0.0, 0.0);
        const double er = gerr2(e0 - q0, e1 - q1, e2 - q2, S.rcm[0] + hn * (S.vcm[0] / gd),
                                S.rcm[1] + hn * (S.vcm[1] / gd), S.rcm[2] + hn * (S.vcm[2] / gd), S.rcm[0] + e0,
                                S.rcm[1] + e1, S.rcm[2] + e2);
        S.tau[0] = et_;
        S.drcm[0][0] = e0;
        S.drcm[0][1] = e1;
        S.drcm[0][2] = e2;
        return et > er ? et : er;
    }
    return 0.0;
}

// ---------------------------------------------------------------- one system
// Integrates system `sys` from t0 to t_end.  COOP: the 4 waves of the
// workgroup (G = 4 groups of 64 lanes); otherwise one wave (G = 64 / L).
template <int KF, int L, int G, bool COOP>
__device__ __forceinline__ void run_system(SysLDS<KF, L, G> &S, const BatchArgs &A, int sys) {
    constexpr int NT = G * L;
    const int tid = COOP ? (int)threadIdx.x : (int)(threadIdx.x & 63);
    const int g = tid / L;
    const int i = tid % L;
    const BatchParams &P = A.p;
    auto sync = [&]() {
        if (COOP) __syncthreads();
        else wsync();
    };
    const int64_t o = A.off[sys];
    const int n = (int)(A.off[sys + 1] - o);
    // ---- set-up by group 0: load, validate, MST, edge vectors, COM, start force
    if (g == 0) {
        const bool live = i < n;
        double mi = 0.0;
        d4 x{0.0, 0.0, 0.0, 0.0}, v{0.0, 0.0, 0.0, 0.0};
        if (live) {
            mi = A.m[o + i];
            x = d4{A.x[3 * (o + i)], A.x[3 * (o + i) + 1], A.x[3 * (o + i) + 2], 0.0};
            v = d4{A.v[3 * (o + i)], A.v[3 * (o + i) + 1], A.v[3 * (o + i) + 2], 0.0};
            S.m[i] = mi;
        }
        const int bad_m = gor<L>((live && !(mi > 0.0 && isfinite(mi))) ? 1 : 0);
        const int bad_f = gor<L>((live && !(isfinite(x.x) && isfinite(x.y) && isfinite(x.z) && isfinite(v.x) &&
                                            isfinite(v.y) && isfinite(v.z)))
                                     ? 1
                                     : 0);
        int status = MSTAR_OK;
        if (n < 2 || n > L || bad_m) status = MSTAR_E_INVAL;
        else if (bad_f) status = MSTAR_E_NONFINITE;
        wsync();
        if (status == MSTAR_OK) {
            group_prim(S, x, n);
            wsync();
            const int par = live ? S.par[i] : -1;
            const int src = par < 0 ? i : par;
            const double xpx = __shfl(x.x, src, L), xpy = __shfl(x.y, src, L), xpz = __shfl(x.z, src, L);
            const double vpx = __shfl(v.x, src, L), vpy = __shfl(v.y, src, L), vpz = __shfl(v.z, src, L);
            if (live) {
                S.X0[i] = par < 0 ? d4{0.0, 0.0, 0.0, 0.0} : d4{x.x - xpx, x.y - xpy, x.z - xpz, 0.0};
                S.V0[i] = par < 0 ? d4{0.0, 0.0, 0.0, 0.0} : d4{v.x - vpx, v.y - vpy, v.z - vpz, 0.0};
            }
            const int zero = gor<L>((live && par >= 0 && w3(xpx, xpy, xpz, x.x, x.y, x.z) == 0.0) ? 1 : 0);
            const double M = gsum<L>(mi);
            double rc0 = mi * x.x, rc1 = mi * x.y, rc2 = mi * x.z;
            double vc0 = mi * v.x, vc1 = mi * v.y, vc2 = mi * v.z;
            gsum3<L>(rc0, rc1, rc2);
            gsum3<L>(vc0, vc1, vc2);
            if (zero) status = MSTAR_E_COINCIDENT;
            if (i == 0) {
                S.M = M;
                S.rcm[0] = rc0 / M;
                S.rcm[1] = rc1 / M;
                S.rcm[2] = rc2 / M;
                S.vcm[0] = vc0 / M;
                S.vcm[1] = vc1 / M;
                S.vcm[2] = vc2 / M;
            }
        }
        if (i == 0) {
            S.n = n;
            S.t0 = A.t0 ? A.t0[sys] : 0.0;
            S.t = S.t0;
            S.t_end = A.t_end[sys];
            S.acc = S.rej = S.nforce = S.nrebuild = S.ntopo = S.time_iters = 0;
            S.status = status;
            S.done = status != MSTAR_OK;
            S.eps = 0.0;
            S.h_next = 0.0;
            S.h_last = 0.0;
            S.since_rebuild = 0;
            S.halvings = 0;
            S.fresh = 0;
        }
        wsync();
        if (status == MSTAR_OK) {
            // one force evaluation gives B and the first step; the driver
            // counts a second one as the start evaluation of the first step,
            // which has the same value
            group_start(S, P, n);
            if (i == 0) {
                S.B = S.U0 - S.T0;
                const double gk = P.alpha * S.U0 + P.gamma;
                S.H = P.h_init > 0.0 ? P.h_init : P.q_first * gk * (S.t_end - S.t0);
                S.nforce += 1;
            }
        }
    }
    sync();
    // ---- GBS steps (Sec. 2.3, 2.4)
    for (;;) {
        if (g == 0) {
            if (i == 0 && !S.done && S.acc + S.rej >= P.max_steps) {
                S.status = MSTAR_E_MAXSTEPS;
                S.done = 1;
            }
            wsync();
            if (!S.done) {
                if (S.fresh) {
                    if (S.since_rebuild >= P.rebuild_every) {
                        group_rebuild(S, P, n);
                        if (i == 0) S.since_rebuild = 0;
                    }
                    wsync();
                    group_start(S, P, n);
                    if (i == 0) S.fresh = 0;
                }
                if (i == 0) {   // end-time clip with the force function at the step start
                    const double gk = P.alpha * S.U0 + P.gamma;
                    const double rem = S.t_end - S.t;
                    const double dt_est = S.H / gk;
                    S.approach = 0;
                    if (dt_est / rem > 1.0 || dt_est / rem < 0.0) {
                        S.H = gk * rem;
                        S.approach = 1;
                    }
                }
            }
        }
        sync();
        if (S.done) break;
        group_divisions<KF, L, G, COOP>(S, P, g, n);
        sync();
        // extrapolation and error measure
        {
            const double gd = P.alpha * (S.T0 + S.B) + P.gamma;
            const double gk = P.alpha * S.U0 + P.gamma;
            const double hn = S.H / (double)(2 * KF);
            double e = 0.0;
            for (int it = tid; it <= 2 * L; it += NT) {
                const double ei = extrap_item(S, it, n, gd, gk, hn);
                e = (isnan(e) || isnan(ei)) ? INFINITY : (ei > e ? ei : e);
            }
            e = wave_max_inf(e);
            if ((threadIdx.x & 63) == 0) S.epsw[COOP ? (threadIdx.x >> 6) : 0] = e;
        }
        sync();
        if (tid == 0) {
            double eps = 0.0;
            for (int w = 0; w < (COOP ? NT / 64 : 1); ++w) {
                const double ew = S.epsw[w];
                eps = (isnan(eps) || isnan(ew)) ? INFINITY : (ew > eps ? ew : eps);
            }
            S.eps = eps;
            S.accepted = eps <= P.eta;
            S.nforce += KF * (KF + 1);
        }
        sync();
        if (S.accepted) {   // state += extrapolated increments
            for (int it = tid; it <= 2 * L; it += NT) {
                if (it < 2 * L) {
                    const int b = it % L;
                    if (b < n) {
                        const int c0 = it < L ? 0 : 3;
                        d4 *Y = it < L ? S.X0 : S.V0;
                        const d4 y = Y[b];
                        Y[b] = d4{y.x + S.E[0][c0][b], y.y + S.E[0][c0 + 1][b], y.z + S.E[0][c0 + 2][b], 0.0};
                    }
                } else {
                    S.t = S.t + S.tau[0];
                    S.rcm[0] = S.rcm[0] + S.drcm[0][0];
                    S.rcm[1] = S.rcm[1] + S.drcm[0][1];
                    S.rcm[2] = S.rcm[2] + S.drcm[0][2];
                }
            }
        }
        sync();
        if (tid == 0) {   // step control (eq. hnext) and termination (Sec. 2.4)
            if (!S.accepted) {
                S.rej += 1;
                S.halvings += 1;
                S.H = 0.5 * S.H;
                if (S.halvings > P.max_halvings) {
                    S.status = MSTAR_E_NOCONV;
                    S.done = 1;
                }
            } else {
                S.acc += 1;
                S.h_last = S.H;
                if (A.hrec && S.acc <= A.hrec_cap) A.hrec[(size_t)sys * A.hrec_cap + (S.acc - 1)] = S.H;
                S.halvings = 0;
                S.since_rebuild += 1;
                S.fresh = 1;
                const double ee = S.eps > 1e-300 ? S.eps : 1e-300;
                double f = P.a_gbs * pow(P.eta / ee, 1.0 / (double)(2 * KF - 1));
                f = f < P.f_min ? P.f_min : (f > P.f_max ? P.f_max : f);
                S.h_next = S.H * f;
                S.H = S.h_next;
                if (S.approach) S.time_iters += 1;
                if (fabs(S.t_end - S.t) <= P.t_tol * fabs(S.t_end - S.t0)) {
                    S.status = MSTAR_OK;
                    S.done = 1;
                } else if (S.time_iters > P.max_time_iter) {
                    S.status = MSTAR_W_TIME_TOL;
                    S.done = 1;
                }
            }
        }
        sync();
    }
    // ---- output by group 0: Cartesian state (Sec. 2.2) and statistics
    if (g == 0) {
        const int st = S.status;
        const bool write = st == MSTAR_OK || st == MSTAR_W_TIME_TOL || st == MSTAR_E_NOCONV || st == MSTAR_E_MAXSTEPS;
        if (write) {
            const bool live = i < n;
            const int par = live ? S.par[i] : -1;
            Jumps<L> J;
            J.init(par, S.R);
            const d4 X0 = live ? S.X0[i] : d4{0.0, 0.0, 0.0, 0.0}, V0 = live ? S.V0[i] : d4{0.0, 0.0, 0.0, 0.0};
            const d4 rho = J.sum(X0), ups = J.sum(V0);
            const double mi = live ? S.m[i] : 0.0;
            const double M = S.M;
            double c0 = mi * rho.x, c1 = mi * rho.y, c2 = mi * rho.z;
            double u0 = mi * ups.x, u1 = mi * ups.y, u2 = mi * ups.z;
            gsum3<L>(c0, c1, c2);
            gsum3<L>(u0, u1, u2);
            c0 = c0 / M;
            c1 = c1 / M;
            c2 = c2 / M;
            u0 = u0 / M;
            u1 = u1 / M;
            u2 = u2 / M;
            if (live) {
                A.x[3 * (o + i)] = S.rcm[0] + (rho.x - c0);
                A.x[3 * (o + i) + 1] = S.rcm[1] + (rho.y - c1);
                A.x[3 * (o + i) + 2] = S.rcm[2] + (rho.z - c2);
                A.v[3 * (o + i)] = S.vcm[0] + (ups.x - u0);
                A.v[3 * (o + i) + 1] = S.vcm[1] + (ups.y - u1);
                A.v[3 * (o + i) + 2] = S.vcm[2] + (ups.z - u2);
            }
        }
        if (i == 0) {
            BatchStat r;
            r.status = st;
            r.reserved = 0;
            r.acc = S.acc;
            r.rej = S.rej;
            r.nforce = S.nforce;
            r.nrebuild = S.nrebuild;
            r.ntopo = S.ntopo;
            r.time_iters = S.time_iters;
            r.t_reached = S.t;
            r.eps_last = S.eps;
            r.h_next = S.h_next;
            r.h_last = S.h_last;
            A.stat[sys] = r;
        }
    }
    sync();
}

template <int KF>
constexpr size_t coop_bytes() { return sizeof(SysLDS<KF, 64, 4>); }
template <int KF, int WL>
constexpr size_t wave_bytes() {
    if constexpr (WL > 0) return 4 * sizeof(SysLDS<KF, WL, 64 / WL>);
    else return 0;
}
template <int KF, int WL>
constexpr size_t smem_bytes() { return coop_bytes<KF>() > wave_bytes<KF, WL>() ? coop_bytes<KF>() : wave_bytes<KF, WL>(); }

__global__ void k_batch_reset(int32_t *queue) {
    if (threadIdx.x < 2) queue[threadIdx.x] = 0;
}

// Persistent kernel: first the cooperative queue (one system per workgroup),
// then the wave queue (one system per wave).  Register use is capped for
// three resident waves per SIMD (three 256-thread workgroups per CU, which
// is also what the LDS of one cooperative system allows); measured faster
// than the uncapped two, the few spills sit outside the substep loop.
template <int KF, int WL>
__global__ __launch_bounds__(kBatchWG, 3) void k_batch(const BatchArgs *__restrict__ args) {
    const BatchArgs &A = *args;
    extern __shared__ __attribute__((aligned(32))) unsigned char smem[];
    __shared__ int next;
    if (A.n_coop > 0) {
        auto &S = *reinterpret_cast<SysLDS<KF, 64, 4> *>(smem);
        for (;;) {
            if (threadIdx.x == 0) {
                const int q = atomicAdd(&A.queue[0], 1);
                next = q < A.n_coop ? A.order[q] : -1;
            }
            __syncthreads();
            const int sys = next;
            __syncthreads();
            if (sys < 0) break;
            run_system<KF, 64, 4, true>(S, A, sys);
        }
    }
    if constexpr (WL > 0) {
        constexpr int G = 64 / WL;
        const int w = (int)(threadIdx.x >> 6);
        auto &S = *reinterpret_cast<SysLDS<KF, WL, G> *>(smem + (size_t)w * sizeof(SysLDS<KF, WL, G>));
        for (;;) {
            int q = 0;
            if ((threadIdx.x & 63) == 0) q = atomicAdd(&A.queue[1], 1);
            q = __shfl(q, 0, 64);
            const int sys = q < A.n_wave ? A.order[A.n_coop + q] : -1;
            if (sys < 0) break;
            run_system<KF, WL, G, false>(S, A, sys);
        }
    }
}

template <int KF, int WL>
int set_lds_limit() {
    static int done = 0;
    if (!done) {
        if (hipFuncSetAttribute((const void *)k_batch<KF, WL>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)smem_bytes<KF, WL>()) != hipSuccess)
            return -1;
        done = 1;
    }
    return 0;
}

template <int KF, int WL>
int launch_one(hipStream_t s, const BatchArgs *a, int nwg) {
    if (set_lds_limit<KF, WL>()) return -1;
    k_batch<KF, WL><<<nwg, kBatchWG, smem_bytes<KF, WL>(), s>>>(a);
    return 0;
}

template <int KF, int WL>
int blocks_one() {
    if (set_lds_limit<KF, WL>()) return 0;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batch<KF, WL>, kBatchWG, smem_bytes<KF, WL>()) != hipSuccess)
        return 0;
    return nb;
}

template <int KF>
int launch_kf(hipStream_t s, const BatchArgs *a, int wl, int nwg) {
    switch (wl) {
        case 0: return launch_one<KF, 0>(s, a, nwg);
        case 16: return launch_one<KF, 16>(s, a, nwg);
        case 32: return launch_one<KF, 32>(s, a, nwg);
        case 64: return launch_one<KF, 64>(s, a, nwg);
        default: return -1;
    }
}
template <int KF>
size_t bytes_kf(int wl) {
    switch (wl) {
        case 0: return smem_bytes<KF, 0>();
        case 16: return smem_bytes<KF, 16>();
        case 32: return smem_bytes<KF, 32>();
        case 64: return smem_bytes<KF, 64>();
        default: return 0;
    }
}
template <int KF>
int blocks_kf(int wl) {
    switch (wl) {
        case 0: return blocks_one<KF, 0>();
        case 16: return blocks_one<KF, 16>();
        case 32: return blocks_one<KF, 32>();
        case 64: return blocks_one<KF, 64>();
        default: return 0;
    }
}

}  // namespace

int launch_batch(hipStream_t s, const BatchArgs *a, int32_t *queue, int kf, int wave_lanes, int nwg) {
    if (nwg < 1) return -1;
    k_batch_reset<<<1, 64, 0, s>>>(queue);
    switch (kf) {
        case 2: return launch_kf<2>(s, a, wave_lanes, nwg);
        case 3: return launch_kf<3>(s, a, wave_lanes, nwg);
        case 4: return launch_kf<4>(s, a, wave_lanes, nwg);
        case 5: return launch_kf<5>(s, a, wave_lanes, nwg);
        case 6: return launch_kf<6>(s, a, wave_lanes, nwg);
        case 7: return launch_kf<7>(s, a, wave_lanes, nwg);
        case 8: return launch_kf<8>(s, a, wave_lanes, nwg);
        default: return -1;
    }
}

size_t batch_smem_bytes(int kf, int wave_lanes) {
    switch (kf) {
        case 2: return bytes_kf<2>(wave_lanes);
        case 3: return bytes_kf<3>(wave_lanes);
        case 4: return bytes_kf<4>(wave_lanes);
        case 5: return bytes_kf<5>(wave_lanes);
        case 6: return bytes_kf<6>(wave_lanes);
        case 7: return bytes_kf<7>(wave_lanes);
        case 8: return bytes_kf<8>(wave_lanes);
        default: return 0;
    }
}

int batch_blocks_per_cu(int kf, int wave_lanes) {
    switch (kf) {
        case 2: return blocks_kf<2>(wave_lanes);
        case 3: return blocks_kf<3>(wave_lanes);
        case 4: return blocks_kf<4>(wave_lanes);
        case 5: return blocks_kf<5>(wave_lanes);
        case 6: return blocks_kf<6>(wave_lanes);
        case 7: return blocks_kf<7>(wave_lanes);
        case 8: return blocks_kf<8>(wave_lanes);
        default: return 0;
    }
}

}  // namespace mstar
