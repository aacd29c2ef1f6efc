// O(N^2) FP64 force / force-function kernel with MST close-pair separations
// (paper Sec. 2.1 equations of motion, Sec. 3.4 close-pair rule, Sec. 4.1
// force loop).
//
// Layout: positions are 32-byte records {x, y, z, m} in the centre-of-mass
// frame, one array per division slot.  One workgroup = kForceWaves waves
// sharing the same 64 i-bodies (one per lane) and splitting the workgroup's
// j-range between them; the j-body of each iteration is wave-uniform and is fetched with a
// scalar load straight into SGPRs, so the inner loop is pure FP64 VALU work
// with no LDS traffic.  Partial sums of the waves are combined in LDS
// in fixed order; j-splits across workgroups are combined later in fixed
// order, so results are bitwise reproducible.
//
// Close pairs (tree distance <= N_d, any N_d up to kMaxNd): the main loop uses Cartesian
// differences for every pair; one extra workgroup per i-block (grid row
// y = 0, dispatched first) computes, for each close pair, the term built from
// the MST path sum minus the Cartesian term (same operation sequence as the
// main loop, so the subtracted term is the one that was added) into a partial
// of its own.  These correction blocks are short and run beside the j-loop
// blocks instead of lengthening one of them.
//
// With the TTL function of Sec. 2.1 switched on (template flag OM), the same
// pass also accumulates Omega = G/2 sum_i mo_i sum_j mo_j/r_ij and
// grad_i Omega = G mo_i sum_j mo_j d_ij/r_ij^3 over the Omega masses mo, into
// partials of their own; r^-1 is shared with the Newtonian terms.
#include "common.h"

namespace mstar {

struct ForceArgs {
    const d4 *P;           // [slot][n] positions + mass
    d4 *part;              // [slot][nsplit_max][n] partial (ax, ay, az, phi)
    double *Upart;         // [slot][nib * nsplit_max] partial sum_i m_i phi_i
    const d4 *X0, *dX;     // MST edge vectors: current = X0 + dX[slot]
    const int32_t *parent, *child_off, *child_idx;
    int n, nib, nib_alloc, nsplit, nsplit_max, jchunk;   // nib: force i-blocks of 64*IPL bodies
    int nparts;            // partials per i-block: nsplit j-splits (+1 correction block when N_d > 0)
    int nd;                // closeness N_d of eq. LCA (0 .. kMaxNd)
    const double *mo;      // [n] Omega masses (OM only)
    d4 *opart;             // [slot][nsplit_max][n] partial (Omega gradient sums, Omega potential)
    double *Opart;         // [slot][nib * nsplit_max] partial sum_i mo_i (sum_j mo_j / r)
    SlotList sl;
};

// Per-lane sums: Newtonian (a, phi) and, with OM, the Omega analogues (o, po).
struct Sums {
    double ax, ay, az, ph, ox, oy, oz, po;
};

// 1/|d| for one separation, the first half of the pair term.
__device__ __forceinline__ double pair_y(double dx, double dy, double dz) {
    return rsqrt_f64(fma(dz, dz, fma(dy, dy, dx * dx)));
}

// Close pair: add the term of the path-sum separation dp and subtract the
// term of the Cartesian separation the main loop used, each formed by the
// main loop's operation sequence (mr = m y, s = mr y^2).
// MUT: the term as the mutual kernel forms it (s = m (y^2 y)) instead of the
// pairwise kernel's (s = (m y) y^2).
template <bool OM, bool MUT = false>
__device__ __forceinline__ void add_close(double dpx, double dpy, double dpz, const d4 &pi, const d4 &pj,
                                          double moj, Sums &c) {
    const double cx = pj.x - pi.x, cy = pj.y - pi.y, cz = pj.z - pi.z;
    const double y1 = pair_y(dpx, dpy, dpz), y0 = pair_y(cx, cy, cz);
    const double q1 = y1 * y1, q0 = y0 * y0;
    const double mr1 = pj.w * y1, mr0 = pj.w * y0;
    const double s1 = MUT ? pj.w * (q1 * y1) : mr1 * q1, s0 = MUT ? pj.w * (q0 * y0) : mr0 * q0;
    c.ax = c.ax + fma(s1, dpx, -(s0 * cx));
    c.ay = c.ay + fma(s1, dpy, -(s0 * cy));
    c.az = c.az + fma(s1, dpz, -(s0 * cz));
    c.ph = c.ph + (mr1 - mr0);
    if constexpr (OM) {
        const double o1 = moj * y1, o0 = moj * y0;
        const double t1 = o1 * q1, t0 = o0 * q0;
        c.ox = c.ox + fma(t1, dpx, -(t0 * cx));
        c.oy = c.oy + fma(t1, dpy, -(t0 * cy));
        c.oz = c.oz + fma(t1, dpz, -(t0 * cz));
        c.po = c.po + (o1 - o0);
    }
}

__device__ __forceinline__ d4 cur_edge(const d4 *X0, const d4 *dX, int u) {
    const d4 a = X0[u], b = dX[u];
    return d4{a.x + b.x, a.y + b.y, a.z + b.z, 0.0};
}

// Top-down sum of the edge vectors on the path from the ancestor `a` levels
// above v down to v (the vector from that ancestor to v).
__device__ __forceinline__ d4 path_down(int v, int a, const int32_t *parent, const d4 *X0, const d4 *dX) {
    int pth[kMaxNd];
    int u = v;
    for (int s = 0; s < a; ++s) {
        pth[s] = u;
        u = parent[u];
    }
    d4 S{0.0, 0.0, 0.0, 0.0};
    for (int s = a - 1; s >= 0; --s) {
        const d4 x = cur_edge(X0, dX, pth[s]);
        S = d4{S.x + x.x, S.y + x.y, S.z + x.z, 0.0};
    }
    return S;
}

// Replace the Cartesian terms of all pairs (i, j) within nd tree edges
// (eq. LCA) by the MST path-sum terms, d_ij = S_j - S_i with S_v the
// top-down sum of edge vectors from the lowest common ancestor to v.  For
// every ancestor A of i up to nd levels above it (A = i included), the pairs
// whose lowest common ancestor is A: A itself, and A's descendants at most
// nd - a levels below it outside the branch that holds i (depth-first, the
// path sum of each descendant built from its parent's).
template <bool GENERIC, bool OM, bool MUT = false>
__device__ void close_correction(int i, int nd, const d4 *P, const double *mo, const d4 *X0, const d4 *dX,
                                 const int32_t *parent, const int32_t *coff, const int32_t *cidx, Sums &c) {
    const d4 pi = P[i];
    auto mom = [&](int j) { return OM ? mo[j] : 0.0; };
    if constexpr (!GENERIC) {
        // the N_d <= 2 neighbourhood written out (same separations as the
        // general walk below, with shorter chains of dependent loads)
        const int p = parent[i];
        if (p >= 0) {
            const d4 Xi = cur_edge(X0, dX, i);
            add_close<OM, MUT>(0.0 - Xi.x, 0.0 - Xi.y, 0.0 - Xi.z, pi, P[p], mom(p), c);          // parent
            if (nd >= 2) {
                const int g = parent[p];
                if (g >= 0) {
                    const d4 Xp = cur_edge(X0, dX, p);
                    const d4 S{Xp.x + Xi.x, Xp.y + Xi.y, Xp.z + Xi.z, 0.0};
                    add_close<OM, MUT>(0.0 - S.x, 0.0 - S.y, 0.0 - S.z, pi, P[g], mom(g), c);      // grandparent
                }
                for (int k = coff[p]; k < coff[p + 1]; ++k) {                                // siblings
                    const int q = cidx[k];
                    if (q == i) continue;
                    const d4 Xs = cur_edge(X0, dX, q);
                    add_close<OM, MUT>(Xs.x - Xi.x, Xs.y - Xi.y, Xs.z - Xi.z, pi, P[q], mom(q), c);
                }
            }
        }
        for (int k = coff[i]; k < coff[i + 1]; ++k) {                                        // children
            const int q = cidx[k];
            const d4 Xc = cur_edge(X0, dX, q);
            add_close<OM, MUT>(Xc.x, Xc.y, Xc.z, pi, P[q], mom(q), c);
            if (nd >= 2) {
                for (int r = coff[q]; r < coff[q + 1]; ++r) {                                // grandchildren
                    const int gc = cidx[r];
                    const d4 Xg = cur_edge(X0, dX, gc);
                    add_close<OM, MUT>(Xc.x + Xg.x, Xc.y + Xg.y, Xc.z + Xg.z, pi, P[gc], mom(gc), c);
                }
            }
        }
    } else {
        int anc = i, below = -1;
        for (int a = 0; a <= nd; ++a) {
            if (a > 0) {
                below = anc;
                anc = parent[anc];
                if (anc < 0) break;
            }
            const d4 Si = path_down(i, a, parent, X0, dX);
            if (a > 0) add_close<OM, MUT>(0.0 - Si.x, 0.0 - Si.y, 0.0 - Si.z, pi, P[anc], mom(anc), c);
            const int bmax = nd - a;
            if (bmax < 1) continue;
            int sk[kMaxNd], se[kMaxNd];
            d4 sS[kMaxNd];
            int top = 0;
            sk[0] = coff[anc];
            se[0] = coff[anc + 1];
            sS[0] = d4{0.0, 0.0, 0.0, 0.0};
            while (top >= 0) {
                if (sk[top] == se[top]) {
                    --top;
                    continue;
                }
                const int ch = cidx[sk[top]++];
                if (top == 0 && ch == below) continue;
                const d4 x = cur_edge(X0, dX, ch);
                const d4 Sc{sS[top].x + x.x, sS[top].y + x.y, sS[top].z + x.z, 0.0};
                add_close<OM, MUT>(Sc.x - Si.x, Sc.y - Si.y, Sc.z - Si.z, pi, P[ch], mom(ch), c);
                if (top + 1 < bmax) {   // ch's children are within nd
                    ++top;
                    sk[top] = coff[ch];
                    se[top] = coff[ch + 1];
                    sS[top] = Sc;
                }
            }
        }
    }
}

// Inner loop over j in [jb, je) for the IPL i-bodies of each lane; GUARD
// masks the self pair (only the diagonal block needs it).  With OM the Omega
// sums ride along on the same 1/r.
template <bool GUARD, int IPL, bool OM>
__device__ __forceinline__ void j_loop(const d4 *__restrict__ P, const double *__restrict__ mo, int jb, int je,
                                       const int (&ii)[IPL], const d4 (&pi)[IPL], Sums (&c)[IPL]) {
#pragma unroll 8
    for (int j = jb; j < je; ++j) {
        const d4 pj = P[j];
        const double moj = OM ? mo[j] : 0.0;
#pragma unroll
        for (int q = 0; q < IPL; ++q) {
            const double dx = pj.x - pi[q].x, dy = pj.y - pi[q].y, dz = pj.z - pi[q].z;
            double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
            double mj = pj.w, mq = moj;
            if (GUARD) {
                const bool self = (j == ii[q]);
                r2 = self ? 1.0 : r2;
                mj = self ? 0.0 : mj;
                mq = self ? 0.0 : mq;
            }
            const double y = rsqrt_f64(r2);
            const double yy = y * y;
            const double mr = mj * y;
            const double s = mr * yy;
            c[q].ph = c[q].ph + mr;
            c[q].ax = fma(s, dx, c[q].ax);
            c[q].ay = fma(s, dy, c[q].ay);
            c[q].az = fma(s, dz, c[q].az);
            if constexpr (OM) {
                const double o = mq * y;
                const double so = o * yy;
                c[q].po = c[q].po + o;
                c[q].ox = fma(so, dx, c[q].ox);
                c[q].oy = fma(so, dy, c[q].oy);
                c[q].oz = fma(so, dz, c[q].oz);
            }
        }
    }
}

// CK: 0 no close pairs (N_d = 0), 1 the written-out N_d <= 2 rule, 2 the
// general walk for N_d up to kMaxNd (its own instance, so that the stack it
// needs does not cost the common instances registers).
template <int CK, int NW, int IPL, bool OM>
__global__ __launch_bounds__(64 * NW) void k_force(ForceArgs a) {
    constexpr bool CLOSE = CK > 0;
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int ib = blockIdx.x % a.nib;
    const int slot = a.sl.slot[blockIdx.x / a.nib];
    const int part = blockIdx.y;                          // partial index
    const int split = CLOSE ? part - 1 : part;             // j-split index (-1: correction block)
    const int n = a.n;
    const d4 *__restrict__ P = a.P + (size_t)slot * n;
    const size_t prow = ((size_t)slot * a.nsplit_max + part) * n;
    const size_t urow = (size_t)slot * a.nib_alloc * a.nsplit_max + (size_t)ib * a.nparts + part;
    const int i0 = ib * 64 * IPL;
    int ii[IPL];
    d4 pi[IPL];
    Sums c[IPL];
#pragma unroll
    for (int q = 0; q < IPL; ++q) {
        const int i = i0 + q * 64 + lane;
        ii[q] = i < n ? i : n - 1;
        pi[q] = P[ii[q]];
        c[q] = Sums{0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    }
    double u = 0.0, uo = 0.0;
    if (CLOSE && split < 0) {   // close-pair correction block (wave 0)
        if (wv != 0) return;
#pragma unroll
        for (int q = 0; q < IPL; ++q) {
            const int i = i0 + q * 64 + lane;
            if (i < n) {
                close_correction<CK == 2, OM>(i, a.nd, P, a.mo, a.X0, a.dX + (size_t)slot * n, a.parent, a.child_off,
                                     a.child_idx, c[q]);
                a.part[prow + i] = d4{c[q].ax, c[q].ay, c[q].az, c[q].ph};
                u = u + pi[q].w * c[q].ph;
                if constexpr (OM) {
                    a.opart[prow + i] = d4{c[q].ox, c[q].oy, c[q].oz, c[q].po};
                    uo = uo + a.mo[i] * c[q].po;
                }
            }
        }
    } else {
        const int j0 = split * a.jchunk;
        const int j1 = min(n, j0 + a.jchunk);
        const int qw = (max(j1 - j0, 0) + NW - 1) / NW;
        int jb = min(j1, j0 + wv * qw);
        int je = min(j1, jb + qw);
        jb = __builtin_amdgcn_readfirstlane(jb);
        je = __builtin_amdgcn_readfirstlane(je);
        const int g0 = __builtin_amdgcn_readfirstlane(max(jb, i0));
        const int g1 = __builtin_amdgcn_readfirstlane(min(je, i0 + 64 * IPL));
        if (g0 < g1) {
            j_loop<false, IPL, OM>(P, a.mo, jb, g0, ii, pi, c);
            j_loop<true, IPL, OM>(P, a.mo, g0, g1, ii, pi, c);
            j_loop<false, IPL, OM>(P, a.mo, g1, je, ii, pi, c);
        } else {
            j_loop<false, IPL, OM>(P, a.mo, jb, je, ii, pi, c);
        }
        __shared__ d4 red[NW][IPL][64];
#pragma unroll
        for (int q = 0; q < IPL; ++q) red[wv][q][lane] = d4{c[q].ax, c[q].ay, c[q].az, c[q].ph};
        if constexpr (OM) {
            __shared__ d4 ored[NW][IPL][64];
#pragma unroll
            for (int q = 0; q < IPL; ++q) ored[wv][q][lane] = d4{c[q].ox, c[q].oy, c[q].oz, c[q].po};
            __syncthreads();
            if (wv != 0) return;
#pragma unroll
            for (int q = 0; q < IPL; ++q) {
                const int i = i0 + q * 64 + lane;
                d4 t = ored[0][q][lane];
                for (int w = 1; w < NW; ++w) {
                    const d4 e = ored[w][q][lane];
                    t.x = t.x + e.x; t.y = t.y + e.y; t.z = t.z + e.z; t.w = t.w + e.w;
                }
                if (i < n) {
                    a.opart[prow + i] = t;
                    uo = uo + a.mo[i] * t.w;
                }
            }
        } else {
            __syncthreads();
            if (wv != 0) return;
        }
#pragma unroll
        for (int q = 0; q < IPL; ++q) {
            const int i = i0 + q * 64 + lane;
            d4 t = red[0][q][lane];
            for (int w = 1; w < NW; ++w) {
                const d4 e = red[w][q][lane];
                t.x = t.x + e.x; t.y = t.y + e.y; t.z = t.z + e.z; t.w = t.w + e.w;
            }
            if (i < n) {
                a.part[prow + i] = t;
                u = u + pi[q].w * t.w;
            }
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) u = u + __shfl_xor(u, off, 64);
    if (lane == 0) a.Upart[urow] = u;
    if constexpr (OM) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) uo = uo + __shfl_xor(uo, off, 64);
        if (lane == 0) a.Opart[urow] = uo;
    }
}

int force_blocks_per_cu(int nd) {
    constexpr int NW = kForceWaves, IPL = kForceIPL;
    int nb = 0;
    hipError_t e;
    if (nd <= 0) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_force<0, NW, IPL, false>, 64 * NW, 0);
    else if (nd <= 2) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_force<1, NW, IPL, false>, 64 * NW, 0);
    else e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_force<2, NW, IPL, false>, 64 * NW, 0);
    return e == hipSuccess && nb > 0 ? nb : 1;
}

// ------------------------------------------------------------------------
// Mutual kernel: every unordered pair (i, j) once, its term applied to both
// bodies with opposite signs (Newton's third law; the 1/sqrt and r^-3 of a
// pair are formed once instead of twice).
//
// A wave holds 64 kMutIPL i-bodies in registers (a "row": lane l holds bodies
// row*64 kMutIPL + q*64 + l, q < kMutIPL) and streams 64-body j-blocks
// through LDS.  At step o, lane l pairs its i-bodies with j-body (l + o) mod
// 64 (the j-block is stored twice in LDS so the index l + o needs no wrap):
// the 64 lanes touch 64 different j-bodies, so the j-side sums go into LDS
// with atomic adds that never collide within an instruction and, the
// instructions of one wave being ordered, always add up in the same order.
// Row P pairs with j-blocks J >= kMutIPL P; on the diagonal j-blocks
// (J = kMutIPL P + q) i-block q takes only the offsets 1..32 (the pairs
// inside one block, each once; at offset 32 only lanes 0..31), and i-blocks
// q > J - kMutIPL P skip the block (those pairs come with i-block J's row
// position).  Bodies beyond n are padded far away (i at +1e50, j at -1e50)
// with zero mass, so they add exact zeros and never make r = 0.
//
// Work split: the steps of all evaluations of the launch form one sequence
// (eval, row, j-block, step) and wave w takes steps [w L, (w + 1) L): every
// wave does the same work, whatever the row lengths (the triangle) and the
// number of evaluations.  Outputs (FLay): per wave and row it touches, the
// i-side sums of the row's bodies and the wave's share of sum m_i m_j / r;
// per j-block, the j-side sums (two pieces when the block was cut between two
// waves).  Close pairs: one extra wave per 64 bodies and evaluation forms the
// path-sum terms minus the Cartesian terms, as in the pairwise kernel.
struct MutArgs {
    const d4 *P;                  // [slot][n]
    d3 *ip, *jp;                  // FLay outputs (Dev::mip, mjp)
    d4 *cp;                       // Dev::mcp
    double *up;                   // Dev::mup
    size_t ip_s, jp_s, up_s;
    const d4 *X0, *dX;
    const int32_t *parent, *child_off, *child_idx;
    FLay f;
    int n, nd, ncb;               // ncb: close-pair correction waves (nact * nb when N_d > 0)
    int nwaves;                   // pair-work waves
    long long total;              // steps of the launch (nact * f.Ec)
    SlotList sl;
};

constexpr double kPadFar = 1e50;   // padding distance: r^2 ~ 1e100 stays far from overflow

template <int IPL>
__device__ __forceinline__ void mut_flush(const MutArgs &a, int slot, int ea, int P, int w, int lane, const double *ax,
                                          const double *ay, const double *az, const double *ph, const double *mi) {
    const FLay &f = a.f;
    const long long base = (long long)ea * f.Ec;
    const long long wf = (base + mut_rs(f, P)) / f.L, wl = (base + mut_rs(f, P + 1) - 1) / f.L;
    const int widx = (int)(w - wf), last = (int)(wl - wf);
    d3 *ip = a.ip + (size_t)slot * a.ip_s + ((size_t)P * f.maxw + widx) * (64 * IPL);
    double u = 0.0;
#pragma unroll
    for (int q = 0; q < IPL; ++q) {
        const int i = 64 * IPL * P + 64 * q + lane;
        if (i < a.n) ip[64 * q + lane] = d3{ax[q], ay[q], az[q]};
        u = u + mi[q] * ph[q];
    }
    u = wave_sum(u);
    double *up = a.up + (size_t)slot * a.up_s + (size_t)P * f.maxw;
    // each unordered pair once: twice its share, so that U = G/2 sum of the partials
    if (lane == 0) up[widx] = 2.0 * u;
    if (widx == last)   // the row's last wave clears the unused slots of the row
        for (int k = widx + 1 + lane; k < f.maxw; k += 64) up[k] = 0.0;
}

// One step of the pair loop: lane l's i-bodies q (active mask qm, wave
// uniform) with j-body k = l + o of the LDS block, whose position and mass
// (xj, yj, zj, mj0) the caller has read; hq: the i-block whose diagonal offset
// 32 is being done (only lanes 0..31 count), or -1.
template <int IPL>
__device__ __forceinline__ void mut_step(int k, int qm, int hq, bool hi_lane, double xj, double yj, double zj,
                                         double mj0, double *AX, double *AY, double *AZ, const double *xi,
                                         const double *yi, const double *zi, const double *mi, double *ax, double *ay,
                                         double *az, double *ph) {
    double jx = 0.0, jy = 0.0, jz = 0.0;
    bool first = true;
#pragma unroll
    for (int q = 0; q < IPL; ++q) {
        if (!(qm & (1 << q))) continue;
        const bool off = (q == hq) && hi_lane;
        const double mj = off ? 0.0 : mj0, mq = off ? 0.0 : mi[q];
        const double dx = xj - xi[q], dy = yj - yi[q], dz = zj - zi[q];
        const double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
        const double y = rsqrt_f64(r2);
        const double y3 = (y * y) * y;
        const double sj = mj * y3, si = mq * y3;
        ph[q] = fma(mj, y, ph[q]);
        ax[q] = fma(sj, dx, ax[q]);
        ay[q] = fma(sj, dy, ay[q]);
        az[q] = fma(sj, dz, az[q]);
        if (first) {
            jx = -(si * dx); jy = -(si * dy); jz = -(si * dz);
            first = false;
        } else {
            jx = fma(-si, dx, jx); jy = fma(-si, dy, jy); jz = fma(-si, dz, jz);
        }
    }
    if (!first) {
        atomicAdd(&AX[k], jx);
        atomicAdd(&AY[k], jy);
        atomicAdd(&AZ[k], jz);
    }
}

// The same step with the j-side sums (jx, jy, jz) kept in registers: lane l
// holds the running sums of j-body (l + o) mod 64, adds its pair terms, then
// takes lane l + 1's sums (a rotation of the wave by one lane), which belong
// to its j-body of the next step.  Each j-body's sums thus collect their
// terms in step order, as with the LDS sums, without LDS atomics.
__device__ __forceinline__ double rot1(double v) {   // DPP wave_rol:1, lane l <- lane (l + 1) mod 64
    const unsigned long long u = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)u, 0x134, 0xF, 0xF, false);
    const unsigned hi = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)(u >> 32), 0x134, 0xF, 0xF, false);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

template <int IPL>
__device__ __forceinline__ void mut_step_r(int qm, int hq, bool hi_lane, double xj, double yj, double zj, double mj0,
                                           double &jx, double &jy, double &jz, const double *xi, const double *yi,
                                           const double *zi, const double *mi, double *ax, double *ay, double *az,
                                           double *ph) {
#pragma unroll
    for (int q = 0; q < IPL; ++q) {
        if (!(qm & (1 << q))) continue;
        const bool off = (q == hq) && hi_lane;
        const double mj = off ? 0.0 : mj0, mq = off ? 0.0 : mi[q];
        const double dx = xj - xi[q], dy = yj - yi[q], dz = zj - zi[q];
        const double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
        const double y = rsqrt_f64(r2);
        const double y3 = (y * y) * y;
        const double sj = mj * y3, si = mq * y3;
        ph[q] = fma(mj, y, ph[q]);
        ax[q] = fma(sj, dx, ax[q]);
        ay[q] = fma(sj, dy, ay[q]);
        az[q] = fma(sj, dz, az[q]);
        jx = fma(-si, dx, jx);
        jy = fma(-si, dy, jy);
        jz = fma(-si, dz, jz);
    }
    jx = rot1(jx);
    jy = rot1(jy);
    jz = rot1(jz);
}

// Position of step g in the launch's step sequence.
struct MutUnit {
    int ea, P, J, s, se;
};
__device__ __forceinline__ MutUnit mut_locate(const FLay &f, int ipl, long long g, long long gend) {
    MutUnit u;
    u.ea = (int)(g / f.Ec);
    const long long r = g - (long long)u.ea * f.Ec;
    int lo = 0, hi = f.npr - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (mut_rs(f, mid) <= r) lo = mid;
        else hi = mid - 1;
    }
    u.P = lo;
    const long long rr = r - mut_rs(f, lo);
    if (rr < 32) { u.J = ipl * lo; u.s = (int)rr; }
    else { u.J = ipl * lo + 1 + (int)((rr - 32) / 64); u.s = (int)((rr - 32) % 64); }
    u.se = (int)min((long long)mut_cost(f, u.P, u.J), (long long)u.s + (gend - g));
    return u;
}

// Close-pair correction of the 64 bodies of block ib of evaluation ea.
__device__ __forceinline__ void mut_close_block(const MutArgs &a, int c, int lane) {
    const int ea = c / a.f.nb, ib = c % a.f.nb;
    const int slot = a.sl.slot[ea];
    const d4 *P = a.P + (size_t)slot * a.n;
    const int i = 64 * ib + lane;
    double u = 0.0;
    if (i < a.n) {
        Sums cs{0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        close_correction<false, false, true>(i, a.nd, P, nullptr, a.X0, a.dX + (size_t)slot * a.n, a.parent,
                                             a.child_off, a.child_idx, cs);
        a.cp[(size_t)slot * a.n + i] = d4{cs.ax, cs.ay, cs.az, 0.0};
        u = P[i].w * cs.ph;
    }
    u = wave_sum(u);
    if (lane == 0) a.up[(size_t)slot * a.up_s + (size_t)a.f.npr * a.f.maxw + ib] = u;
}

template <int IPL, bool JREG>
__global__ __launch_bounds__(64) void k_force_mut(MutArgs a) {
    const int lane = threadIdx.x;
    const int w = blockIdx.x;
    // the close-pair correction blocks, spread evenly over the waves (before
    // their pair work, so that their scattered loads overlap other waves' work)
    for (int c = (int)((long long)w * a.ncb / a.nwaves); c < (int)((long long)(w + 1) * a.ncb / a.nwaves); ++c)
        mut_close_block(a, c, lane);
    __shared__ double JX[128], JY[128], JZ[128], JM[128], AX[128], AY[128], AZ[128];
    const FLay f = a.f;
    long long g = (long long)w * f.L;
    const long long gend = min(g + f.L, a.total);
    if (g >= gend) return;
    int ca = -1, cP = -1, cslot = 0;
    double xi[IPL], yi[IPL], zi[IPL], mi[IPL], ax[IPL], ay[IPL], az[IPL], ph[IPL];
#pragma unroll
    for (int q = 0; q < IPL; ++q) { xi[q] = yi[q] = zi[q] = mi[q] = ax[q] = ay[q] = az[q] = ph[q] = 0.0; }
    MutUnit u = mut_locate(f, IPL, g, gend);
    auto jrec = [&](const MutUnit &x) {
        const int b = 64 * x.J + lane;
        return b < a.n ? a.P[(size_t)a.sl.slot[x.ea] * a.n + b] : d4{-kPadFar, 0.0, 0.0, 0.0};
    };
    d4 pj = jrec(u);
    for (;;) {
        const int slot = a.sl.slot[u.ea];
        if (u.ea != ca || u.P != cP) {
            if (cP >= 0) mut_flush<IPL>(a, cslot, ca, cP, w, lane, ax, ay, az, ph, mi);
            ca = u.ea; cP = u.P; cslot = slot;
            const d4 *Ps = a.P + (size_t)slot * a.n;
#pragma unroll
            for (int q = 0; q < IPL; ++q) {
                const int i = 64 * IPL * u.P + 64 * q + lane;
                const d4 p = i < a.n ? Ps[i] : d4{kPadFar, 0.0, 0.0, 0.0};
                xi[q] = p.x; yi[q] = p.y; zi[q] = p.z; mi[q] = p.w;
                ax[q] = ay[q] = az[q] = ph[q] = 0.0;
            }
        }
        // the j-block, twice, and cleared j-side sums
        JX[lane] = pj.x; JX[lane + 64] = pj.x;
        JY[lane] = pj.y; JY[lane + 64] = pj.y;
        JZ[lane] = pj.z; JZ[lane + 64] = pj.z;
        JM[lane] = pj.w; JM[lane + 64] = pj.w;
        AX[lane] = 0.0; AX[lane + 64] = 0.0;
        AY[lane] = 0.0; AY[lane + 64] = 0.0;
        AZ[lane] = 0.0; AZ[lane + 64] = 0.0;
        __syncthreads();
        // the next unit's j-block is fetched while this one is computed
        const long long gn = g + (u.se - u.s);
        const bool more = gn < gend;
        MutUnit un = u;
        if (more) {
            un = mut_locate(f, IPL, gn, gend);
            pj = jrec(un);
        }
        const int jb = u.J - IPL * u.P;
        const bool hl = lane >= 32;
        if constexpr (JREG) {
            double jx = 0.0, jy = 0.0, jz = 0.0;
            int onext;
            if (jb >= IPL) {
                constexpr int all = (1 << IPL) - 1;
                for (int o = u.s; o < u.se; ++o) {
                    const int k = lane + o;
                    mut_step_r<IPL>(all, -1, hl, JX[k], JY[k], JZ[k], JM[k], jx, jy, jz, xi, yi, zi, mi, ax, ay, az,
                                    ph);
                }
                onext = u.se;
            } else if (jb == 0) {
                for (int t = u.s; t < u.se; ++t) {
                    const int o = t + 1, k = lane + o;
                    mut_step_r<IPL>(1, o == 32 ? 0 : -1, hl, JX[k], JY[k], JZ[k], JM[k], jx, jy, jz, xi, yi, zi, mi,
                                    ax, ay, az, ph);
                }
                onext = u.se + 1;
            } else {
                for (int o = u.s; o < u.se; ++o) {
                    const int k = lane + o;
                    const int qm = ((1 << jb) - 1) | ((o >= 1 && o <= 32) ? (1 << jb) : 0);
                    mut_step_r<IPL>(qm, o == 32 ? jb : -1, hl, JX[k], JY[k], JZ[k], JM[k], jx, jy, jz, xi, yi, zi, mi,
                                    ax, ay, az, ph);
                }
                onext = u.se;
            }
            // lane l now holds the sums of j-body (l + onext) mod 64
            const int b = 64 * u.J + ((lane + onext) & 63);
            if (b < a.n) {
                const int piece = u.s > 0 ? 1 : 0;
                a.jp[(size_t)slot * a.jp_s + ((size_t)piece * f.npr + u.P) * a.n + b] = d3{jx, jy, jz};
            }
            __syncthreads();
            if (!more) break;
            g = gn;
            u = un;
            continue;
        }
        if (jb >= IPL) {            // off the diagonal: every i-block, every offset
            constexpr int all = (1 << IPL) - 1;
            // the LDS reads of step o + 1 are issued before step o is computed
            // (index lane + o + 1 <= 127 stays inside the doubled block)
            double xj = JX[lane + u.s], yj = JY[lane + u.s], zj = JZ[lane + u.s], mj = JM[lane + u.s];
            for (int o = u.s; o < u.se; ++o) {
                const int k = lane + o;
                const double xn = JX[k + 1], yn = JY[k + 1], zn = JZ[k + 1], mn = JM[k + 1];
                mut_step<IPL>(k, all, -1, hl, xj, yj, zj, mj, AX, AY, AZ, xi, yi, zi, mi, ax, ay, az, ph);
                xj = xn; yj = yn; zj = zn; mj = mn;
            }
        } else if (jb == 0) {       // i-block 0's own block: offsets 1..32
            for (int t = u.s; t < u.se; ++t) {
                const int o = t + 1, k = lane + o;
                mut_step<IPL>(k, 1, o == 32 ? 0 : -1, hl, JX[k], JY[k], JZ[k], JM[k], AX, AY, AZ, xi, yi, zi, mi,
                              ax, ay, az, ph);
            }
        } else {                    // i-blocks q < jb in full, q = jb on offsets 1..32
            for (int o = u.s; o < u.se; ++o) {
                const int k = lane + o;
                const int qm = ((1 << jb) - 1) | ((o >= 1 && o <= 32) ? (1 << jb) : 0);
                mut_step<IPL>(k, qm, o == 32 ? jb : -1, hl, JX[k], JY[k], JZ[k], JM[k], AX, AY, AZ, xi, yi, zi, mi,
                              ax, ay, az, ph);
            }
        }
        __syncthreads();
        {   // this wave's share of the j-side sums of the block
            const int b = 64 * u.J + lane;
            if (b < a.n) {
                const int piece = u.s > 0 ? 1 : 0;
                a.jp[(size_t)slot * a.jp_s + ((size_t)piece * f.npr + u.P) * a.n + b] =
                    d3{AX[lane] + AX[lane + 64], AY[lane] + AY[lane + 64], AZ[lane] + AZ[lane + 64]};
            }
        }
        __syncthreads();
        if (!more) break;
        g = gn;
        u = un;
    }
    mut_flush<IPL>(a, cslot, ca, cP, w, lane, ax, ay, az, ph, mi);
}

int force_mut_blocks_per_cu() {
    int nb = 0;
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_force_mut<kMutIPL, kMutJReg>, 64, 0);
    return e == hipSuccess && nb > 0 ? nb : 1;
}

static void launch_force_mut(const Dev &d, hipStream_t s, const SlotList &sl, int nd, const FLay &f) {
    MutArgs a;
    a.P = d.P;
    a.ip = d.mip; a.jp = d.mjp; a.cp = d.mcp; a.up = d.mup;
    a.ip_s = d.mip_s; a.jp_s = d.mjp_s; a.up_s = d.mup_s;
    a.X0 = d.X0; a.dX = d.dX;
    a.parent = d.parent; a.child_off = d.child_off; a.child_idx = d.child_idx;
    a.f = f;
    a.n = d.n;
    a.nd = nd;
    a.ncb = nd > 0 ? sl.nact * f.nb : 0;
    a.total = (long long)sl.nact * f.Ec;
    a.nwaves = (int)((a.total + f.L - 1) / f.L);
    a.sl = sl;
    k_force_mut<kMutIPL, kMutJReg><<<a.nwaves, 64, 0, s>>>(a);
}

void launch_force(const Dev &d, hipStream_t s, const SlotList &sl, int nd, const FLay &f, bool om) {
    if (f.mut) {
        launch_force_mut(d, s, sl, nd, f);
        return;
    }
    const int nsplit = f.nparts - (nd > 0 ? 1 : 0);
    ForceArgs a;
    a.P = d.P;
    a.part = d.part;
    a.Upart = d.Upart;
    a.X0 = d.X0;
    a.dX = d.dX;
    a.parent = d.parent;
    a.child_off = d.child_off;
    a.child_idx = d.child_idx;
    a.n = d.n;
    a.nib = d.nfb;
    a.nib_alloc = d.nib;
    a.nsplit = nsplit;
    a.nsplit_max = d.nsplit_max;
    a.jchunk = (d.n + nsplit - 1) / nsplit;
    a.nparts = f.nparts;
    a.nd = nd;
    a.mo = d.mo;
    a.opart = d.opart;
    a.Opart = d.Opart;
    a.sl = sl;
    dim3 grid(sl.nact * d.nfb, a.nparts);
    constexpr int NW = kForceWaves, IPL = kForceIPL;
    const int ck = nd <= 0 ? 0 : (nd <= 2 ? 1 : 2);
    if (om) {
        if (ck == 0) k_force<0, NW, IPL, true><<<grid, 64 * NW, 0, s>>>(a);
        else if (ck == 1) k_force<1, NW, IPL, true><<<grid, 64 * NW, 0, s>>>(a);
        else k_force<2, NW, IPL, true><<<grid, 64 * NW, 0, s>>>(a);
    } else {
        if (ck == 0) k_force<0, NW, IPL, false><<<grid, 64 * NW, 0, s>>>(a);
        else if (ck == 1) k_force<1, NW, IPL, false><<<grid, 64 * NW, 0, s>>>(a);
        else k_force<2, NW, IPL, false><<<grid, 64 * NW, 0, s>>>(a);
    }
}

// Reduce the force partials of one slot (nparts of them per i-block, see
// force_parts): acc = G sum_part part, and the force function
// U = G/2 sum_i m_i phi_i (every workgroup reduces the same partials in the
// same order; block 0 stores U).  With OM also Omega, grad Omega and, given
// the velocities vt, per-workgroup partials of sum_i grad_i Omega . v_i.
struct ReduceArgs {
    Dev d;
    FLay fl;
    int slot;
    const d4 *part, *opart;
    const double *Opart, *mo;
    const d4 *vt;          // velocities for the w-rate partials (nullptr: none)
    int n, nib, nsplit, nsplit_max;
    double G;
    d4 *acc, *dom;
    double *Uout, *Omout, *wpart;
};

template <bool OM>
__global__ __launch_bounds__(kWG) void k_reduce_start(ReduceArgs r) {
    __shared__ double sh[3][kWG / 64];
    const int n = r.n;
    const int v = blockIdx.x * kWG + threadIdx.x;
    double wl = 0.0;
    if (v < n) {
        double x = 0.0, y = 0.0, z = 0.0;
        force_sum(r.d, r.part, r.fl, r.slot, 0, v, 0, 1, x, y, z);
        r.acc[v] = d4{r.G * x, r.G * y, r.G * z, 0.0};
        if constexpr (OM) {
            double ox = 0.0, oy = 0.0, oz = 0.0;
            for (int sp = 0; sp < r.nsplit; ++sp) {
                const d4 t = r.opart[(size_t)sp * n + v];
                ox = ox + t.x; oy = oy + t.y; oz = oz + t.z;
            }
            const double gm = r.G * r.mo[v];
            const d4 g{gm * ox, gm * oy, gm * oz, 0.0};
            r.dom[v] = g;
            if (r.vt) {
                const d4 w = r.vt[v];
                wl = (g.x * w.x + g.y * w.y) + g.z * w.z;
            }
        }
    }
    int cnt = 0;
    const double *up = force_upart(r.d, r.fl, r.slot, &cnt);
    double u = 0.0;
    for (int k = threadIdx.x; k < cnt; k += kWG) u = u + up[k];
    const double U = 0.5 * r.G * block_sum1<kWG>(u, sh[0]);
    double Om = 0.0;
    if constexpr (OM) {
        const int ocnt = r.nib * r.nsplit;
        double o = 0.0;
        for (int k = threadIdx.x; k < ocnt; k += kWG) o = o + r.Opart[k];
        Om = 0.5 * r.G * block_sum1<kWG>(o, sh[1]);
        if (r.vt) {
            const double ws = block_sum1<kWG>(wl, sh[2]);
            if (threadIdx.x == 0) r.wpart[blockIdx.x] = ws;
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *r.Uout = U;
        *r.Omout = Om;
    }
}

void launch_reduce_start(const Dev &d, hipStream_t s, int slot, double G, const FLay &f, d4 *acc_out,
                         double *U_out, bool om, bool with_w) {
    const int nb = (d.n + kWG - 1) / kWG;
    ReduceArgs r;
    const size_t po = (size_t)slot * d.nsplit_max * d.n, uo = (size_t)slot * d.nib * d.nsplit_max;
    r.d = d;
    r.fl = f;
    r.slot = slot;
    r.part = d.part + po;
    r.opart = om ? d.opart + po : nullptr;
    r.Opart = om ? d.Opart + uo : nullptr;
    r.mo = d.mo;
    r.vt = with_w ? d.Vt + (size_t)slot * d.n : nullptr;
    r.n = d.n;
    r.nib = d.nfb;
    r.nsplit = f.nparts;
    r.nsplit_max = d.nsplit_max;
    r.G = G;
    r.acc = acc_out;
    r.dom = d.dOm0;
    r.Uout = U_out;
    r.Omout = &d.ctl->Om0;
    r.wpart = om ? d.wpart + (size_t)slot * d.nkwg4 : nullptr;
    if (om) k_reduce_start<true><<<nb, kWG, 0, s>>>(r);
    else k_reduce_start<false><<<nb, kWG, 0, s>>>(r);
}

}  // namespace mstar
