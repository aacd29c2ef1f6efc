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
template <bool OM>
__device__ __forceinline__ void add_close(double dpx, double dpy, double dpz, const d4 &pi, const d4 &pj,
                                          double moj, Sums &c) {
    const double cx = pj.x - pi.x, cy = pj.y - pi.y, cz = pj.z - pi.z;
    const double y1 = pair_y(dpx, dpy, dpz), y0 = pair_y(cx, cy, cz);
    const double q1 = y1 * y1, q0 = y0 * y0;
    const double mr1 = pj.w * y1, mr0 = pj.w * y0;
    const double s1 = mr1 * q1, s0 = mr0 * q0;
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
template <bool GENERIC, bool OM>
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
            add_close<OM>(0.0 - Xi.x, 0.0 - Xi.y, 0.0 - Xi.z, pi, P[p], mom(p), c);          // parent
            if (nd >= 2) {
                const int g = parent[p];
                if (g >= 0) {
                    const d4 Xp = cur_edge(X0, dX, p);
                    const d4 S{Xp.x + Xi.x, Xp.y + Xi.y, Xp.z + Xi.z, 0.0};
                    add_close<OM>(0.0 - S.x, 0.0 - S.y, 0.0 - S.z, pi, P[g], mom(g), c);      // grandparent
                }
                for (int k = coff[p]; k < coff[p + 1]; ++k) {                                // siblings
                    const int q = cidx[k];
                    if (q == i) continue;
                    const d4 Xs = cur_edge(X0, dX, q);
                    add_close<OM>(Xs.x - Xi.x, Xs.y - Xi.y, Xs.z - Xi.z, pi, P[q], mom(q), c);
                }
            }
        }
        for (int k = coff[i]; k < coff[i + 1]; ++k) {                                        // children
            const int q = cidx[k];
            const d4 Xc = cur_edge(X0, dX, q);
            add_close<OM>(Xc.x, Xc.y, Xc.z, pi, P[q], mom(q), c);
            if (nd >= 2) {
                for (int r = coff[q]; r < coff[q + 1]; ++r) {                                // grandchildren
                    const int gc = cidx[r];
                    const d4 Xg = cur_edge(X0, dX, gc);
                    add_close<OM>(Xc.x + Xg.x, Xc.y + Xg.y, Xc.z + Xg.z, pi, P[gc], mom(gc), c);
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
            if (a > 0) add_close<OM>(0.0 - Si.x, 0.0 - Si.y, 0.0 - Si.z, pi, P[anc], mom(anc), c);
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
                add_close<OM>(Sc.x - Si.x, Sc.y - Si.y, Sc.z - Si.z, pi, P[ch], mom(ch), c);
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

void launch_force(const Dev &d, hipStream_t s, const SlotList &sl, int nd, int nsplit, bool om) {
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
    a.nparts = force_parts(nsplit, nd);
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
    const d4 *part, *opart;
    const double *Upart, *Opart, *mo;
    const d4 *vt;          // velocities for the w-rate partials (nullptr: none)
    int n, nib, nsplit, nsplit_max;
    double G;
    d4 *acc, *dom;
    double *Uout, *Omout, *wpart;
};

template <bool OM>
__global__ __launch_bounds__(kWG) void k_reduce_start(ReduceArgs r) {
    __shared__ double sh[3][kWG / 64];
    const int n = r.n, cnt = r.nib * r.nsplit;
    const int v = blockIdx.x * kWG + threadIdx.x;
    double wl = 0.0;
    if (v < n) {
        double x = 0.0, y = 0.0, z = 0.0;
        for (int sp = 0; sp < r.nsplit; ++sp) {
            const d4 t = r.part[(size_t)sp * n + v];
            x = x + t.x; y = y + t.y; z = z + t.z;
        }
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
    double u = 0.0;
    for (int k = threadIdx.x; k < cnt; k += kWG) u = u + r.Upart[k];
    const double U = 0.5 * r.G * block_sum1<kWG>(u, sh[0]);
    double Om = 0.0;
    if constexpr (OM) {
        double o = 0.0;
        for (int k = threadIdx.x; k < cnt; k += kWG) o = o + r.Opart[k];
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

void launch_reduce_start(const Dev &d, hipStream_t s, int slot, double G, int nsplit, d4 *acc_out,
                         double *U_out, bool om, bool with_w) {
    const int nb = (d.n + kWG - 1) / kWG;
    ReduceArgs r;
    const size_t po = (size_t)slot * d.nsplit_max * d.n, uo = (size_t)slot * d.nib * d.nsplit_max;
    r.part = d.part + po;
    r.Upart = d.Upart + uo;
    r.opart = om ? d.opart + po : nullptr;
    r.Opart = om ? d.Opart + uo : nullptr;
    r.mo = d.mo;
    r.vt = with_w ? d.Vt + (size_t)slot * d.n : nullptr;
    r.n = d.n;
    r.nib = d.nfb;
    r.nsplit = nsplit;
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
