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
// Close pairs (tree distance <= N_d): the main loop uses Cartesian
// differences for every pair; one extra workgroup per i-block (grid row
// y = 0, dispatched first) computes, for each close pair, the term built from
// the MST path sum minus the Cartesian term (same operation sequence as the
// main loop, so the subtracted term is the one that was added) into a partial
// of its own.  These correction blocks are short and run beside the j-loop
// blocks instead of lengthening one of them.
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
    SlotList sl;
};

__device__ __forceinline__ void add_close(double dpx, double dpy, double dpz, const d4 &pi, const d4 &pj,
                                          double &ax, double &ay, double &az, double &ph) {
    double s1, mr1, s0, mr0;
    pair_terms(dpx, dpy, dpz, pj.w, s1, mr1);
    const double cx = pj.x - pi.x, cy = pj.y - pi.y, cz = pj.z - pi.z;
    pair_terms(cx, cy, cz, pj.w, s0, mr0);
    ax = ax + fma(s1, dpx, -(s0 * cx));
    ay = ay + fma(s1, dpy, -(s0 * cy));
    az = az + fma(s1, dpz, -(s0 * cz));
    ph = ph + (mr1 - mr0);
}

__device__ __forceinline__ d4 cur_edge(const d4 *X0, const d4 *dX, int u) {
    const d4 a = X0[u], b = dX[u];
    return d4{a.x + b.x, a.y + b.y, a.z + b.z, 0.0};
}

// Replace the Cartesian terms of all pairs (i, j) within ND tree edges by the
// MST path-sum terms.  Separations follow the rule d_ij = S_j - S_i with S_v
// the sum of edge vectors from the lowest common ancestor down to v.
template <int ND>
__device__ void close_correction(int i, const d4 *P, const d4 *X0, const d4 *dX, const int32_t *parent,
                                 const int32_t *coff, const int32_t *cidx, double &ax, double &ay,
                                 double &az, double &ph) {
    const d4 pi = P[i];
    const int p = parent[i];
    if (p >= 0) {
        const d4 Xi = cur_edge(X0, dX, i);
        add_close(-Xi.x, -Xi.y, -Xi.z, pi, P[p], ax, ay, az, ph);              // parent
        if (ND >= 2) {
            const int g = parent[p];
            if (g >= 0) {
                const d4 Xp = cur_edge(X0, dX, p);
                add_close(-(Xp.x + Xi.x), -(Xp.y + Xi.y), -(Xp.z + Xi.z), pi, P[g], ax, ay, az, ph);  // grandparent
            }
            for (int k = coff[p]; k < coff[p + 1]; ++k) {                        // siblings
                const int c = cidx[k];
                if (c == i) continue;
                const d4 Xs = cur_edge(X0, dX, c);
                add_close(Xs.x - Xi.x, Xs.y - Xi.y, Xs.z - Xi.z, pi, P[c], ax, ay, az, ph);
            }
        }
    }
    for (int k = coff[i]; k < coff[i + 1]; ++k) {                                // children
        const int c = cidx[k];
        const d4 Xc = cur_edge(X0, dX, c);
        add_close(Xc.x, Xc.y, Xc.z, pi, P[c], ax, ay, az, ph);
        if (ND >= 2) {
            for (int q = coff[c]; q < coff[c + 1]; ++q) {                        // grandchildren
                const int gc = cidx[q];
                const d4 Xg = cur_edge(X0, dX, gc);
                add_close(Xc.x + Xg.x, Xc.y + Xg.y, Xc.z + Xg.z, pi, P[gc], ax, ay, az, ph);
            }
        }
    }
}

// Inner loop over j in [jb, je) for the IPL i-bodies of each lane; GUARD
// masks the self pair (only the diagonal block needs it).
template <bool GUARD, int IPL>
__device__ __forceinline__ void j_loop(const d4 *__restrict__ P, int jb, int je, const int (&ii)[IPL],
                                       const d4 (&pi)[IPL], double (&ax)[IPL], double (&ay)[IPL],
                                       double (&az)[IPL], double (&ph)[IPL]) {
#pragma unroll 8
    for (int j = jb; j < je; ++j) {
        const d4 pj = P[j];
#pragma unroll
        for (int q = 0; q < IPL; ++q) {
            const double dx = pj.x - pi[q].x, dy = pj.y - pi[q].y, dz = pj.z - pi[q].z;
            double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
            double mj = pj.w;
            if (GUARD) {
                const bool self = (j == ii[q]);
                r2 = self ? 1.0 : r2;
                mj = self ? 0.0 : mj;
            }
            const double y = rsqrt_f64(r2);
            const double mr = mj * y;
            const double s = mr * (y * y);
            ph[q] = ph[q] + mr;
            ax[q] = fma(s, dx, ax[q]);
            ay[q] = fma(s, dy, ay[q]);
            az[q] = fma(s, dz, az[q]);
        }
    }
}

template <int ND, int NW, int IPL>
__global__ __launch_bounds__(64 * NW) void k_force(ForceArgs a) {
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int ib = blockIdx.x % a.nib;
    const int slot = a.sl.slot[blockIdx.x / a.nib];
    const int part = blockIdx.y;                          // partial index
    const int split = ND > 0 ? part - 1 : part;            // j-split index (-1: correction block)
    const int n = a.n;
    const d4 *__restrict__ P = a.P + (size_t)slot * n;
    const int i0 = ib * 64 * IPL;
    int ii[IPL];
    d4 pi[IPL];
#pragma unroll
    for (int q = 0; q < IPL; ++q) {
        const int i = i0 + q * 64 + lane;
        ii[q] = i < n ? i : n - 1;
        pi[q] = P[ii[q]];
    }
    if (ND > 0 && split < 0) {   // close-pair correction block (wave 0)
        if (wv != 0) return;
        double u = 0.0;
#pragma unroll
        for (int q = 0; q < IPL; ++q) {
            const int i = i0 + q * 64 + lane;
            if (i < n) {
                double cx = 0.0, cy = 0.0, cz = 0.0, cp = 0.0;
                close_correction<ND>(i, P, a.X0, a.dX + (size_t)slot * n, a.parent, a.child_off, a.child_idx, cx,
                                     cy, cz, cp);
                a.part[((size_t)slot * a.nsplit_max + part) * n + i] = d4{cx, cy, cz, cp};
                u = u + pi[q].w * cp;
            }
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) u = u + __shfl_xor(u, off, 64);
        if (lane == 0) a.Upart[(size_t)slot * a.nib_alloc * a.nsplit_max + (size_t)ib * a.nparts + part] = u;
        return;
    }
    const int j0 = split * a.jchunk;
    const int j1 = min(n, j0 + a.jchunk);
    const int qw = (max(j1 - j0, 0) + NW - 1) / NW;
    int jb = min(j1, j0 + wv * qw);
    int je = min(j1, jb + qw);
    jb = __builtin_amdgcn_readfirstlane(jb);
    je = __builtin_amdgcn_readfirstlane(je);
    const int g0 = __builtin_amdgcn_readfirstlane(max(jb, i0));
    const int g1 = __builtin_amdgcn_readfirstlane(min(je, i0 + 64 * IPL));
    double ax[IPL], ay[IPL], az[IPL], ph[IPL];
#pragma unroll
    for (int q = 0; q < IPL; ++q) ax[q] = ay[q] = az[q] = ph[q] = 0.0;
    if (g0 < g1) {
        j_loop<false, IPL>(P, jb, g0, ii, pi, ax, ay, az, ph);
        j_loop<true, IPL>(P, g0, g1, ii, pi, ax, ay, az, ph);
        j_loop<false, IPL>(P, g1, je, ii, pi, ax, ay, az, ph);
    } else {
        j_loop<false, IPL>(P, jb, je, ii, pi, ax, ay, az, ph);
    }
    __shared__ d4 red[NW][IPL][64];
#pragma unroll
    for (int q = 0; q < IPL; ++q) red[wv][q][lane] = d4{ax[q], ay[q], az[q], ph[q]};
    __syncthreads();
    if (wv != 0) return;
    double u = 0.0;
#pragma unroll
    for (int q = 0; q < IPL; ++q) {
        const int i = i0 + q * 64 + lane;
        d4 s = red[0][q][lane];
        for (int w = 1; w < NW; ++w) {
            const d4 t = red[w][q][lane];
            s.x = s.x + t.x; s.y = s.y + t.y; s.z = s.z + t.z; s.w = s.w + t.w;
        }
        if (i < n) {
            a.part[((size_t)slot * a.nsplit_max + part) * n + i] = s;
            u = u + pi[q].w * s.w;
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) u = u + __shfl_xor(u, off, 64);
    if (lane == 0) a.Upart[(size_t)slot * a.nib_alloc * a.nsplit_max + (size_t)ib * a.nparts + part] = u;
}

int force_blocks_per_cu(int nd) {
    constexpr int NW = kForceWaves, IPL = kForceIPL;
    int nb = 0;
    hipError_t e;
    if (nd <= 0) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_force<0, NW, IPL>, 64 * NW, 0);
    else if (nd == 1) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_force<1, NW, IPL>, 64 * NW, 0);
    else e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_force<2, NW, IPL>, 64 * NW, 0);
    return e == hipSuccess && nb > 0 ? nb : 1;
}

void launch_force(const Dev &d, hipStream_t s, const SlotList &sl, int nd, int nsplit) {
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
    a.sl = sl;
    dim3 grid(sl.nact * d.nfb, a.nparts);
    constexpr int NW = kForceWaves, IPL = kForceIPL;
    if (nd <= 0) k_force<0, NW, IPL><<<grid, 64 * NW, 0, s>>>(a);
    else if (nd == 1) k_force<1, NW, IPL><<<grid, 64 * NW, 0, s>>>(a);
    else k_force<2, NW, IPL><<<grid, 64 * NW, 0, s>>>(a);
}

// Reduce the force partials of one slot (nparts of them per i-block, see
// force_parts): acc = G sum_part part, and the
// force function U = G/2 sum_i m_i phi_i (every workgroup reduces the same
// partials in the same order; block 0 stores U).
__global__ __launch_bounds__(kWG) void k_reduce_start(const d4 *part, const double *Upart, int n, int nib,
                                                      int nsplit, int nsplit_max, double G, d4 *acc,
                                                      double *Uout) {
    __shared__ double sh[kWG];
    const int cnt = nib * nsplit;
    double u = 0.0;
    for (int k = threadIdx.x; k < cnt; k += kWG) u = u + Upart[k];
    const double U = 0.5 * G * block_sum<kWG>(u, sh);
    if (blockIdx.x == 0 && threadIdx.x == 0) *Uout = U;
    const int v = blockIdx.x * kWG + threadIdx.x;
    if (v >= n) return;
    double x = 0.0, y = 0.0, z = 0.0;
    for (int sp = 0; sp < nsplit; ++sp) {
        const d4 t = part[(size_t)sp * n + v];
        x = x + t.x; y = y + t.y; z = z + t.z;
    }
    acc[v] = d4{G * x, G * y, G * z, 0.0};
}

void launch_reduce_start(const Dev &d, hipStream_t s, int slot, double G, int nsplit, d4 *acc_out,
                         double *U_out) {
    const int nb = (d.n + kWG - 1) / kWG;
    k_reduce_start<<<nb, kWG, 0, s>>>(d.part + (size_t)slot * d.nsplit_max * d.n,
                                      d.Upart + (size_t)slot * d.nib * d.nsplit_max, d.n, d.nfb, nsplit,
                                      d.nsplit_max, G, acc_out, U_out);
}

}  // namespace mstar
