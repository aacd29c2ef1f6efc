// Shared device helpers and the launch interface between the host driver
// (api.hip) and the kernel files.  FP64 throughout; all files are compiled
// with -ffp-contract=off so every fused multiply-add below is explicit.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pair.h"

namespace mstar {

// One 32-byte record per body: xyz plus a fourth slot (mass for positions,
// zero padding for edge vectors and velocities).  32-byte rows let a wave
// fetch a whole j-body with one scalar load.
struct __attribute__((aligned(32))) d4 {
    double x, y, z, w;
};
// Packed xyz (24 bytes) for the mutual force kernel's partial sums: the kernel
// writes them and the kick reads them back, so every byte is HBM traffic twice.
struct d3 {
    double x, y, z;
};

constexpr int kMaxDiv = 17;        // k_fix <= 16 divisions plus the start-state slot
constexpr int kBaseSlot = kMaxDiv - 1;   // slot holding the start state of a GBS step
constexpr int kMaxExtPoints = 16;   // point masses of an external field
constexpr int kWG = 256;           // threads per workgroup of the O(N) kernels
constexpr int kForceWaves = 4;     // waves per force workgroup (same i-block, split j-range)
constexpr int kForceIPL = 1;       // i-bodies per lane in the force kernel (2 and 4 measured slower)
constexpr int kTreeWG = 1024;      // single-workgroup tree kernels
constexpr int kMaxNd = 4;          // largest closeness N_d of eq. LCA on the GPU path
constexpr int kMutIPL = 4;         // i-bodies per lane of the mutual force kernel (one row = 64 kMutIPL bodies)
constexpr bool kMutJReg = true;    // mutual kernel: j-side sums rotate through registers (else LDS atomic adds)

// Deterministic sum of a block of values held one per thread (fixed tree).
template <int NT>
__device__ __forceinline__ double block_sum(double v, double *sh) {
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
#pragma unroll
    for (int s = NT / 2; s > 0; s >>= 1) {
        if (t < s) sh[t] = sh[t] + sh[t + s];
        __syncthreads();
    }
    double r = sh[0];
    __syncthreads();
    return r;
}

// Sum over a wave; lane 0 holds the sum taken in a fixed order.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = v + __shfl_xor(v, off, 64);
    return v;
}

// Sum over a workgroup of NT threads with one barrier: lane 0 of every wave
// writes its wave's sum to sh[0 .. NT/64), then every thread adds them in
// wave order (the same value in every thread and workgroup).  A later
// reduction in the same kernel must use other words of shared memory.
template <int NT>
__device__ __forceinline__ double block_sum1(double v, double *sh) {
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = sh[0];
#pragma unroll
    for (int k = 1; k < NT / 64; ++k) s = s + sh[k];
    return s;
}

// ---------------------------------------------------------------- stages
// Per-slot description of one launch of the drift / force / kick stage over
// several substep divisions at once ("slots"; slot kMaxDiv-1 style indices are
// chosen by the host).
struct SlotList {
    int nact;
    int slot[kMaxDiv];
    int nsub[kMaxDiv];     // substeps of the division in this slot
    int half[kMaxDiv];     // drift: 1 = half substep
    int first[kMaxDiv];    // drift: 1 = first drift (uses T of the start state)
};

struct Ctl {               // device control block, read back once per GBS step
    double H;              // fictitious step of this attempt (after the end-time clip)
    double eps;            // GBS error measure
    double h_next;
    double U0, T0, gk0;    // start-state force function, kinetic energy, alpha U + beta Omega + gamma
    double Om0;            // start-state TTL function Omega (0 when beta = 0)
    double dw0;            // sum_i grad_i Omega . v_i at the start state (dw/dt, TTL)
    double t_est;          // predicted physical time after the step
    int32_t accepted;
    int32_t clipped;
    int32_t coincident;    // a zero-length MST edge was found
    int32_t topo;          // the last rebuild changed the tree
    int32_t tree_bad;      // the last rebuild's Boruvka rounds did not finish: the old tree is kept
    int32_t mst_rounds;    // Boruvka rounds of the last finished build
    int32_t kacc;          // order k whose extrapolation was accepted (0: rejected)
    int32_t pad_;
};

struct SysScal {           // start-of-step scalars of the integrated state
    double t, B, w;
    double rcm[3], vcm[3];
};

struct CtlBlock {          // Ctl and SysScal side by side: one read-back per GBS step
    Ctl ctl;
    SysScal sys;
};

struct DivScal {           // per-division increments of the scalar variables
    double tau, dw, drcm[3];
    double dtk;            // time step of the latest kick
    double dwn;            // TTL: dw including the latest kick (set by the drift after it)
    double dB;             // external field: change of B up to the kick before the latest
    double dBn;            // external field: dB including the latest kick (set by the drift after it)
    double dvcm[3];        // external field: change of v_cm
    double pad[4];
};

// External perturbation (device memory): uniform acceleration g and np fixed
// Plummer-softened point masses pt[k] = (G M_k, X_k, Y_k, Z_k, b_k^2).
struct ExtField {
    double g[3];
    double Minv;           // 1 / total mass of the system
    double pt[kMaxExtPoints][5];
    int32_t np, pad;
};

// Workspace pointers used by the kernels (device memory).
struct Dev {
    int n, nib, kfmax;          // bodies, 64-wide i-blocks, division slots allocated
    int nfb;                    // force-kernel i-blocks (64 * kForceIPL bodies each)
    // tree
    int32_t *parent, *level, *child_off, *child_idx, *root;
    int32_t *parent_new, *level_new;
    // start state
    d4 *X0, *V0;                // MST edge vectors / velocities (row v = edge parent->v)
    d4 *P0, *Vt0;               // COM-frame positions (+mass) and velocities
    d4 *a0;                     // accelerations at the start state
    double *m;
    SysScal *sys;
    Ctl *ctl;
    // divisions (slot-major)
    d4 *P, *Vt, *dX, *dV;       // [slot][n]: positions+mass, COM-frame velocities, edge increments
    d4 *dP, *dVt;               // [slot][n]: increments of positions / velocities
    d4 *akick;                  // [slot][n]: accelerations of the latest kick
    d4 *dX1, *dV1, *dP1, *dVt1; // extrapolated increments
    DivScal *dscal, *dscal1;    // [slot], extrapolated
    d4 *part;                   // force partials [slot][nsplit_max][n]
    double *Upart;              // [slot][nib * nsplit_max]
    // TTL function Omega (beta != 0; allocated on first use)
    double *mo;                 // [n] Omega masses: m_i if m_i <= omega_mass_max else 0
    d4 *opart;                  // [slot][nsplit_max][n] partial (sum mo_j d/r^3, sum mo_j/r)
    double *Opart;              // [slot][nib * nsplit_max] partial sum_i mo_i (sum_j mo_j/r)
    double *wpart;              // [slot][nkwg4] partial sum_i grad_i Omega . v_i
    d4 *dOm0;                   // [n] grad Omega at the start state
    double *Tpart;              // [slot][nkwg4] (kick: nkwg4 workgroups; commit: nkwg)
    // external perturbation (allocated on first use)
    ExtField *ext;
    d4 *fext;                   // [slot][n] external accelerations at the latest kick's positions
    d4 *fpart;                  // [slot][nkwg4] partial (sum m f, sum m f . v) per workgroup
    double *bpart;              // [slot][nkwg4] partial sum m f . (v_old + v_new)/2 of the latest kick
    double *epspart;            // [nkwg + 1]
    int nsplit_max, nkwg, nkwg4;  // nkwg = ceil(n/256), nkwg4 = ceil(n/64)
    // tree scratch
    d4 *tsA, *tsB;              // tree sums: root-relative positions / velocities
    d4 *tsC, *tsD, *tsE, *tsF;  // ping-pong scratch
    int32_t *ancA, *ancB;
    double *bor_w;              // Boruvka per-split best weight [nsplit][n]
    int32_t *bor_j;             // Boruvka per-split best index [nsplit][n]
    int32_t *rounds;            // Boruvka rounds taken by the last build
    int32_t *comp, *ecomp_tmp;
    unsigned long long *cw, *cidx;
    int32_t *tgt, *done, *ncomp;
    int32_t *deg, *off, *fill, *adj, *arcpos, *nxtA, *nxtB, *rkA, *rkB;
    int32_t *cnt;
    double *scr;                // misc scalar scratch
    // mutual (i < j) force kernel output (allocated when N suits that kernel)
    d3 *mip;                    // [slot][rows][maxw][64 kMutIPL] i-side partials, one per wave and row
    d3 *mjp;                    // [slot][2][rows][n] j-side partials, one per row (two if a wave split the block)
    d4 *mcp;                    // [slot][n] close-pair corrections
    double *mup;                // [slot][rows * maxw + nib] potential partials
    size_t mip_s, mjp_s, mup_s; // per-slot strides
};

// ------------------------------------------------- force output layout
// Where one launch of the force kernel leaves the force on each body.
//  mut = 0 (pairwise kernel): nparts partial rows part[slot][k][n].
//  mut = 1 (mutual kernel, each unordered pair once): the bodies form rows of
//  64 ipl (the i-bodies one wave holds); row P pairs with the 64-body j-blocks
//  J >= ipl P.  The pair work of all nact evaluations of the launch is one
//  sequence of steps (eval, row, j-block, step), cut into equal ranges of L
//  steps, one per wave.  A wave leaves one i-side partial per row it touches
//  and one j-side partial per j-block; a j-block cut between two waves leaves
//  two (pieces 0 and 1).  Every partial is written exactly once per launch.
// Buffers of the divide-and-conquer tree builder (Sec. 3.3); n = capacity.
struct DcBuf {
    uint32_t *key;              // [2n] Morton keys (two radix-sort buffers)
    int32_t *idx;               // [2n] body of each key
    int32_t *flag;              // [n + 1] part starts over sorted positions
    int2 *cells;                // [2n] octree cell ranges of two levels
    int32_t *pstart;            // [n + 1] first sorted position of each part
    int32_t *part;              // [n] part of each body
    d4 *spos;                   // [n] positions in sorted order
    double *bw;                 // [n] Prim of a large part: lightest edge into the part tree
    int32_t *bu;                // [n] its tree end
    int32_t *in;                // [n] in the part tree
    int32_t *np;                // number of parts
};
// Partition and part trees; the Boruvka rounds of the exact builder finish the tree.
void launch_mst_dc(const Dev &d, const DcBuf &b, hipStream_t s, const d4 *pos, int mcap);

struct FLay {
    int mut;
    int nparts;                 // mut = 0
    int nb, npr, ipl, maxw;     // mut = 1: 64-blocks, rows, i-bodies per lane, i-side partials per row
    int ncorr;                  // mut = 1: 1 if the close-pair correction partial exists (N_d > 0)
    int pad;
    long long Ec, L;            // mut = 1: steps per evaluation, steps per wave
};

// Steps of the rows before row P: a row P has one half j-block (32 steps: the
// diagonal block of its first i-block) and 64 steps for every later j-block.
__host__ __device__ inline long long mut_rs(const FLay &f, long long P) {
    return 32 * P + 64 * P * (long long)(f.nb - 1) - 32LL * f.ipl * P * (P - 1);
}
__host__ __device__ inline int mut_cost(const FLay &f, int P, int J) { return J == f.ipl * P ? 32 : 64; }
__host__ __device__ inline long long mut_js(const FLay &f, int P, int J) {
    return J == f.ipl * P ? 0 : 32 + 64LL * (J - f.ipl * P - 1);
}

// Sum of the force partials of body v (eval ea of the launch, division slot
// `slot`): the items with index = t (mod nt), in a fixed order.
__device__ inline void force_sum(const Dev &d, const d4 *part, const FLay &f, int slot, int ea, int v, int t, int nt,
                                 double &x, double &y, double &z) {
    const int n = d.n;
    if (!f.mut) {
        for (int k = t; k < f.nparts; k += nt) {
            const d4 e = part[(size_t)k * n + v];
            x = x + e.x; y = y + e.y; z = z + e.z;
        }
        return;
    }
    const int rowb = 64 * f.ipl;
    const int P = v / rowb;
    const long long base = (long long)ea * f.Ec;
    const long long wf = (base + mut_rs(f, P)) / f.L, wl = (base + mut_rs(f, P + 1) - 1) / f.L;
    const int nw = (int)(wl - wf + 1);
    const d3 *ip = d.mip + (size_t)slot * d.mip_s + ((size_t)P * f.maxw) * rowb + (v - rowb * P);
    for (int k = t; k < nw; k += nt) {
        const d3 e = ip[(size_t)k * rowb];
        x = x + e.x; y = y + e.y; z = z + e.z;
    }
    const int J = v / 64;
    const d3 *jp = d.mjp + (size_t)slot * d.mjp_s + v;
    for (int Q = t; Q <= P; Q += nt) {
        const d3 e = jp[(size_t)Q * n];
        x = x + e.x; y = y + e.y; z = z + e.z;
        const long long st = base + mut_rs(f, Q) + mut_js(f, Q, J);
        if (st / f.L != (st + mut_cost(f, Q, J) - 1) / f.L) {
            const d3 e2 = jp[((size_t)f.npr + Q) * n];
            x = x + e2.x; y = y + e2.y; z = z + e2.z;
        }
    }
    if (f.ncorr && t == 0) {
        const d4 e = d.mcp[(size_t)slot * n + v];
        x = x + e.x; y = y + e.y; z = z + e.z;
    }
}

// The potential partials of one launch for division slot `slot`:
// U = G/2 * sum of the *cnt values at the returned address.
__device__ inline const double *force_upart(const Dev &d, const FLay &f, int slot, int *cnt) {
    if (!f.mut) {
        *cnt = d.nfb * f.nparts;
        return d.Upart + (size_t)slot * d.nib * d.nsplit_max;
    }
    *cnt = f.npr * f.maxw + (f.ncorr ? f.nb : 0);
    return d.mup + (size_t)slot * d.mup_s;
}

// ---------------------------------------------------------------- launches
// kernels_force.hip
void launch_force(const Dev &d, hipStream_t s, const SlotList &sl, int nd, const FLay &f, bool om);
// Partial sums per i-block written by the pairwise kernel: the nsplit
// j-splits plus one close-pair correction block when N_d > 0.
inline int force_parts(int nsplit, int nd) { return nsplit + (nd > 0 ? 1 : 0); }
// Resident force workgroups per CU (occupancy of the pairwise force kernel).
int force_blocks_per_cu(int nd);
// Resident 64-thread workgroups per CU of the mutual force kernel.
int force_mut_blocks_per_cu();
void launch_reduce_start(const Dev &d, hipStream_t s, int slot, double G, const FLay &f, d4 *acc_out,
                         double *U_out, bool om, bool with_w);
// kernels_step.hip
void launch_div_init(const Dev &d, hipStream_t s, int ndiv, int base_slot);
// (alpha, beta, gamma): the time-transformation triplet; beta != 0 switches
// on the TTL function Omega and its auxiliary variable w.
struct Ttl {
    double alpha, beta, gamma;
};
void launch_drift(const Dev &d, hipStream_t s, const SlotList &sl, Ttl tr, bool ex);
void launch_kick(const Dev &d, hipStream_t s, const SlotList &sl, const FLay &f, double G, Ttl tr, bool ex);
void launch_ext(const Dev &d, hipStream_t s, const SlotList &sl, int at_start);
void launch_ext_minv(const Dev &d, hipStream_t s);
void launch_set_h(const Dev &d, hipStream_t s, double H, double t_end, int clip, Ttl tr, int from_ctl);
void launch_put_hnext(const Dev &d, hipStream_t s, double H);
void prepare_tree_launches();   // one-time runtime settings of the tree kernels (before any capture)
// rule 0: error at k_fix and the outputs T_{kf,kf}; rule 1: errors of every
// order k = 2..kf only (the outputs follow from launch_extrap_pick once the
// control has chosen the order).
void launch_extrapolate(const Dev &d, hipStream_t s, int kf, Ttl tr, int base_slot, bool ex, int rule = 0);
void launch_extrap_pick(const Dev &d, hipStream_t s, int kf, bool ex);
void launch_control(const Dev &d, hipStream_t s, int kf, double eta, double a_gbs, double f_min, double f_max,
                    int rule = 0);
void launch_commit(const Dev &d, hipStream_t s, int from_extrap, int slot);
void launch_state_from_cartesian(const Dev &d, hipStream_t s, const double *x, const double *v);
void launch_com_frame(const Dev &d, hipStream_t s, int with_T);
void launch_output_cartesian(const Dev &d, hipStream_t s, double *x, double *v);
void launch_set_B(const Dev &d, hipStream_t s);   // B = U0 - T0 and w = Omega0
void launch_pack3(hipStream_t s, const double *x, const double *m, d4 *out, int n);
void launch_unpack3(hipStream_t s, const d4 *in, double *out, int n);
void launch_set_sys(const Dev &d, hipStream_t s, double t, double B, double w, const double *rcm,
                    const double *vcm, int set_com);
void launch_check_coincident(const Dev &d, hipStream_t s);
// kernels_probe.hip
size_t issue_probe_bytes();
hipError_t issue_probe(hipStream_t s, double *out, int n_simd, double clock_ghz, double cycles[2]);
// kernels_tree.hip
void launch_tree_sums(const Dev &d, hipStream_t s, const d4 *X, const d4 *V, d4 *rho, d4 *ups);
void launch_mst_init(const Dev &d, hipStream_t s, const d4 *pos, int root_in);
void launch_mst_rounds(const Dev &d, hipStream_t s, const d4 *pos, int rounds, int nsplit);
void launch_mst_root(const Dev &d, hipStream_t s);
void launch_tree_finish(const Dev &d, hipStream_t s);
void launch_rebuild_edges(const Dev &d, hipStream_t s, const d4 *rho, const d4 *ups, int nd);
void launch_levels_children(const Dev &d, hipStream_t s);

}  // namespace mstar
