// Frozen-controller replay and its adjoint (reverse-mode derivative).
//
// With the accepted fictitious steps H_k recorded, the integrator is a smooth
// map from (r0, v0) to the end state.  In exact arithmetic the map does not
// depend on the coordinates it is evaluated in: the MST transforms and
// rebuilds (Sec. 2.2, 3.5) are linear changes of variables, a drift moves
// every body by dt v_i and a kick changes every velocity by dt a_i.  These
// kernels therefore evaluate and differentiate the Cartesian form:
//   drift D(ds): dt = ds / (alpha (T + B) + gamma), r += dt v, t += dt
//   kick  K(ds): dt = ds / (alpha U + gamma),       v += dt a(r)
//   leapfrog (Sec. 2.3): D(h/2) [K(h) D(h)]^(n-1) K(h) D(h/2), h = H/n
//   GBS step: Y' = Y + sum_k c_k (L_k(Y) - Y) over the divisions n_k = 2k,
//   c_k the weights of the extrapolation to h = 0 in h^2 (Sec. 2.3, 4.2),
// with B = U(r0) - T(v0) (B = -H, Sec. 2.1) and T in the centre-of-mass
// frame.  The reverse of a kick needs the transposed Jacobian of the
// accelerations, G sum_j M(d_ij) (m_i w_j - m_j w_i) with
// M(d) = (I - 3 d d^T / |d|^2) / |d|^3 (the tidal tensor; the force
// Hessian-vector product).
//
// One workgroup integrates (or reverses) one substep division of one GBS
// step with up to 1024 threads: up to 4 threads per body, each summing a
// contiguous chunk of the j-range, the chunks added in order through LDS.
// Positions and the adjoint weights of the j-bodies are broadcast from LDS,
// and U, T, the COM velocity and the d(dt) sums are workgroup sums in a
// fixed order.
#include "../../include/mstar.h"
#include "adjoint.h"

namespace mstar {
namespace {

// ---------------------------------------------------------------- reductions
template <int CTRL>
__device__ __forceinline__ double dppv(double v) {
    return __builtin_amdgcn_update_dpp(0.0, v, CTRL, 0xF, 0xF, false);
}
__device__ __forceinline__ double swap_sum(double v, bool wide) {
    const uint64_t u = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = (uint32_t)u, hi = (uint32_t)(u >> 32);
    uint32_t a0, a1, b0, b1;
    if (wide) {
        const auto l = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
        const auto h = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
        a0 = l[0]; b0 = l[1]; a1 = h[0]; b1 = h[1];
    } else {
        const auto l = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
        const auto h = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
        a0 = l[0]; b0 = l[1]; a1 = h[0]; b1 = h[1];
    }
    return __longlong_as_double((long long)(((uint64_t)a1 << 32) | a0)) +
           __longlong_as_double((long long)(((uint64_t)b1 << 32) | b0));
}
// sum over the 64 lanes of a wave, the same bits in every lane
__device__ __forceinline__ double wave_sum(double v) {
    v = v + dppv<0xB1>(v);
    v = v + dppv<0x4E>(v);
    v = v + dppv<0x141>(v);
    v = v + dppv<0x140>(v);
    v = swap_sum(v, false);
    return swap_sum(v, true);
}

constexpr int kMaxWaves = kAdjMaxN / 64;

// Sums of K values over the workgroup with one barrier: wave sums written to
// one of two alternating buffers, then every thread adds the wave partials in
// wave order.  A buffer is rewritten only two calls later, after the barrier
// of the call in between, which every thread reaches after its reads.
template <int K>
__device__ __forceinline__ void wave_partials(const double (&v)[K], double *red, int buf) {
    const int w = threadIdx.x >> 6;
    double *sh = red + buf * (4 * kMaxWaves);
#pragma unroll
    for (int c = 0; c < K; ++c) {
        const double s = wave_sum(v[c]);
        if ((threadIdx.x & 63) == 0) sh[c * kMaxWaves + w] = s;
    }
}
template <int K>
__device__ __forceinline__ void read_partials(double (&v)[K], const double *red, int &buf) {
    const int nw = blockDim.x >> 6;
    const double *sh = red + buf * (4 * kMaxWaves);
#pragma unroll
    for (int c = 0; c < K; ++c) {
        double s = 0.0;
        for (int q = 0; q < nw; ++q) s = s + sh[c * kMaxWaves + q];
        v[c] = s;
    }
    buf ^= 1;
}
template <int K>
__device__ __forceinline__ void block_sums(double (&v)[K], double *red, int &buf) {
    wave_partials<K>(v, red, buf);
    __syncthreads();
    read_partials<K>(v, red, buf);
}

__device__ __forceinline__ double rsqrt_refined(double x) {
    return rsqrt_f64(x);
}

struct LamA {
    double x, y, z, w;
};

// LDS of one division workgroup.  Between kicks, pos / la hold the j-bodies
// (positions + mass, adjoint weights); right after a j-loop they are reused
// for the per-thread partial sums of that loop.
struct AdjShared {
    d4 pos[kAdjMaxN];
    LamA la[kAdjMaxN];
    double red[2 * 4 * kMaxWaves];
};

// Thread layout: the first d.ext bodies take d.tpb + 1 threads, the others
// d.tpb (so that up to 1024 threads share the pair work evenly); thread
// (b, q) of a body with T threads owns body b and the q-th of T contiguous
// chunks of the j-range.  Per-body state is replicated in the T threads
// (they compute identical values); sums over bodies take the q = 0 threads
// only.  split (uniform) tells whether any body has more than one thread.
struct Lay {
    int b, q, T;
    bool live, lead, split;
    int jb, je;
};
__device__ __forceinline__ Lay layout(const AdjDev &d) {
    Lay L;
    const int t = (int)threadIdx.x, T1 = d.tpb + 1, wide = d.ext * T1;
    if (t < wide) {
        L.T = T1;
        L.b = t / T1;
        L.q = t - L.b * T1;
    } else {
        L.T = d.tpb;
        L.b = d.ext + (t - wide) / d.tpb;
        L.q = (t - wide) - (L.b - d.ext) * d.tpb;
    }
    L.live = L.b < d.n;
    L.lead = L.live && L.q == 0;
    L.split = d.tpb > 1 || d.ext > 0;
    const int c = (d.n + L.T - 1) / L.T;
    L.jb = min(d.n, L.q * c);
    L.je = min(d.n, L.jb + c);
    return L;
}

// Partial acceleration (without G) and phi of body i over j in [jb, je).
__device__ __forceinline__ void accel_part(const AdjShared &S, int jb, int je, int i, const d4 &r, double &ax,
                                           double &ay, double &az, double &ph) {
    ax = ay = az = ph = 0.0;
    for (int j = jb; j < je; ++j) {
        const d4 pj = S.pos[j];
        const double dx = pj.x - r.x, dy = pj.y - r.y, dz = pj.z - r.z;
        double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
        const bool self = j == i;
        r2 = self ? 1.0 : r2;
        const double mj = self ? 0.0 : pj.w;
        const double y = rsqrt_refined(r2);
        const double mr = mj * y;
        const double s = mr * (y * y);
        ph = ph + mr;
        ax = fma(s, dx, ax);
        ay = fma(s, dy, ay);
        az = fma(s, dz, az);
    }
}

// Partial acceleration (without G) and transposed-Jacobian product
// sum_j M(d_ij) (m_i w_j - m_j w_i) (without G) of body i over j in [jb, je).
// Also phi_i = sum_j m_j / r_ij and the mass term sum_j (w_j . d_ij) / r_ij^3
// (d a_j / d m_i applied to w_j, without G and sign).
__device__ __forceinline__ void accel_hvp_part(const AdjShared &S, int jb, int je, int i, const d4 &r, double mi,
                                               const LamA &wi, double &ax, double &ay, double &az, double &hx,
                                               double &hy, double &hz, double &ph, double &gm) {
    ax = ay = az = hx = hy = hz = ph = gm = 0.0;
    for (int j = jb; j < je; ++j) {
        const d4 pj = S.pos[j];
        const LamA wj = S.la[j];
        const double dx = pj.x - r.x, dy = pj.y - r.y, dz = pj.z - r.z;
        double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
        const bool self = j == i;
        r2 = self ? 1.0 : r2;
        const double mj = self ? 0.0 : pj.w;
        const double y = rsqrt_refined(r2);
        const double y2 = y * y;
        const double y3 = y2 * y;
        const double s = mj * y3;
        ax = fma(s, dx, ax);
        ay = fma(s, dy, ay);
        az = fma(s, dz, az);
        ph = fma(mj, y, ph);
        gm = fma(fma(dz, wj.z, fma(dy, wj.y, dx * wj.x)), y3, gm);   // d = 0 for the self pair
        const double m_i = self ? 0.0 : mi;   // the self pair contributes nothing
        const double qx = m_i * wj.x - mj * wi.x, qy = m_i * wj.y - mj * wi.y, qz = m_i * wj.z - mj * wi.z;
        const double dq = fma(dz, qz, fma(dy, qy, dx * qx));
        const double c = 3.0 * dq * y2;   // 3 (d . q) / |d|^2
        hx = fma(y3, qx - c * dx, hx);
        hy = fma(y3, qy - c * dy, hy);
        hz = fma(y3, qz - c * dz, hz);
    }
}

// Sum the T partials of each body in chunk order (identical in the T threads).
// The barrier before the writes ends every thread's reads of pos / la.
__device__ __forceinline__ void sum_parts(AdjShared &S, const Lay &L, int n, double &ax, double &ay, double &az,
                                          double &ph) {
    if (!L.split) return;
    __syncthreads();
    if (L.live) S.pos[L.q * n + L.b] = d4{ax, ay, az, ph};
    __syncthreads();
    if (L.live) {
        d4 t = S.pos[L.b];
        for (int q = 1; q < L.T; ++q) {
            const d4 u = S.pos[q * n + L.b];
            t = d4{t.x + u.x, t.y + u.y, t.z + u.z, t.w + u.w};
        }
        ax = t.x; ay = t.y; az = t.z; ph = t.w;
    }
}
// B = U(r0) - T(v0) for the state in (Yr, Yv); one workgroup.
__global__ __launch_bounds__(kAdjMaxN) void k_adj_init(AdjDev d, const d4 *Yr, const d4 *Yv, double *B) {
    __shared__ AdjShared S;
    const Lay L = layout(d);
    const double mi = L.live ? d.m[L.b] : 0.0;
    const double ml = L.lead ? mi : 0.0;
    const d4 r = L.live ? Yr[L.b] : d4{0.0, 0.0, 0.0, 0.0}, v = L.live ? Yv[L.b] : d4{0.0, 0.0, 0.0, 0.0};
    int rb = 0;
    if (L.lead) S.pos[L.b] = d4{r.x, r.y, r.z, mi};
    double s4[4] = {ml, ml * v.x, ml * v.y, ml * v.z};
    block_sums<4>(s4, S.red, rb);   // the barrier also publishes pos
    const double M = s4[0];
    const double bx = s4[1] / M, by = s4[2] / M, bz = s4[3] / M;
    double ax = 0.0, ay = 0.0, az = 0.0, ph = 0.0;
    if (L.live) accel_part(S, L.jb, L.je, L.b, r, ax, ay, az, ph);
    const double cx = v.x - bx, cy = v.y - by, cz = v.z - bz;
    double s2[2] = {L.live ? mi * ph : 0.0, ml * ((cx * cx + cy * cy) + cz * cz)};
    block_sums<2>(s2, S.red, rb);
    if (threadIdx.x == 0) *B = 0.5 * d.G * s2[0] - 0.5 * s2[1];
}

// One division per workgroup (blockIdx.x = k): the leapfrog with n_k = 2(k+1)
// substeps over H from (Yr, Yv, *Yt).  End state to Er[k], Ev[k], Et[k].  With
// STORE, the input of every kick (r), of every drift (v) and the op scalars
// are kept for the reverse pass.
template <bool STORE>
__global__ __launch_bounds__(kAdjMaxN) void k_adj_fwd(AdjDev d, const d4 *Yr, const d4 *Yv, const double *Yt,
                                                      double H) {
    __shared__ AdjShared S;
    const Lay L = layout(d);
    const int k = blockIdx.x, n = d.n;
    const int nsub = 2 * (k + 1);
    const int kb = k * (k + 1), db = k * (k + 1) + k, ob = 2 * k * (k + 1) + k;
    const double h = H / (double)nsub;
    const double mi = L.live ? d.m[L.b] : 0.0;
    const double ml = L.lead ? mi : 0.0;
    d4 r = L.live ? Yr[L.b] : d4{0.0, 0.0, 0.0, 0.0}, v = L.live ? Yv[L.b] : d4{0.0, 0.0, 0.0, 0.0};
    double t = *Yt;
    const double B = *d.B;
    int rb = 0;
    // total mass and COM velocity of the start state: kicks conserve momentum
    // exactly in the map being evaluated, so v_cm is constant over the division
    double s4[4] = {ml, ml * v.x, ml * v.y, ml * v.z};
    block_sums<4>(s4, S.red, rb);
    const double M = s4[0];
    const double bx = s4[1] / M, by = s4[2] / M, bz = s4[3] / M;
    for (int s = 0; s <= nsub; ++s) {
        // drift
        {
            const double ds = (s == 0 || s == nsub) ? 0.5 * h : h;
            if (STORE && L.lead) d.vst[(size_t)(db + s) * n + L.b] = v;
            const double cx = v.x - bx, cy = v.y - by, cz = v.z - bz;
            double s1[1] = {ml * ((cx * cx + cy * cy) + cz * cz)};
            block_sums<1>(s1, S.red, rb);
            const double T = 0.5 * s1[0];
            const double g = d.alpha * (T + B) + d.gamma;
            const double dt = ds / g;
            if (STORE && threadIdx.x == 0) {
                double *o = d.sc + (size_t)(ob + 2 * s) * kAdjOpScal;
                o[0] = dt; o[1] = g; o[2] = T; o[3] = bx; o[4] = by; o[5] = bz;
            }
            r = d4{r.x + dt * v.x, r.y + dt * v.y, r.z + dt * v.z, 0.0};
            t = t + dt;
        }
        if (s == nsub) break;
        // kick: publish positions; j-loop; U from the per-thread partials of
        // m_i phi_i; the acceleration partials of the T threads of a body
        // meet in la (unused by the forward pass)
        {
            if (STORE && L.lead) d.rst[(size_t)(kb + s) * n + L.b] = r;
            if (L.lead) S.pos[L.b] = d4{r.x, r.y, r.z, mi};
            __syncthreads();
            double ax = 0.0, ay = 0.0, az = 0.0, ph = 0.0;
            if (L.live) accel_part(S, L.jb, L.je, L.b, r, ax, ay, az, ph);
            double su[1] = {L.live ? mi * ph : 0.0};
            wave_partials<1>(su, S.red, rb);
            if (L.T > 1 && L.live) S.la[L.q * n + L.b] = LamA{ax, ay, az};
            __syncthreads();
            read_partials<1>(su, S.red, rb);
            if (L.T > 1 && L.live) {
                LamA a = S.la[L.b];
                for (int q = 1; q < L.T; ++q) {
                    const LamA u = S.la[q * n + L.b];
                    a = LamA{a.x + u.x, a.y + u.y, a.z + u.z};
                }
                ax = a.x; ay = a.y; az = a.z;
            }
            const double U = 0.5 * d.G * su[0];
            const double g = d.alpha * U + d.gamma;
            const double dt = h / g;
            if (STORE && threadIdx.x == 0) {
                double *o = d.sc + (size_t)(ob + 2 * s + 1) * kAdjOpScal;
                o[0] = dt; o[1] = g; o[2] = U;
            }
            v = d4{v.x + dt * (d.G * ax), v.y + dt * (d.G * ay), v.z + dt * (d.G * az), 0.0};
        }
    }
    if (L.lead) {
        d.Er[(size_t)k * n + L.b] = r;
        d.Ev[(size_t)k * n + L.b] = v;
    }
    if (threadIdx.x == 0) d.Et[k] = t;
}

// Y' = Y + sum_k c_k (L_k - Y) into (Or, Ov, Ot) (may alias Y).
__global__ void k_adj_combine(AdjDev d, const d4 *Yr, const d4 *Yv, const double *Yt, d4 *Or, d4 *Ov, double *Ot) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x, n = d.n;
    if (i < n) {
        const d4 r0 = Yr[i], v0 = Yv[i];
        double rx = 0.0, ry = 0.0, rz = 0.0, vx = 0.0, vy = 0.0, vz = 0.0;
        for (int k = 0; k < d.kf; ++k) {
            const d4 a = d.Er[(size_t)k * n + i], b = d.Ev[(size_t)k * n + i];
            const double c = d.c[k];
            rx = rx + c * (a.x - r0.x); ry = ry + c * (a.y - r0.y); rz = rz + c * (a.z - r0.z);
            vx = vx + c * (b.x - v0.x); vy = vy + c * (b.y - v0.y); vz = vz + c * (b.z - v0.z);
        }
        Or[i] = d4{r0.x + rx, r0.y + ry, r0.z + rz, 0.0};
        Ov[i] = d4{v0.x + vx, v0.y + vy, v0.z + vz, 0.0};
    }
    if (i == 0) {
        const double t0 = *Yt;
        double tt = 0.0;
        for (int k = 0; k < d.kf; ++k) tt = tt + d.c[k] * (d.Et[k] - t0);
        *Ot = t0 + tt;
    }
}

// Reverse of division k (blockIdx.x) from the cotangent c_k (Lr, Lv, Lt) of
// its end state, using what k_adj_fwd<true> stored; the cotangent of its
// start state goes to Sr[k], Sv[k], St[k] and the B part to SB[k].
__global__ __launch_bounds__(kAdjMaxN) void k_adj_rev(AdjDev d) {
    __shared__ AdjShared S;
    const Lay L = layout(d);
    const int k = blockIdx.x, n = d.n;
    const int nsub = 2 * (k + 1);
    const int kb = k * (k + 1), db = k * (k + 1) + k, ob = 2 * k * (k + 1) + k;
    const double mi = L.live ? d.m[L.b] : 0.0;
    const double ck = d.c[k];
    const double al = d.alpha;
    d4 lr{0.0, 0.0, 0.0, 0.0}, lv{0.0, 0.0, 0.0, 0.0};
    if (L.live) {
        const d4 a = d.Lr[L.b], b = d.Lv[L.b];
        lr = d4{ck * a.x, ck * a.y, ck * a.z, 0.0};
        lv = d4{ck * b.x, ck * b.y, ck * b.z, 0.0};
    }
    const double lt = ck * *d.Lt;
    double lB = 0.0, lm = 0.0;
    int rb = 0;
    for (int s = nsub; s >= 0; --s) {
        // reverse drift s: r' = r + dt v, t' = t + dt, dt = ds / (alpha (T(v) + B) + gamma)
        {
            const double *o = d.sc + (size_t)(ob + 2 * s) * kAdjOpScal;
            const double dt = o[0], g = o[1];
            const double bx = o[3], by = o[4], bz = o[5];
            const d4 v = L.live ? d.vst[(size_t)(db + s) * n + L.b] : d4{0.0, 0.0, 0.0, 0.0};
            double s1[1] = {L.lead ? (lr.x * v.x + lr.y * v.y) + lr.z * v.z : 0.0};
            block_sums<1>(s1, S.red, rb);
            const double ldt = s1[0] + lt;
            const double lT = ldt * (-(dt / g) * al);
            lB = lB + lT;
            if (L.live) {
                // T = sum m_i |v_i - v_bar|^2 / 2: dT/dm_i = |v_i - v_bar|^2 / 2 (sum m (v - v_bar) = 0)
                const double cx = v.x - bx, cy = v.y - by, cz = v.z - bz;
                lm = lm + lT * (0.5 * ((cx * cx + cy * cy) + cz * cz));
                lv = d4{lv.x + dt * lr.x + lT * (mi * (v.x - bx)), lv.y + dt * lr.y + lT * (mi * (v.y - by)),
                        lv.z + dt * lr.z + lT * (mi * (v.z - bz)), 0.0};
            }
        }
        if (s == 0) break;
        // reverse kick s-1: v' = v + dt a(r), dt = h / (alpha U(r) + gamma)
        {
            const double *o = d.sc + (size_t)(ob + 2 * (s - 1) + 1) * kAdjOpScal;
            const double dt = o[0], g = o[1];
            const d4 r = L.live ? d.rst[(size_t)(kb + s - 1) * n + L.b] : d4{0.0, 0.0, 0.0, 0.0};
            const LamA wi{dt * lv.x, dt * lv.y, dt * lv.z, 0.0};
            if (L.lead) {
                S.pos[L.b] = d4{r.x, r.y, r.z, mi};
                S.la[L.b] = wi;
            }
            __syncthreads();
            double ax = 0.0, ay = 0.0, az = 0.0, hx = 0.0, hy = 0.0, hz = 0.0, ph = 0.0, gq = 0.0;
            if (L.live) accel_hvp_part(S, L.jb, L.je, L.b, r, mi, wi, ax, ay, az, hx, hy, hz, ph, gq);
            // lambda_dt = sum_i lambda_v,i . a_i, from the per-thread partials
            double s1[1] = {L.live ? (lv.x * (d.G * ax) + lv.y * (d.G * ay)) + lv.z * (d.G * az) : 0.0};
            wave_partials<1>(s1, S.red, rb);
            if (L.split) {
                __syncthreads();   // every j-loop has finished reading pos / la
                if (L.live) {
                    S.pos[L.q * n + L.b] = d4{ax, ay, az, ph};
                    S.la[L.q * n + L.b] = LamA{hx, hy, hz, gq};
                }
            }
            __syncthreads();
            read_partials<1>(s1, S.red, rb);
            if (L.T > 1 && L.live) {
                d4 a = S.pos[L.b];
                LamA hh = S.la[L.b];
                for (int q = 1; q < L.T; ++q) {
                    const d4 u = S.pos[q * n + L.b];
                    const LamA w = S.la[q * n + L.b];
                    a = d4{a.x + u.x, a.y + u.y, a.z + u.z, a.w + u.w};
                    hh = LamA{hh.x + w.x, hh.y + w.y, hh.z + w.z, hh.w + w.w};
                }
                ax = a.x; ay = a.y; az = a.z; ph = a.w;
                hx = hh.x; hy = hh.y; hz = hh.z; gq = hh.w;
            }
            ax = d.G * ax; ay = d.G * ay; az = d.G * az;
            hx = d.G * hx; hy = d.G * hy; hz = d.G * hz;
            const double lU = s1[0] * (-(dt / g) * al);
            if (L.live) {
                lr = d4{lr.x + lU * (mi * ax) + hx, lr.y + lU * (mi * ay) + hy, lr.z + lU * (mi * az) + hz, 0.0};
                // dU/dm_i = G phi_i; a_j depends on m_i through G m_i d_ji / r^3
                lm = lm + (lU * (d.G * ph) - d.G * gq);
            }
        }
    }
    if (L.lead) {
        d.Sr[(size_t)k * n + L.b] = lr;
        d.Sv[(size_t)k * n + L.b] = lv;
        d.Sm[(size_t)k * n + L.b] = lm;
    }
    if (threadIdx.x == 0) {
        d.St[k] = lt;
        d.SB[k] = lB;
    }
}

// Cotangent of a step's start state: (1 - sum c) L + sum_k S_k, in place in
// (Lr, Lv, Lt); the B parts are added to *LB.
__global__ void k_adj_combine_rev(AdjDev d) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x, n = d.n;
    double cs = 0.0;
    for (int k = 0; k < d.kf; ++k) cs = cs + d.c[k];
    const double keep = 1.0 - cs;
    if (i < n) {
        const d4 a = d.Lr[i], b = d.Lv[i];
        double rx = keep * a.x, ry = keep * a.y, rz = keep * a.z, vx = keep * b.x, vy = keep * b.y, vz = keep * b.z;
        for (int k = 0; k < d.kf; ++k) {
            const d4 p = d.Sr[(size_t)k * n + i], q = d.Sv[(size_t)k * n + i];
            rx = rx + p.x; ry = ry + p.y; rz = rz + p.z;
            vx = vx + q.x; vy = vy + q.y; vz = vz + q.z;
        }
        d.Lr[i] = d4{rx, ry, rz, 0.0};
        d.Lv[i] = d4{vx, vy, vz, 0.0};
        double mm = d.Lm[i];
        for (int k = 0; k < d.kf; ++k) mm = mm + d.Sm[(size_t)k * n + i];
        d.Lm[i] = mm;
    }
    if (i == 0) {
        double tt = keep * *d.Lt, bb = 0.0;
        for (int k = 0; k < d.kf; ++k) {
            tt = tt + d.St[k];
            bb = bb + d.SB[k];
        }
        *d.Lt = tt;
        *d.LB = *d.LB + bb;
    }
}

// Gradient with respect to the initial state: the chain through
// B = U(r0) - T(v0) added to the propagated cotangent.  One workgroup.
__global__ __launch_bounds__(kAdjMaxN) void k_adj_finish(AdjDev d, const d4 *Yr, const d4 *Yv, double *gx,
                                                         double *gv, double *gm) {
    __shared__ AdjShared S;
    const Lay L = layout(d);
    const int n = d.n;
    const double mi = L.live ? d.m[L.b] : 0.0;
    const double ml = L.lead ? mi : 0.0;
    const d4 r = L.live ? Yr[L.b] : d4{0.0, 0.0, 0.0, 0.0}, v = L.live ? Yv[L.b] : d4{0.0, 0.0, 0.0, 0.0};
    int rb = 0;
    if (L.lead) S.pos[L.b] = d4{r.x, r.y, r.z, mi};
    double s4[4] = {ml, ml * v.x, ml * v.y, ml * v.z};
    block_sums<4>(s4, S.red, rb);   // the barrier also publishes pos
    const double M = s4[0];
    const double bx = s4[1] / M, by = s4[2] / M, bz = s4[3] / M;
    double ax = 0.0, ay = 0.0, az = 0.0, ph = 0.0;
    if (L.live) accel_part(S, L.jb, L.je, L.b, r, ax, ay, az, ph);
    sum_parts(S, L, n, ax, ay, az, ph);
    ax = d.G * ax; ay = d.G * ay; az = d.G * az;
    const double lB = *d.LB;
    if (L.lead) {
        const d4 a = d.Lr[L.b], b = d.Lv[L.b];
        gx[3 * L.b] = a.x + lB * (mi * ax);
        gx[3 * L.b + 1] = a.y + lB * (mi * ay);
        gx[3 * L.b + 2] = a.z + lB * (mi * az);
        gv[3 * L.b] = b.x - lB * (mi * (v.x - bx));
        gv[3 * L.b + 1] = b.y - lB * (mi * (v.y - by));
        gv[3 * L.b + 2] = b.z - lB * (mi * (v.z - bz));
        if (gm) {   // B = U(r0) - T(v0): dB/dm_i = G phi_i - |v_i - v_bar|^2 / 2
            const double cx = v.x - bx, cy = v.y - by, cz = v.z - bz;
            gm[L.b] = d.Lm[L.b] + lB * (d.G * ph - 0.5 * ((cx * cx + cy * cy) + cz * cz));
        }
    }
}

// Stage kernel: h_i = G sum_j M(d_ij) (m_i w_j - m_j w_i) for any N (one thread
// per i, j-bodies from global memory).
__global__ void k_force_hvp(int n, double G, const double *m, const double *x, const double *w, double *out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double rx = x[3 * i], ry = x[3 * i + 1], rz = x[3 * i + 2];
    const double mi = m[i], wx = w[3 * i], wy = w[3 * i + 1], wz = w[3 * i + 2];
    double hx = 0.0, hy = 0.0, hz = 0.0;
    for (int j = 0; j < n; ++j) {
        if (j == i) continue;
        const double dx = x[3 * j] - rx, dy = x[3 * j + 1] - ry, dz = x[3 * j + 2] - rz;
        const double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
        const double y = rsqrt_refined(r2);
        const double y2 = y * y, y3 = y2 * y;
        const double mj = m[j];
        const double qx = mi * w[3 * j] - mj * wx, qy = mi * w[3 * j + 1] - mj * wy, qz = mi * w[3 * j + 2] - mj * wz;
        const double dq = fma(dz, qz, fma(dy, qy, dx * qx));
        const double c = 3.0 * dq * y2;
        hx = fma(y3, qx - c * dx, hx);
        hy = fma(y3, qy - c * dy, hy);
        hz = fma(y3, qz - c * dz, hz);
    }
    out[3 * i] = G * hx;
    out[3 * i + 1] = G * hy;
    out[3 * i + 2] = G * hz;
}

__global__ void k_adj_pack(int n, const double *x, d4 *o, double t, double *ot) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) o[i] = d4{x[3 * i], x[3 * i + 1], x[3 * i + 2], 0.0};
    if (ot && i == 0) *ot = t;
}
__global__ void k_adj_unpack(int n, const d4 *a, double *x) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        x[3 * i] = a[i].x;
        x[3 * i + 1] = a[i].y;
        x[3 * i + 2] = a[i].z;
    }
}
__global__ void k_adj_zero(double *p) {
    if (threadIdx.x == 0) *p = 0.0;
}
__global__ void k_adj_zero_n(int n, double *p) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}
__global__ void k_adj_copy(int n, const d4 *a, const d4 *b, const double *t, d4 *oa, d4 *ob, double *ot) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        oa[i] = a[i];
        ob[i] = b[i];
    }
    if (i == 0) *ot = *t;
}

int threads_for(const AdjDev &d) { return ((d.n * d.tpb + d.ext + 63) / 64) * 64; }

}  // namespace

void launch_adj_init(const AdjDev &d, hipStream_t s, const d4 *Yr, const d4 *Yv) {
    k_adj_init<<<1, threads_for(d), 0, s>>>(d, Yr, Yv, d.B);
}
void launch_adj_fwd(const AdjDev &d, hipStream_t s, const d4 *Yr, const d4 *Yv, const double *Yt, double H,
                    bool store) {
    if (store) k_adj_fwd<true><<<d.kf, threads_for(d), 0, s>>>(d, Yr, Yv, Yt, H);
    else k_adj_fwd<false><<<d.kf, threads_for(d), 0, s>>>(d, Yr, Yv, Yt, H);
}
void launch_adj_combine(const AdjDev &d, hipStream_t s, const d4 *Yr, const d4 *Yv, const double *Yt, d4 *Or,
                        d4 *Ov, double *Ot) {
    k_adj_combine<<<(d.n + 255) / 256, 256, 0, s>>>(d, Yr, Yv, Yt, Or, Ov, Ot);
}
void launch_adj_rev(const AdjDev &d, hipStream_t s) { k_adj_rev<<<d.kf, threads_for(d), 0, s>>>(d); }
void launch_adj_combine_rev(const AdjDev &d, hipStream_t s) {
    k_adj_combine_rev<<<(d.n + 255) / 256, 256, 0, s>>>(d);
}
void launch_adj_finish(const AdjDev &d, hipStream_t s, const d4 *Yr, const d4 *Yv, double *gx, double *gv,
                       double *gm) {
    k_adj_finish<<<1, threads_for(d), 0, s>>>(d, Yr, Yv, gx, gv, gm);
}
void launch_adj_zero_n(hipStream_t s, int n, double *p) { k_adj_zero_n<<<(n + 255) / 256, 256, 0, s>>>(n, p); }
void launch_force_hvp(hipStream_t s, int n, double G, const double *m, const double *x, const double *w,
                      double *out) {
    k_force_hvp<<<(n + 127) / 128, 128, 0, s>>>(n, G, m, x, w, out);
}
void launch_adj_pack(hipStream_t s, int n, const double *x, d4 *o, double t, double *ot) {
    k_adj_pack<<<(n + 255) / 256, 256, 0, s>>>(n, x, o, t, ot);
}
void launch_adj_unpack(hipStream_t s, int n, const d4 *a, double *x) {
    k_adj_unpack<<<(n + 255) / 256, 256, 0, s>>>(n, a, x);
}
void launch_adj_zero(hipStream_t s, double *p) { k_adj_zero<<<1, 64, 0, s>>>(p); }
void launch_adj_copy(hipStream_t s, int n, const d4 *a, const d4 *b, const double *t, d4 *oa, d4 *ob, double *ot) {
    k_adj_copy<<<(n + 255) / 256, 256, 0, s>>>(n, a, b, t, oa, ob, ot);
}

}  // namespace mstar
