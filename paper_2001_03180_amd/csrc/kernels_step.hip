// O(N) kernels of the GBS step: division set-up, the drift and kick
// operators of the regularised leapfrog (paper Sec. 2.1-2.3), Neville-Aitken
// extrapolation with the error measure of eq. gbs-criterion, step control
// (eq. hnext), the end-time clip (Sec. 2.4) and state transforms.
//
// Each division integrates increments from the step's start state (X = X0 +
// dX, V = V0 + dV, t = t0 + tau), so the extrapolation works on small
// numbers.  Between kernels the only cross-body quantities are the force
// function U and the kinetic energy T; every workgroup that needs them
// reduces the same per-workgroup partials in the same order, so all
// workgroups agree bit for bit without an extra launch.
#include "common.h"

namespace mstar {

__global__ __launch_bounds__(kWG) void k_div_init(Dev d, int ndiv, int base) {
    const int slot = blockIdx.y;
    const int v = blockIdx.x * kWG + threadIdx.x;
    const int n = d.n;
    if (slot >= ndiv) return;
    if (v < n) {
        const size_t o = (size_t)slot * n + v;
        d.P[o] = d.P[(size_t)base * n + v];
        d.Vt[o] = d.Vt[(size_t)base * n + v];
        d.dX[o] = d4{0.0, 0.0, 0.0, 0.0};
        d.dV[o] = d4{0.0, 0.0, 0.0, 0.0};
        d.dP[o] = d4{0.0, 0.0, 0.0, 0.0};
        d.dVt[o] = d4{0.0, 0.0, 0.0, 0.0};
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) d.dscal[slot] = DivScal{};
}

void launch_div_init(const Dev &d, hipStream_t s, int ndiv, int base_slot) {
    dim3 grid((d.n + kWG - 1) / kWG, ndiv);
    k_div_init<<<grid, kWG, 0, s>>>(d, ndiv, base_slot);
}

// Drift D(ds): dt = ds / (alpha (T + B) + beta w + gamma); X += dt V, after
// V has taken the preceding kick (see k_kick);
// positions += dt v (kept as increments dP from the start positions,
// P = P0 + dP); t += dt; r_cm += dt v_cm.  With OM (TTL), the w increment of
// the preceding kick is completed here: dw += dt_kick sum_wg wpart, summed by
// every workgroup in the same order; block 0 records the result in dwn (the
// kick copies it to dw before it overwrites dtk and wpart).  With EX (an
// external field) the preceding kick's work on B is completed the same way:
// dB -= dt_kick sum_wg bpart, recorded in dBn; r_cm moves with v_cm + dv_cm.
template <bool OM, bool EX>
__global__ __launch_bounds__(kWG) void k_drift(Dev d, SlotList sl, Ttl tr) {
    __shared__ double sh[3][kWG / 64];
    const int ai = blockIdx.y;
    const int slot = sl.slot[ai];
    const int n = d.n;
    // the body's operands first: their loads overlap the reductions below
    const int v = blockIdx.x * kWG + threadIdx.x;
    const size_t o = (size_t)slot * n + v;
    const bool live = v < n;
    const int par = live ? d.parent[v] : -1;
    const bool edge = par >= 0;
    const bool after_kick = !sl.first[ai];
    d4 V0{0.0, 0.0, 0.0, 0.0}, dV = V0, dX = V0, vt = V0, p0 = V0, dp = V0, av = V0, ap = V0;
    if (edge) {
        V0 = d.V0[v]; dV = d.dV[o]; dX = d.dX[o];
        if (after_kick) { av = d.akick[o]; ap = d.akick[(size_t)slot * n + par]; }
    }
    if (live) { vt = d.Vt[o]; p0 = d.P[(size_t)kBaseSlot * n + v]; dp = d.dP[o]; }
    double T, w = d.sys->w, B = d.sys->B;
    if (sl.first[ai]) {
        T = d.ctl->T0;
    } else {
        const double *tp = d.Tpart + (size_t)slot * d.nkwg4;
        double t = 0.0;
        for (int k = threadIdx.x; k < d.nkwg4; k += kWG) t = t + tp[k];
        T = 0.5 * block_sum1<kWG>(t, sh[0]);
        if constexpr (OM) {
            const double *wp = d.wpart + (size_t)slot * d.nkwg4;
            double a = 0.0;
            for (int k = threadIdx.x; k < d.nkwg4; k += kWG) a = a + wp[k];
            const double S = block_sum1<kWG>(a, sh[1]);
            const DivScal &q = d.dscal[slot];
            const double dw = q.dw + q.dtk * S;
            w = w + dw;
            if (blockIdx.x == 0 && threadIdx.x == 0) d.dscal[slot].dwn = dw;
        }
        if constexpr (EX) {
            const double *bp = d.bpart + (size_t)slot * d.nkwg4;
            double a = 0.0;
            for (int k = threadIdx.x; k < d.nkwg4; k += kWG) a = a + bp[k];
            const double S = block_sum1<kWG>(a, sh[2]);
            const DivScal &q = d.dscal[slot];
            const double dB = q.dB - q.dtk * S;
            B = B + dB;
            if (blockIdx.x == 0 && threadIdx.x == 0) d.dscal[slot].dBn = dB;
        }
    }
    const double H = d.ctl->H;
    const double h = H / (double)sl.nsub[ai];
    const double ds = sl.half[ai] ? 0.5 * h : h;
    const double dt = ds / ((tr.alpha * (T + B) + tr.beta * w) + tr.gamma);
    if (edge) {
        if (after_kick) {   // the preceding kick's update of the edge velocity
            const double dtk = d.dscal[slot].dtk;
            dV.x = dV.x + dtk * (av.x - ap.x);
            dV.y = dV.y + dtk * (av.y - ap.y);
            dV.z = dV.z + dtk * (av.z - ap.z);
            d.dV[o] = dV;
        }
        dX.x = dX.x + dt * (V0.x + dV.x);
        dX.y = dX.y + dt * (V0.y + dV.y);
        dX.z = dX.z + dt * (V0.z + dV.z);
        d.dX[o] = dX;
    }
    if (live) {
        dp.x = dp.x + dt * vt.x;
        dp.y = dp.y + dt * vt.y;
        dp.z = dp.z + dt * vt.z;
        d.dP[o] = dp;
        d.P[o] = d4{p0.x + dp.x, p0.y + dp.y, p0.z + dp.z, p0.w};
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        DivScal &q = d.dscal[slot];
        q.tau = q.tau + dt;
        if constexpr (EX) {
            for (int c = 0; c < 3; ++c) q.drcm[c] = q.drcm[c] + dt * (d.sys->vcm[c] + q.dvcm[c]);
        } else {
            for (int c = 0; c < 3; ++c) q.drcm[c] = q.drcm[c] + dt * d.sys->vcm[c];
        }
    }
}

void launch_drift(const Dev &d, hipStream_t s, const SlotList &sl, Ttl tr, bool ex) {
    dim3 grid((d.n + kWG - 1) / kWG, sl.nact);
    if (ex) k_drift<false, true><<<grid, kWG, 0, s>>>(d, sl, tr);
    else if (tr.beta != 0.0) k_drift<true, false><<<grid, kWG, 0, s>>>(d, sl, tr);
    else k_drift<false, false><<<grid, kWG, 0, s>>>(d, sl, tr);
}

// External perturbation (Sec. 2.1) at the bodies' positions r_i = r_cm + P_i
// of every slot in the list (at_start: the start state, r_cm = the system's):
//   f_i = g + sum_k G M_k (R_k - r_i) / (|R_k - r_i|^2 + b_k^2)^(3/2),
// stored per body, and per-workgroup partials of sum m_i f_i and of
// sum m_i f_i . v_i (COM-frame velocities; the start state's dB/dt).
__global__ __launch_bounds__(kWG) void k_ext(Dev d, SlotList sl, int at_start) {
    __shared__ double sh[4][kWG / 64];
    const int slot = sl.slot[blockIdx.y];
    const int n = d.n;
    const int v = blockIdx.x * kWG + threadIdx.x;
    const size_t o = (size_t)slot * n + v;
    const ExtField &e = *d.ext;
    double rc[3];
    for (int c = 0; c < 3; ++c) rc[c] = at_start ? d.sys->rcm[c] : d.sys->rcm[c] + d.dscal[slot].drcm[c];
    double mfx = 0.0, mfy = 0.0, mfz = 0.0, mfv = 0.0;
    if (v < n) {
        const d4 P = d.P[o], W = d.Vt[o];
        const double rx = rc[0] + P.x, ry = rc[1] + P.y, rz = rc[2] + P.z;
        double fx = e.g[0], fy = e.g[1], fz = e.g[2];
        for (int k = 0; k < e.np; ++k) {
            const double dx = e.pt[k][1] - rx, dy = e.pt[k][2] - ry, dz = e.pt[k][3] - rz;
            const double s2 = ((dx * dx + dy * dy) + dz * dz) + e.pt[k][4];
            const double w = e.pt[k][0] / (s2 * sqrt(s2));
            fx = fx + w * dx; fy = fy + w * dy; fz = fz + w * dz;
        }
        d.fext[o] = d4{fx, fy, fz, 0.0};
        mfx = P.w * fx; mfy = P.w * fy; mfz = P.w * fz;
        mfv = P.w * ((fx * W.x + fy * W.y) + fz * W.z);
    }
    const double a = block_sum1<kWG>(mfx, sh[0]);
    const double b = block_sum1<kWG>(mfy, sh[1]);
    const double c = block_sum1<kWG>(mfz, sh[2]);
    const double q = block_sum1<kWG>(mfv, sh[3]);
    if (threadIdx.x == 0) d.fpart[(size_t)slot * d.nkwg4 + blockIdx.x] = d4{a, b, c, q};
}

void launch_ext(const Dev &d, hipStream_t s, const SlotList &sl, int at_start) {
    dim3 grid((d.n + kWG - 1) / kWG, sl.nact);
    k_ext<<<grid, kWG, 0, s>>>(d, sl, at_start);
}

// 1 / total mass, for the external field's acceleration of the centre of mass.
__global__ __launch_bounds__(kTreeWG) void k_ext_minv(Dev d) {
    __shared__ double sh[kTreeWG];
    double s = 0.0;
    for (int u = threadIdx.x; u < d.n; u += kTreeWG) s = s + d.m[u];
    const double M = block_sum<kTreeWG>(s, sh);
    if (threadIdx.x == 0) d.ext->Minv = 1.0 / M;
}

void launch_ext_minv(const Dev &d, hipStream_t s) { k_ext_minv<<<1, kTreeWG, 0, s>>>(d); }

// Kick K(ds): dt = ds / (alpha U + beta Omega + gamma); COM-frame velocities
// v += dt a (as increments dVt, v = v0 + dVt); partial sums of m |v|^2 for the
// next drift.  The edge velocities V_v += dt (a_v - a_parent(v)) are updated
// by that drift from the accelerations stored here and dt (kept in dtk): each
// body's acceleration is then summed from its j-split partials once, not once
// more for every child.  With OM (TTL)
// also per-workgroup partials of sum_i grad_i Omega . (v_i_old + v_i_new)/2;
// the next drift scales them by dt (kept in dtk) into w.  With EX (external
// field f from k_ext): every body takes a_i + f_i, the COM-frame velocities
// take dt (a_i + f_i - F/M) with F = sum m f, v_cm takes dt F/M (in dvcm),
// and per-workgroup partials of sum m_i f_i . (v_i_old + v_i_new)/2 give the
// work on B, which the next drift scales by dt.
template <bool OM, bool EX>
__global__ __launch_bounds__(kWG) void k_kick(Dev d, SlotList sl, FLay fl, double G, Ttl tr) {
    __shared__ double sh[8][kWG / 64];
    __shared__ d4 ra[kWG], rc[OM ? kWG : 1];
    const int ai = blockIdx.y;
    const int slot = sl.slot[ai];
    const int n = d.n;
    // four threads per body, each a fixed quarter of the split partials; all
    // loads that do not depend on the step length are issued first
    const int v = blockIdx.x * (kWG / 4) + (threadIdx.x >> 2);
    const int part = threadIdx.x & 3;
    const bool live = v < n, lead = live && part == 0;
    const size_t prow = (size_t)slot * d.nsplit_max * n;
    const size_t o = (size_t)slot * n + v;
    const d4 *pp = d.part + prow;
    // the sums are plain scalars and the other locals start from literal
    // zeros: copies of one zero struct let the compiler merge the lead
    // lanes' loads with reads of that struct, which then lives in scratch
    double sx = 0.0, sy = 0.0, sz = 0.0, ox = 0.0, oy = 0.0, oz = 0.0;
    if (live) {
        force_sum(d, pp, fl, slot, ai, v, part, 4, sx, sy, sz);
        if constexpr (OM) {   // the TTL kernel is always the pairwise one
            for (int sp = part; sp < fl.nparts; sp += 4) {
                const d4 t3 = d.opart[prow + (size_t)sp * n + v];
                ox = ox + t3.x; oy = oy + t3.y; oz = oz + t3.z;
            }
        }
    }
    d4 sa{sx, sy, sz, 0.0}, so{ox, oy, oz, 0.0};
    d4 dvt{0.0, 0.0, 0.0, 0.0}, v0{0.0, 0.0, 0.0, 0.0}, vo{0.0, 0.0, 0.0, 0.0}, fe{0.0, 0.0, 0.0, 0.0};
    double mv = 0.0, mo = 0.0;
    if (lead) {
        dvt = d.dVt[o];
        v0 = d.Vt[(size_t)kBaseSlot * n + v];
        mv = d.P[o].w;
        if constexpr (OM) { vo = d.Vt[o]; mo = d.mo[v]; }
        if constexpr (EX) { vo = d.Vt[o]; fe = d.fext[o]; }
    }
    ra[threadIdx.x] = sa;
    if constexpr (OM) rc[threadIdx.x] = so;
    int cnt = 0;
    const double *up = force_upart(d, fl, slot, &cnt);
    double u = 0.0;
    for (int k = threadIdx.x; k < cnt; k += kWG) u = u + up[k];
    const double U = 0.5 * G * block_sum1<kWG>(u, sh[0]);   // its barrier also publishes ra, rc
    double Om = 0.0;
    if constexpr (OM) {
        const double *op = d.Opart + (size_t)slot * d.nib * d.nsplit_max;
        double q = 0.0;
        for (int k = threadIdx.x; k < cnt; k += kWG) q = q + op[k];
        Om = 0.5 * G * block_sum1<kWG>(q, sh[1]);
    }
    double Fx = 0.0, Fy = 0.0, Fz = 0.0;
    if constexpr (EX) {
        const d4 *fp = d.fpart + (size_t)slot * d.nkwg4;
        double a = 0.0, b = 0.0, c = 0.0;
        for (int k = threadIdx.x; k < d.nkwg; k += kWG) {
            const d4 t = fp[k];
            a = a + t.x; b = b + t.y; c = c + t.z;
        }
        const double Minv = d.ext->Minv;
        Fx = block_sum1<kWG>(a, sh[4]) * Minv;
        Fy = block_sum1<kWG>(b, sh[5]) * Minv;
        Fz = block_sum1<kWG>(c, sh[6]) * Minv;
    }
    const double H = d.ctl->H;
    const double ds = H / (double)sl.nsub[ai];
    const double dt = ds / ((tr.alpha * U + tr.beta * Om) + tr.gamma);
    double tl = 0.0, wl = 0.0;
    if (lead) {
        for (int k = 1; k < 4; ++k) {
            const d4 t = ra[threadIdx.x + k];
            sa.x = sa.x + t.x; sa.y = sa.y + t.y; sa.z = sa.z + t.z;
            if constexpr (OM) {
                const d4 t3 = rc[threadIdx.x + k];
                so.x = so.x + t3.x; so.y = so.y + t3.y; so.z = so.z + t3.z;
            }
        }
        double ax = G * sa.x, ay = G * sa.y, az = G * sa.z;
        if constexpr (EX) { ax = ax + fe.x; ay = ay + fe.y; az = az + fe.z; }
        d.akick[o] = d4{ax, ay, az, 0.0};   // the edge velocities take it in the next drift
        if constexpr (EX) {
            dvt.x = dvt.x + dt * (ax - Fx);
            dvt.y = dvt.y + dt * (ay - Fy);
            dvt.z = dvt.z + dt * (az - Fz);
        } else {
            dvt.x = dvt.x + dt * ax;
            dvt.y = dvt.y + dt * ay;
            dvt.z = dvt.z + dt * az;
        }
        d.dVt[o] = dvt;
        const d4 vt{v0.x + dvt.x, v0.y + dvt.y, v0.z + dvt.z, 0.0};
        if constexpr (EX)
            wl = mv * ((fe.x * (0.5 * (vo.x + vt.x)) + fe.y * (0.5 * (vo.y + vt.y))) + fe.z * (0.5 * (vo.z + vt.z)));
        if constexpr (OM) {
            const double gm = G * mo;
            const double gx = gm * so.x, gy = gm * so.y, gz = gm * so.z;
            wl = (gx * (0.5 * (vo.x + vt.x)) + gy * (0.5 * (vo.y + vt.y))) + gz * (0.5 * (vo.z + vt.z));
        }
        d.Vt[o] = vt;
        tl = mv * ((vt.x * vt.x + vt.y * vt.y) + vt.z * vt.z);
    }
    const double ts = block_sum1<kWG>(tl, sh[2]);
    if (threadIdx.x == 0) d.Tpart[(size_t)slot * d.nkwg4 + blockIdx.x] = ts;
    if constexpr (OM) {
        const double ws = block_sum1<kWG>(wl, sh[3]);
        if (threadIdx.x == 0) d.wpart[(size_t)slot * d.nkwg4 + blockIdx.x] = ws;
    }
    if constexpr (EX) {
        const double bs = block_sum1<kWG>(wl, sh[7]);
        if (threadIdx.x == 0) d.bpart[(size_t)slot * d.nkwg4 + blockIdx.x] = bs;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        DivScal &q = d.dscal[slot];
        if constexpr (OM) q.dw = q.dwn;
        if constexpr (EX) {
            q.dB = q.dBn;
            q.dvcm[0] = q.dvcm[0] + dt * Fx;
            q.dvcm[1] = q.dvcm[1] + dt * Fy;
            q.dvcm[2] = q.dvcm[2] + dt * Fz;
        }
        q.dtk = dt;
    }
}

void launch_kick(const Dev &d, hipStream_t s, const SlotList &sl, const FLay &f, double G, Ttl tr, bool ex) {
    dim3 grid((d.n + kWG / 4 - 1) / (kWG / 4), sl.nact);
    if (ex) k_kick<false, true><<<grid, kWG, 0, s>>>(d, sl, f, G, tr);
    else if (tr.beta != 0.0) k_kick<true, false><<<grid, kWG, 0, s>>>(d, sl, f, G, tr);
    else k_kick<false, false><<<grid, kWG, 0, s>>>(d, sl, f, G, tr);
}

// Step length of this attempt with the end-time clip of Sec. 2.4: the
// predicted time after the step, t + H/g with g = alpha U + beta Omega + gamma,
// must not pass t_end (nor may the step point away from it); otherwise
// ds = g (t_end - t).  With TTL also dw/dt at the start state from the
// partials of the start-state force reduction.
__global__ void k_set_h(Dev d, double H, double t_end, int clip, Ttl tr, int from_ctl) {
    Ctl &c = *d.ctl;
    if (from_ctl) H = c.h_next;   // the step proposed by the previous attempt (or set by k_put_hnext)
    {   // T of the start state from the per-workgroup partials left by the commit
        const double *tp = d.Tpart + (size_t)kBaseSlot * d.nkwg4;
        double t = 0.0;
        for (int k = 0; k < d.nkwg; ++k) t = t + tp[k];
        c.T0 = 0.5 * t;
    }
    double dw = 0.0;
    if (tr.beta != 0.0) {
        const double *wp = d.wpart + (size_t)kBaseSlot * d.nkwg4;
        for (int k = 0; k < d.nkwg; ++k) dw = dw + wp[k];
    }
    c.dw0 = dw;
    const double gk = (tr.alpha * c.U0 + tr.beta * c.Om0) + tr.gamma;
    c.gk0 = gk;
    c.clipped = 0;
    if (clip) {
        const double rem = t_end - d.sys->t;
        const double dt_est = H / gk;
        if (dt_est / rem > 1.0 || dt_est / rem < 0.0) {
            H = gk * rem;
            c.clipped = 1;
        }
    }
    c.H = H;
    c.t_est = d.sys->t + H / gk;
}

void launch_set_h(const Dev &d, hipStream_t s, double H, double t_end, int clip, Ttl tr, int from_ctl) {
    k_set_h<<<1, 1, 0, s>>>(d, H, t_end, clip, tr, from_ctl);
}

// Proposed step of the next attempt, for a driver whose attempt reads it from
// the control block (a replayed graph cannot take it as an argument).
__global__ void k_put_hnext(Dev d, double H) { d.ctl->h_next = H; }
void launch_put_hnext(const Dev &d, hipStream_t s, double H) { k_put_hnext<<<1, 1, 0, s>>>(d, H); }

// In-place Aitken-Neville tableau over KF divisions n_k = 2(k+1); on return
// p[k] = T_{k,k}.
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

__device__ __forceinline__ double norm3(double x, double y, double z) { return sqrt((x * x + y * y) + z * z); }

// Group error |dS| / |S0 + hn S'| of eq. gbs-criterion; groups with a zero
// denominator are skipped (returns 0); non-finite values give +inf.
__device__ __forceinline__ double group_err(double nx, double ny, double nz, double dx, double dy, double dz) {
    if (!isfinite(nx) || !isfinite(ny) || !isfinite(nz)) return INFINITY;
    const double dd = norm3(dx, dy, dz);
    if (!(dd > 0.0)) return 0.0;
    const double e = norm3(nx, ny, nz) / dd;
    return isnan(e) ? INFINITY : e;
}

// The same with the larger of two denominators: the centre-of-mass groups,
// whose value can start at the rounding level (a system at rest at the
// origin), also take the extrapolated end value as their scale.
__device__ __forceinline__ double group_err2(double nx, double ny, double nz, double dx, double dy, double dz,
                                             double ex, double ey, double ez) {
    if (!isfinite(nx) || !isfinite(ny) || !isfinite(nz)) return INFINITY;
    double dd = norm3(dx, dy, dz);
    const double de = norm3(ex, ey, ez);
    if (de > dd) dd = de;
    if (!(dd > 0.0)) return 0.0;
    const double e = norm3(nx, ny, nz) / dd;
    return isnan(e) ? INFINITY : e;
}

__device__ __forceinline__ double fmax_nan(double a, double b) {
    if (isnan(a) || isnan(b)) return INFINITY;
    return a > b ? a : b;
}

template <int KF>
__device__ __forceinline__ void load_col(const d4 *arr, int n, int v, double (&x)[KF], double (&y)[KF],
                                         double (&z)[KF]) {
#pragma unroll
    for (int k = 0; k < KF; ++k) {
        const d4 a = arr[(size_t)k * n + v];
        x[k] = a.x; y[k] = a.y; z[k] = a.z;
    }
}

// Extrapolate the increments of one 3-vector per body over the KF divisions;
// returns T_{KF,KF} in out and T_{KF,KF} - T_{KF-1,KF-1} in diff.
template <int KF>
__device__ __forceinline__ void extrap3(const d4 *arr, int n, int v, d4 &out, double &ex, double &ey, double &ez) {
    double x[KF], y[KF], z[KF];
    load_col<KF>(arr, n, v, x, y, z);
    neville<KF>(x); neville<KF>(y); neville<KF>(z);
    out = d4{x[KF - 1], y[KF - 1], z[KF - 1], 0.0};
    ex = x[KF - 1] - x[KF - 2];
    ey = y[KF - 1] - y[KF - 2];
    ez = z[KF - 1] - z[KF - 2];
}

// The outputs T_{ko,ko} (ko = kout, 1-based) of every extrapolated variable
// except the scalars' error groups: edge vectors, edge velocities and the
// carried positions and velocities, and the scalar increments.
template <int KF>
__device__ __forceinline__ void pick3(const d4 *arr, int n, int v, int ko, d4 &out) {
    double x[KF], y[KF], z[KF];
    load_col<KF>(arr, n, v, x, y, z);
    neville<KF>(x); neville<KF>(y); neville<KF>(z);
    out = d4{x[0], y[0], z[0], 0.0};
#pragma unroll
    for (int k = 1; k < KF; ++k)
        if (k == ko - 1) out = d4{x[k], y[k], z[k], 0.0};
}

// Second pass of the earliest-k acceptance (accept_rule 1): the outputs at
// the order k_acc the control chose (T_{k_acc,k_acc} of every variable).
template <int KF>
__global__ __launch_bounds__(kWG) void k_extrap_pick(Dev d, int with_ext) {
    const int n = d.n;
    const int v = blockIdx.x * kWG + threadIdx.x;
    const int ko = d.ctl->kacc > 0 ? d.ctl->kacc : KF;
    if (v < n) {
        d4 o;
        pick3<KF>(d.dX, n, v, ko, o); d.dX1[v] = o;
        pick3<KF>(d.dV, n, v, ko, o); d.dV1[v] = o;
        pick3<KF>(d.dP, n, v, ko, o); d.dP1[v] = o;
        pick3<KF>(d.dVt, n, v, ko, o); d.dVt1[v] = o;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        double pt[KF], rx[KF], ry[KF], rz[KF], pw[KF], pb[KF], ux[KF], uy[KF], uz[KF];
#pragma unroll
        for (int k = 0; k < KF; ++k) {
            const DivScal q = d.dscal[k];
            pt[k] = q.tau; rx[k] = q.drcm[0]; ry[k] = q.drcm[1]; rz[k] = q.drcm[2]; pw[k] = q.dwn;
            pb[k] = q.dBn; ux[k] = q.dvcm[0]; uy[k] = q.dvcm[1]; uz[k] = q.dvcm[2];
        }
        neville<KF>(pt); neville<KF>(rx); neville<KF>(ry); neville<KF>(rz); neville<KF>(pw);
        if (with_ext) { neville<KF>(pb); neville<KF>(ux); neville<KF>(uy); neville<KF>(uz); }
        DivScal out{};
#pragma unroll
        for (int k = 0; k < KF; ++k)
            if (k == ko - 1) {
                out.tau = pt[k];
                out.dw = pw[k];
                out.drcm[0] = rx[k]; out.drcm[1] = ry[k]; out.drcm[2] = rz[k];
                if (with_ext) {
                    out.dB = pb[k];
                    out.dvcm[0] = ux[k]; out.dvcm[1] = uy[k]; out.dvcm[2] = uz[k];
                }
            }
        *d.dscal1 = out;
    }
}

// Error measure of eq. gbs-criterion for every order k = 2..KF (the
// earliest-k acceptance, accept_rule 1): per workgroup, the maximum over its
// bodies' edge groups of |T_kk - T_{k-1,k-1}| / |S0 + (H/n_k) S'(s0)| into
// epspart[(k-1) * parts + block]; block 0 adds the scalar groups.  Outputs
// are written by k_extrap_pick once the order is chosen.
template <int KF>
__global__ __launch_bounds__(kWG) void k_extrap_allk(Dev d, Ttl tr, int with_ext) {
    __shared__ double sh[kWG];
    const int n = d.n;
    const int v = blockIdx.x * kWG + threadIdx.x;
    const int parts = d.nkwg + 1;
    const Ctl &c = *d.ctl;
    const double H = c.H;
    const double gd = (tr.alpha * (c.T0 + d.sys->B) + tr.beta * d.sys->w) + tr.gamma;
    const double gk = (tr.alpha * c.U0 + tr.beta * c.Om0) + tr.gamma;
    double ek[KF];
#pragma unroll
    for (int k = 0; k < KF; ++k) ek[k] = 0.0;
    if (v < n) {
        const int p = d.parent[v];
        if (p >= 0) {
            double x[KF], y[KF], z[KF], a[KF], b[KF], e[KF];
            load_col<KF>(d.dX, n, v, x, y, z);
            load_col<KF>(d.dV, n, v, a, b, e);
            neville<KF>(x); neville<KF>(y); neville<KF>(z);
            neville<KF>(a); neville<KF>(b); neville<KF>(e);
            const d4 X0 = d.X0[v], V0 = d.V0[v];
            d4 av = d.a0[v], ap = d.a0[p];
            if (with_ext) {
                const d4 fv = d.fext[(size_t)kBaseSlot * n + v], fp = d.fext[(size_t)kBaseSlot * n + p];
                av.x = av.x + fv.x; av.y = av.y + fv.y; av.z = av.z + fv.z;
                ap.x = ap.x + fp.x; ap.y = ap.y + fp.y; ap.z = ap.z + fp.z;
            }
#pragma unroll
            for (int k = 1; k < KF; ++k) {
                const double hn = H / (double)(2 * (k + 1));
                const double ex = group_err(x[k] - x[k - 1], y[k] - y[k - 1], z[k] - z[k - 1], X0.x + hn * (V0.x / gd),
                                            X0.y + hn * (V0.y / gd), X0.z + hn * (V0.z / gd));
                const double ev = group_err(a[k] - a[k - 1], b[k] - b[k - 1], e[k] - e[k - 1],
                                            V0.x + hn * ((av.x - ap.x) / gk), V0.y + hn * ((av.y - ap.y) / gk),
                                            V0.z + hn * ((av.z - ap.z) / gk));
                ek[k] = fmax_nan(ex, ev);
            }
        }
    }
#pragma unroll
    for (int k = 1; k < KF; ++k) {
        sh[threadIdx.x] = ek[k];
        __syncthreads();
        for (int s = kWG / 2; s > 0; s >>= 1) {
            if (threadIdx.x < s) sh[threadIdx.x] = fmax_nan(sh[threadIdx.x], sh[threadIdx.x + s]);
            __syncthreads();
        }
        if (threadIdx.x == 0) d.epspart[(size_t)(k - 1) * parts + blockIdx.x] = sh[0];
        __syncthreads();
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        double pt[KF], rx[KF], ry[KF], rz[KF], pw[KF], pb[KF], ux[KF], uy[KF], uz[KF];
#pragma unroll
        for (int k = 0; k < KF; ++k) {
            const DivScal q = d.dscal[k];
            pt[k] = q.tau; rx[k] = q.drcm[0]; ry[k] = q.drcm[1]; rz[k] = q.drcm[2]; pw[k] = q.dwn;
            pb[k] = q.dBn; ux[k] = q.dvcm[0]; uy[k] = q.dvcm[1]; uz[k] = q.dvcm[2];
        }
        neville<KF>(pt); neville<KF>(rx); neville<KF>(ry); neville<KF>(rz); neville<KF>(pw);
        double F[4] = {0.0, 0.0, 0.0, 0.0};
        if (with_ext) {
            neville<KF>(pb); neville<KF>(ux); neville<KF>(uy); neville<KF>(uz);
            const d4 *fp = d.fpart + (size_t)kBaseSlot * d.nkwg4;
            for (int k = 0; k < d.nkwg; ++k) {
                const d4 t = fp[k];
                F[0] = F[0] + t.x; F[1] = F[1] + t.y; F[2] = F[2] + t.z; F[3] = F[3] + t.w;
            }
        }
        const SysScal &y = *d.sys;
#pragma unroll
        for (int k = 1; k < KF; ++k) {
            const double hn = H / (double)(2 * (k + 1));
            const double et = group_err(pt[k] - pt[k - 1], 0.0, 0.0, y.t + hn * (1.0 / gd), 0.0, 0.0);
            const double er = group_err2(rx[k] - rx[k - 1], ry[k] - ry[k - 1], rz[k] - rz[k - 1],
                                         y.rcm[0] + hn * (y.vcm[0] / gd), y.rcm[1] + hn * (y.vcm[1] / gd),
                                         y.rcm[2] + hn * (y.vcm[2] / gd), y.rcm[0] + rx[k], y.rcm[1] + ry[k],
                                         y.rcm[2] + rz[k]);
            double es = fmax_nan(et, er);
            if (tr.beta != 0.0)
                es = fmax_nan(es, group_err(pw[k] - pw[k - 1], 0.0, 0.0, y.w + hn * (c.dw0 / gk), 0.0, 0.0));
            if (with_ext) {
                const double Minv = d.ext->Minv;
                es = fmax_nan(es, group_err(pb[k] - pb[k - 1], 0.0, 0.0, y.B + hn * (-F[3] / gk), 0.0, 0.0));
                es = fmax_nan(es, group_err2(ux[k] - ux[k - 1], uy[k] - uy[k - 1], uz[k] - uz[k - 1],
                                             y.vcm[0] + hn * (F[0] * Minv / gk), y.vcm[1] + hn * (F[1] * Minv / gk),
                                             y.vcm[2] + hn * (F[2] * Minv / gk), y.vcm[0] + ux[k], y.vcm[1] + uy[k],
                                             y.vcm[2] + uz[k]));
            }
            d.epspart[(size_t)(k - 1) * parts + d.nkwg] = es;
        }
    }
}

template <int KF>
__global__ __launch_bounds__(kWG) void k_extrapolate(Dev d, Ttl tr, int base, int with_ext) {
    __shared__ double sh[kWG];
    const int n = d.n;
    const int v = blockIdx.x * kWG + threadIdx.x;
    const Ctl &c = *d.ctl;
    const double H = c.H;
    const double hn = H / (double)(2 * KF);
    const double gd = (tr.alpha * (c.T0 + d.sys->B) + tr.beta * d.sys->w) + tr.gamma;
    const double gk = (tr.alpha * c.U0 + tr.beta * c.Om0) + tr.gamma;
    double eps = 0.0;
    if (v < n) {
        d4 ox, ov, op, ow;
        double xx, xy, xz, vx, vy, vz, t0, t1, t2;
        extrap3<KF>(d.dX, n, v, ox, xx, xy, xz);
        extrap3<KF>(d.dV, n, v, ov, vx, vy, vz);
        extrap3<KF>(d.dP, n, v, op, t0, t1, t2);     // positions and velocities are carried
        extrap3<KF>(d.dVt, n, v, ow, t0, t1, t2);    // along; they are not error-tested
        d.dX1[v] = ox;
        d.dV1[v] = ov;
        d.dP1[v] = op;
        d.dVt1[v] = ow;
        const int p = d.parent[v];
        if (p >= 0) {
            const d4 X0 = d.X0[v], V0 = d.V0[v];
            d4 av = d.a0[v], ap = d.a0[p];
            if (with_ext) {   // S' of the edge velocities includes the external field
                const d4 fv = d.fext[(size_t)kBaseSlot * n + v], fp = d.fext[(size_t)kBaseSlot * n + p];
                av.x = av.x + fv.x; av.y = av.y + fv.y; av.z = av.z + fv.z;
                ap.x = ap.x + fp.x; ap.y = ap.y + fp.y; ap.z = ap.z + fp.z;
            }
            const double ex = group_err(xx, xy, xz, X0.x + hn * (V0.x / gd), X0.y + hn * (V0.y / gd),
                                        X0.z + hn * (V0.z / gd));
            const double ev = group_err(vx, vy, vz, V0.x + hn * ((av.x - ap.x) / gk), V0.y + hn * ((av.y - ap.y) / gk),
                                        V0.z + hn * ((av.z - ap.z) / gk));
            eps = fmax_nan(ex, ev);
        }
    }
    // block max (exact, order independent)
    sh[threadIdx.x] = eps;
    __syncthreads();
    for (int s = kWG / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] = fmax_nan(sh[threadIdx.x], sh[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) d.epspart[blockIdx.x] = sh[0];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        // scalar groups: t (extrapolated through its increment tau), r_cm
        // and, with TTL, w; under an external field also B and v_cm
        double pt[KF], rx[KF], ry[KF], rz[KF], pw[KF];
#pragma unroll
        for (int k = 0; k < KF; ++k) {
            const DivScal q = d.dscal[k];
            pt[k] = q.tau; rx[k] = q.drcm[0]; ry[k] = q.drcm[1]; rz[k] = q.drcm[2]; pw[k] = q.dwn;
        }
        neville<KF>(pt); neville<KF>(rx); neville<KF>(ry); neville<KF>(rz); neville<KF>(pw);
        DivScal out{};
        out.tau = pt[KF - 1];
        out.dw = pw[KF - 1];
        out.drcm[0] = rx[KF - 1]; out.drcm[1] = ry[KF - 1]; out.drcm[2] = rz[KF - 1];
        double eb = 0.0;
        if (with_ext) {
            double pb[KF], ux[KF], uy[KF], uz[KF];
#pragma unroll
            for (int k = 0; k < KF; ++k) {
                const DivScal q = d.dscal[k];
                pb[k] = q.dBn; ux[k] = q.dvcm[0]; uy[k] = q.dvcm[1]; uz[k] = q.dvcm[2];
            }
            neville<KF>(pb); neville<KF>(ux); neville<KF>(uy); neville<KF>(uz);
            out.dB = pb[KF - 1];
            out.dvcm[0] = ux[KF - 1]; out.dvcm[1] = uy[KF - 1]; out.dvcm[2] = uz[KF - 1];
            // start-state rates: dB/ds = -sum m f.v / g_k, dv_cm/ds = F / (M g_k)
            const d4 *fp = d.fpart + (size_t)kBaseSlot * d.nkwg4;
            double F[4] = {0.0, 0.0, 0.0, 0.0};
            for (int k = 0; k < d.nkwg; ++k) {
                const d4 t = fp[k];
                F[0] = F[0] + t.x; F[1] = F[1] + t.y; F[2] = F[2] + t.z; F[3] = F[3] + t.w;
            }
            const double Minv = d.ext->Minv;
            const SysScal &y0 = *d.sys;
            eb = fmax_nan(group_err(pb[KF - 1] - pb[KF - 2], 0.0, 0.0, y0.B + hn * (-F[3] / gk), 0.0, 0.0),
                          group_err2(ux[KF - 1] - ux[KF - 2], uy[KF - 1] - uy[KF - 2], uz[KF - 1] - uz[KF - 2],
                                     y0.vcm[0] + hn * (F[0] * Minv / gk), y0.vcm[1] + hn * (F[1] * Minv / gk),
                                     y0.vcm[2] + hn * (F[2] * Minv / gk), y0.vcm[0] + ux[KF - 1],
                                     y0.vcm[1] + uy[KF - 1], y0.vcm[2] + uz[KF - 1]));
        }
        *d.dscal1 = out;
        const SysScal &y = *d.sys;
        const double et = group_err(pt[KF - 1] - pt[KF - 2], 0.0, 0.0, y.t + hn * (1.0 / gd), 0.0, 0.0);
        const double er = group_err2(rx[KF - 1] - rx[KF - 2], ry[KF - 1] - ry[KF - 2], rz[KF - 1] - rz[KF - 2],
                                     y.rcm[0] + hn * (y.vcm[0] / gd), y.rcm[1] + hn * (y.vcm[1] / gd),
                                     y.rcm[2] + hn * (y.vcm[2] / gd), y.rcm[0] + rx[KF - 1], y.rcm[1] + ry[KF - 1],
                                     y.rcm[2] + rz[KF - 1]);
        double es = fmax_nan(et, er);
        if (tr.beta != 0.0)
            es = fmax_nan(es, group_err(pw[KF - 1] - pw[KF - 2], 0.0, 0.0, y.w + hn * (c.dw0 / gk), 0.0, 0.0));
        if (with_ext) es = fmax_nan(es, eb);
        d.epspart[d.nkwg] = es;
    }
}

void launch_extrapolate(const Dev &d, hipStream_t s, int kf, Ttl tr, int base, bool ex, int rule) {
    const int nb = (d.n + kWG - 1) / kWG;
    if (rule == 1) {
        switch (kf) {
#define KFC(K) case K: k_extrap_allk<K><<<nb, kWG, 0, s>>>(d, tr, ex ? 1 : 0); break;
            KFC(2) KFC(3) KFC(4) KFC(5) KFC(6) KFC(7) KFC(8) KFC(9) KFC(10) KFC(11) KFC(12) KFC(13) KFC(14)
            KFC(15) KFC(16)
#undef KFC
            default: break;
        }
        return;
    }
    switch (kf) {
#define KFC(K) case K: k_extrapolate<K><<<nb, kWG, 0, s>>>(d, tr, base, ex ? 1 : 0); break;
        KFC(2) KFC(3) KFC(4) KFC(5) KFC(6) KFC(7) KFC(8) KFC(9) KFC(10) KFC(11) KFC(12) KFC(13) KFC(14)
        KFC(15) KFC(16)
#undef KFC
        default: break;
    }
}

void launch_extrap_pick(const Dev &d, hipStream_t s, int kf, bool ex) {
    const int nb = (d.n + kWG - 1) / kWG;
    switch (kf) {
#define KFC(K) case K: k_extrap_pick<K><<<nb, kWG, 0, s>>>(d, ex ? 1 : 0); break;
        KFC(2) KFC(3) KFC(4) KFC(5) KFC(6) KFC(7) KFC(8) KFC(9) KFC(10) KFC(11) KFC(12) KFC(13) KFC(14)
        KFC(15) KFC(16)
#undef KFC
        default: break;
    }
}

// Accept iff eps <= eta; next step per eq. hnext with the clamps, or H/2.
// rule 0: eps of order kf (Sec. 4.2); rule 1: the first order k = 2..kf
// whose eps_k <= eta (eq. hnext then uses that k); k_acc records the order.
__global__ void k_control(Dev d, int kf, int nparts, double eta, double a_gbs, double f_min, double f_max, int rule) {
    Ctl &c = *d.ctl;
    double eps = 0.0;
    int kacc = 0;
    for (int k = rule == 1 ? 2 : kf; k <= kf; ++k) {
        const double *ep = d.epspart + (rule == 1 ? (size_t)(k - 2) * nparts : 0);
        eps = 0.0;
        for (int q = 0; q < nparts; ++q) eps = fmax_nan(eps, ep[q]);
        if (eps <= eta) {
            kacc = k;
            break;
        }
    }
    c.eps = eps;
    c.kacc = kacc;
    c.accepted = kacc > 0 ? 1 : 0;
    if (c.accepted) {
        const double e = eps > 1e-300 ? eps : 1e-300;
        double f = a_gbs * pow(eta / e, 1.0 / (double)(2 * kacc - 1));
        if (f < f_min) f = f_min;
        if (f > f_max) f = f_max;
        c.h_next = c.H * f;
    } else {
        c.h_next = 0.5 * c.H;
    }
}

void launch_control(const Dev &d, hipStream_t s, int kf, double eta, double a_gbs, double f_min, double f_max,
                    int rule) {
    const int nb = (d.n + kWG - 1) / kWG;
    k_control<<<1, 1, 0, s>>>(d, kf, nb + 1, eta, a_gbs, f_min, f_max, rule);
}

// Commit the extrapolated increments (if the step was accepted) or the end
// state of division `slot` (from_extrap = 0, used by the single-leapfrog
// call): MST edges, COM-frame positions and velocities, t, r_cm; partial sums
// of m |v|^2 of the new start state for T.
__global__ __launch_bounds__(kWG) void k_commit(Dev d, int from_extrap, int slot) {
    __shared__ double sh[kWG];
    // a step taken while a rebuild had not finished its tree is repeated
    if (from_extrap && (!d.ctl->accepted || d.ctl->tree_bad)) return;
    const int n = d.n;
    const int v = blockIdx.x * kWG + threadIdx.x;
    const size_t o = (size_t)slot * n + v;
    const d4 *dx = from_extrap ? d.dX1 : d.dX + (size_t)slot * n;
    const d4 *dv = from_extrap ? d.dV1 : d.dV + (size_t)slot * n;
    const d4 *dp = from_extrap ? d.dP1 : d.dP + (size_t)slot * n;
    const d4 *dw = from_extrap ? d.dVt1 : d.dVt + (size_t)slot * n;
    (void)o;
    double tl = 0.0;
    if (v < n) {
        d4 X = d.X0[v], V = d.V0[v];
        const d4 a = dx[v], b = dv[v];
        X.x = X.x + a.x; X.y = X.y + a.y; X.z = X.z + a.z;
        V.x = V.x + b.x; V.y = V.y + b.y; V.z = V.z + b.z;
        d.X0[v] = X;
        d.V0[v] = V;
        const size_t ob = (size_t)kBaseSlot * n + v;
        d4 P = d.P[ob], W = d.Vt[ob];
        const d4 e = dp[v], f = dw[v];
        P.x = P.x + e.x; P.y = P.y + e.y; P.z = P.z + e.z;
        W.x = W.x + f.x; W.y = W.y + f.y; W.z = W.z + f.z;
        d.P[ob] = P;
        d.Vt[ob] = W;
        tl = P.w * ((W.x * W.x + W.y * W.y) + W.z * W.z);
    }
    const double ts = block_sum<kWG>(tl, sh);
    if (threadIdx.x == 0) d.Tpart[(size_t)kBaseSlot * d.nkwg4 + blockIdx.x] = ts;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const DivScal q = from_extrap ? *d.dscal1 : d.dscal[slot];
        SysScal &y = *d.sys;
        y.t = y.t + q.tau;
        y.w = y.w + (from_extrap ? q.dw : q.dwn);
        y.B = y.B + (from_extrap ? q.dB : q.dBn);
        for (int c = 0; c < 3; ++c) {
            y.rcm[c] = y.rcm[c] + q.drcm[c];
            y.vcm[c] = y.vcm[c] + q.dvcm[c];
        }
    }
}

void launch_commit(const Dev &d, hipStream_t s, int from_extrap, int slot) {
    k_commit<<<(d.n + kWG - 1) / kWG, kWG, 0, s>>>(d, from_extrap, slot);
}

// Edge vectors of the MST from Cartesian input (Sec. 3.4: vectors point away
// from the root): X_v = x_v - x_parent(v), V_v likewise; COM of x and v.
__global__ __launch_bounds__(kTreeWG) void k_state_from_cartesian(Dev d, const double *x, const double *v) {
    __shared__ double sh[kTreeWG];
    const int n = d.n;
    double sm = 0.0, s[6] = {0, 0, 0, 0, 0, 0};
    for (int u = threadIdx.x; u < n; u += kTreeWG) {
        const int p = d.parent[u];
        d4 X{0.0, 0.0, 0.0, 0.0}, V{0.0, 0.0, 0.0, 0.0};
        if (p >= 0) {
            X = d4{x[3 * u] - x[3 * p], x[3 * u + 1] - x[3 * p + 1], x[3 * u + 2] - x[3 * p + 2], 0.0};
            V = d4{v[3 * u] - v[3 * p], v[3 * u + 1] - v[3 * p + 1], v[3 * u + 2] - v[3 * p + 2], 0.0};
        }
        d.X0[u] = X;
        d.V0[u] = V;
        const double mu = d.m[u];
        sm = sm + mu;
        for (int c = 0; c < 3; ++c) {
            s[c] = s[c] + mu * x[3 * u + c];
            s[3 + c] = s[3 + c] + mu * v[3 * u + c];
        }
    }
    const double M = block_sum<kTreeWG>(sm, sh);
    double r[6];
    for (int c = 0; c < 6; ++c) r[c] = block_sum<kTreeWG>(s[c], sh);
    if (threadIdx.x == 0) {
        SysScal &y = *d.sys;
        for (int c = 0; c < 3; ++c) {
            y.rcm[c] = r[c] / M;
            y.vcm[c] = r[3 + c] / M;
        }
        y.w = 0.0;
    }
}

void launch_state_from_cartesian(const Dev &d, hipStream_t s, const double *x, const double *v) {
    k_state_from_cartesian<<<1, kTreeWG, 0, s>>>(d, x, v);
}

// COM-frame positions (+mass) and velocities of the start state from the
// root-relative tree sums rho (tsA) and ups (tsB); T0 = 1/2 sum m |v|^2.
__global__ __launch_bounds__(kTreeWG) void k_com_frame(Dev d, int base) {
    __shared__ double sh[kTreeWG];
    const int n = d.n;
    const d4 *rho = d.tsA, *ups = d.tsB;
    double sm = 0.0, s[6] = {0, 0, 0, 0, 0, 0};
    for (int u = threadIdx.x; u < n; u += kTreeWG) {
        const double mu = d.m[u];
        const d4 r = rho[u], w = ups[u];
        sm = sm + mu;
        s[0] = s[0] + mu * r.x; s[1] = s[1] + mu * r.y; s[2] = s[2] + mu * r.z;
        s[3] = s[3] + mu * w.x; s[4] = s[4] + mu * w.y; s[5] = s[5] + mu * w.z;
    }
    const double M = block_sum<kTreeWG>(sm, sh);
    double c[6];
    for (int k = 0; k < 6; ++k) c[k] = block_sum<kTreeWG>(s[k], sh) / M;
    double tl = 0.0;
    d4 *P0 = d.P + (size_t)base * n;
    d4 *V0 = d.Vt + (size_t)base * n;
    for (int u = threadIdx.x; u < n; u += kTreeWG) {
        const double mu = d.m[u];
        const d4 r = rho[u], w = ups[u];
        P0[u] = d4{r.x - c[0], r.y - c[1], r.z - c[2], mu};
        const d4 vt{w.x - c[3], w.y - c[4], w.z - c[5], 0.0};
        V0[u] = vt;
        tl = tl + mu * ((vt.x * vt.x + vt.y * vt.y) + vt.z * vt.z);
    }
    const double T2 = block_sum<kTreeWG>(tl, sh);
    double *tp = d.Tpart + (size_t)kBaseSlot * d.nkwg4;
    for (int k = threadIdx.x; k < d.nkwg; k += kTreeWG) tp[k] = (k == 0) ? T2 : 0.0;
    if (threadIdx.x == 0) d.ctl->T0 = 0.5 * T2;
}

void launch_com_frame(const Dev &d, hipStream_t s, int base) { k_com_frame<<<1, kTreeWG, 0, s>>>(d, base); }

// Cartesian output x_i = r_cm + (rho_i - rho_bar), v_i = v_cm + (ups_i - ups_bar).
__global__ __launch_bounds__(kTreeWG) void k_output_cartesian(Dev d, double *x, double *v) {
    __shared__ double sh[kTreeWG];
    const int n = d.n;
    const d4 *rho = d.tsA, *ups = d.tsB;
    double sm = 0.0, s[6] = {0, 0, 0, 0, 0, 0};
    for (int u = threadIdx.x; u < n; u += kTreeWG) {
        const double mu = d.m[u];
        const d4 r = rho[u], w = ups[u];
        sm = sm + mu;
        s[0] = s[0] + mu * r.x; s[1] = s[1] + mu * r.y; s[2] = s[2] + mu * r.z;
        s[3] = s[3] + mu * w.x; s[4] = s[4] + mu * w.y; s[5] = s[5] + mu * w.z;
    }
    const double M = block_sum<kTreeWG>(sm, sh);
    double c[6];
    for (int k = 0; k < 6; ++k) c[k] = block_sum<kTreeWG>(s[k], sh) / M;
    const SysScal y = *d.sys;
    for (int u = threadIdx.x; u < n; u += kTreeWG) {
        const d4 r = rho[u], w = ups[u];
        x[3 * u] = y.rcm[0] + (r.x - c[0]);
        x[3 * u + 1] = y.rcm[1] + (r.y - c[1]);
        x[3 * u + 2] = y.rcm[2] + (r.z - c[2]);
        v[3 * u] = y.vcm[0] + (w.x - c[3]);
        v[3 * u + 1] = y.vcm[1] + (w.y - c[4]);
        v[3 * u + 2] = y.vcm[2] + (w.z - c[5]);
    }
}

void launch_output_cartesian(const Dev &d, hipStream_t s, double *x, double *v) {
    k_output_cartesian<<<1, kTreeWG, 0, s>>>(d, x, v);
}

// B = -H = U - T at the start of an integration (Sec. 2.1); the TTL
// variable starts at w = Omega (0 without TTL).
__global__ void k_set_B(Dev d) {
    d.sys->B = d.ctl->U0 - d.ctl->T0;
    d.sys->w = d.ctl->Om0;
}
void launch_set_B(const Dev &d, hipStream_t s) { k_set_B<<<1, 1, 0, s>>>(d); }

// [n][3] doubles <-> 32-byte rows (fourth slot = mass or 0).
__global__ __launch_bounds__(kWG) void k_pack3(const double *x, const double *m, d4 *out, int n) {
    const int v = blockIdx.x * kWG + threadIdx.x;
    if (v < n) out[v] = d4{x[3 * v], x[3 * v + 1], x[3 * v + 2], m ? m[v] : 0.0};
}
void launch_pack3(hipStream_t s, const double *x, const double *m, d4 *out, int n) {
    k_pack3<<<(n + kWG - 1) / kWG, kWG, 0, s>>>(x, m, out, n);
}
__global__ __launch_bounds__(kWG) void k_unpack3(const d4 *in, double *out, int n) {
    const int v = blockIdx.x * kWG + threadIdx.x;
    if (v < n) {
        const d4 a = in[v];
        out[3 * v] = a.x; out[3 * v + 1] = a.y; out[3 * v + 2] = a.z;
    }
}
void launch_unpack3(hipStream_t s, const d4 *in, double *out, int n) {
    k_unpack3<<<(n + kWG - 1) / kWG, kWG, 0, s>>>(in, out, n);
}

__global__ void k_set_sys(Dev d, double t, double B, double w, double r0, double r1, double r2, double v0,
                          double v1, double v2, int set_com) {
    SysScal &y = *d.sys;
    y.t = t;
    y.B = B;
    y.w = w;
    if (set_com) {
        y.rcm[0] = r0; y.rcm[1] = r1; y.rcm[2] = r2;
        y.vcm[0] = v0; y.vcm[1] = v1; y.vcm[2] = v2;
    }
    d.ctl->coincident = 0;
    d.ctl->tree_bad = 0;
}
void launch_set_sys(const Dev &d, hipStream_t s, double t, double B, double w, const double *rcm, const double *vcm,
                    int set_com) {
    k_set_sys<<<1, 1, 0, s>>>(d, t, B, w, set_com ? rcm[0] : 0.0, set_com ? rcm[1] : 0.0, set_com ? rcm[2] : 0.0,
                              set_com ? vcm[0] : 0.0, set_com ? vcm[1] : 0.0, set_com ? vcm[2] : 0.0, set_com);
}

// Coincident bodies: the nearest neighbour of every body is joined to it by
// an MST edge, so a zero-length pair shows up as a zero edge vector.
__global__ __launch_bounds__(kWG) void k_check_coincident(Dev d) {
    const int v = blockIdx.x * kWG + threadIdx.x;
    if (v >= d.n || d.parent[v] < 0) return;
    const d4 x = d.X0[v];
    if (x.x == 0.0 && x.y == 0.0 && x.z == 0.0) d.ctl->coincident = 1;
}
void launch_check_coincident(const Dev &d, hipStream_t s) {
    k_check_coincident<<<(d.n + kWG - 1) / kWG, kWG, 0, s>>>(d);
}

}  // namespace mstar
