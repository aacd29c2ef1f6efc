// Interface between the host driver and the replay / adjoint kernels
// (kernels_adjoint.hip).
#pragma once
#include "common.h"

namespace mstar {

constexpr int kAdjMaxN = 1024;   // bodies (one per thread of a workgroup)
constexpr int kAdjMaxKF = 16;
constexpr int kAdjOpScal = 8;    // scalars kept per leapfrog op: dt, g, T or U, v_cm[3]

// Device buffers of one replay / adjoint run.  Division k stores its kick
// inputs at rows k(k+1) .. of rst, its drift inputs at rows k(k+1)+k .. of
// vst, and its op scalars at ops 2k(k+1)+k .. of sc.
struct AdjDev {
    int n, kf;
    int tpb;                // threads per body (1..4): the j-range of each body is split tpb ways,
    int ext;                // that of the first ext bodies tpb + 1 ways (tpb n + ext <= 1024 threads)
    double G, alpha, gamma;
    const double *m;        // [n]
    const double *c;        // [kf] extrapolation weights
    double *B;              // U(r0) - T(v0)
    d4 *Er, *Ev;            // [kf][n] division end states
    double *Et;             // [kf]
    d4 *Lr, *Lv;            // [n] cotangent of the current step's end state
    double *Lt, *LB;        // cotangent of t; accumulated cotangent of B
    d4 *Sr, *Sv;            // [kf][n] cotangents of the division start states
    double *St, *SB;        // [kf]
    double *Sm;             // [kf][n] cotangent of the masses from one division
    double *Lm;             // [n] cotangent of the masses, accumulated over the reverse pass
    d4 *rst, *vst;          // stored kick / drift inputs
    double *sc;             // [ops][kAdjOpScal]
};

void launch_adj_init(const AdjDev &d, hipStream_t s, const d4 *Yr, const d4 *Yv);
void launch_adj_fwd(const AdjDev &d, hipStream_t s, const d4 *Yr, const d4 *Yv, const double *Yt, double H,
                    bool store);
void launch_adj_combine(const AdjDev &d, hipStream_t s, const d4 *Yr, const d4 *Yv, const double *Yt, d4 *Or,
                        d4 *Ov, double *Ot);
void launch_adj_rev(const AdjDev &d, hipStream_t s);
void launch_adj_combine_rev(const AdjDev &d, hipStream_t s);
void launch_adj_finish(const AdjDev &d, hipStream_t s, const d4 *Yr, const d4 *Yv, double *gx, double *gv,
                       double *gm);
void launch_adj_zero_n(hipStream_t s, int n, double *p);
void launch_force_hvp(hipStream_t s, int n, double G, const double *m, const double *x, const double *w,
                      double *out);
void launch_adj_pack(hipStream_t s, int n, const double *x, d4 *o, double t, double *ot);
void launch_adj_unpack(hipStream_t s, int n, const d4 *a, double *x);
void launch_adj_zero(hipStream_t s, double *p);
void launch_adj_copy(hipStream_t s, int n, const d4 *a, const d4 *b, const double *t, d4 *oa, d4 *ob, double *ot);

}  // namespace mstar
