// Gradient of sky-position residuals with respect to the initial state.
//
// Forward: the collocation integrator of the propagation kernels (one
// lane per object, wave-shared steps) lands on checkpoint times every
// ckpt_days; observations at per-object times are read off the step's
// collocation polynomial, hopped with light time to the emission point
// (Sect. 2) and turned into RA/Dec.
//
// Backward: the discrete adjoint of that forward map.  Checkpoint
// segments are processed last to first: the segment's steps are
// recomputed from its checkpoint (same step sequence, bit for bit) while
// each step's data and the force Jacobians at its 8 nodes are stored; the
// steps are then swept in reverse, solving the linear stage equations of
// the step's transpose by fixed-point iteration.  The light-time hop's
// Jacobian comes from one forward-mode (six-direction dual number)
// evaluation of the universal-variable solution at its converged anomaly
// plus the implicit light-time term.
#include <math.h>

#include "kete_adjoint.hpp"
#include "kete_radau.hpp"

namespace kete {
namespace {

constexpr int kStepDoubles = 32;     // t, h, x0[3], v0[3], F0[3], D[7][3]
constexpr int kJacDoubles = 18;      // Jx (9) + Jv (9) per node

// ---------------------------------------------------------------- duals
struct D6 {
    double v, d[6];
};
__device__ __forceinline__ D6 mk(double v) { D6 r; r.v = v; for (int i = 0; i < 6; ++i) r.d[i] = 0.0; return r; }
__device__ __forceinline__ D6 operator+(const D6& a, const D6& b) { D6 r; r.v = a.v + b.v; for (int i = 0; i < 6; ++i) r.d[i] = a.d[i] + b.d[i]; return r; }
__device__ __forceinline__ D6 operator-(const D6& a, const D6& b) { D6 r; r.v = a.v - b.v; for (int i = 0; i < 6; ++i) r.d[i] = a.d[i] - b.d[i]; return r; }
__device__ __forceinline__ D6 operator*(const D6& a, const D6& b) { D6 r; r.v = a.v * b.v; for (int i = 0; i < 6; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i]; return r; }
__device__ __forceinline__ D6 operator*(double s, const D6& a) { D6 r; r.v = s * a.v; for (int i = 0; i < 6; ++i) r.d[i] = s * a.d[i]; return r; }
__device__ __forceinline__ D6 operator/(const D6& a, const D6& b) {
    D6 r; r.v = a.v / b.v;
    const double ib = 1.0 / b.v;
    for (int i = 0; i < 6; ++i) r.d[i] = (a.d[i] - r.v * b.d[i]) * ib;
    return r;
}
__device__ __forceinline__ D6 dsqrt(const D6& a) {
    D6 r; r.v = sqrt(a.v);
    const double k = 0.5 / r.v;
    for (int i = 0; i < 6; ++i) r.d[i] = a.d[i] * k;
    return r;
}

// Stumpff c0..c3 on dual arguments (series after quartering, then the
// quadrupling identities, as in the scalar version).
__device__ __forceinline__ void stumpff_d(D6 z, D6& c0, D6& c1, D6& c2, D6& c3) {
    int n = 0;
    while (fabs(z.v) > 0.1 && n < 64) { z = 0.25 * z; ++n; }
    const double a2[8] = {1.0 / 2.0, 1.0 / 24.0, 1.0 / 720.0, 1.0 / 40320.0, 1.0 / 3628800.0, 1.0 / 479001600.0,
                          1.0 / 87178291200.0, 1.0 / 20922789888000.0};
    const double a3[8] = {1.0 / 6.0, 1.0 / 120.0, 1.0 / 5040.0, 1.0 / 362880.0, 1.0 / 39916800.0, 1.0 / 6227020800.0,
                          1.0 / 1307674368000.0, 1.0 / 355687428096000.0};
    c2 = mk(a2[7]); c3 = mk(a3[7]);
    for (int k = 6; k >= 0; --k) {
        c2 = mk(a2[k]) - z * c2;
        c3 = mk(a3[k]) - z * c3;
    }
    c0 = mk(1.0) - z * c2;
    c1 = mk(1.0) - z * c3;
    for (; n > 0; --n) {
        D6 n0 = 2.0 * (c0 * c0) - mk(1.0);
        D6 n1 = c0 * c1;
        D6 n2 = 0.5 * (c1 * c1);
        D6 n3 = 0.25 * (c2 + c0 * c3);
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
}

// P = d r(dt) / d(r0, v0) (3 x 6) of the two-body hop at fixed dt, given
// the converged universal anomaly chi: the implicit dependence of chi is
// one Newton correction evaluated in dual arithmetic.
__device__ void hop_jacobian(double mu, double smu, const double r0v[3], const double v0v[3], double dt, double chi,
                             double P[3][6]) {
    D6 r0[3], v0[3];
    for (int i = 0; i < 3; ++i) {
        r0[i] = mk(r0v[i]); r0[i].d[i] = 1.0;
        v0[i] = mk(v0v[i]); v0[i].d[3 + i] = 1.0;
    }
    const D6 r0n = dsqrt(r0[0] * r0[0] + r0[1] * r0[1] + r0[2] * r0[2]);
    const D6 s0 = (1.0 / smu) * (r0[0] * v0[0] + r0[1] * v0[1] + r0[2] * v0[2]);
    const D6 alpha = mk(2.0) / r0n - (1.0 / mu) * (v0[0] * v0[0] + v0[1] * v0[1] + v0[2] * v0[2]);
    D6 x = mk(chi);
    D6 c0, c1, c2, c3;
    stumpff_d(alpha * x * x, c0, c1, c2, c3);
    const D6 F = r0n * x * c1 + s0 * x * x * c2 + x * x * x * c3 - mk(smu * dt);
    const D6 Fp = r0n * c0 + s0 * x * c1 + x * x * c2;
    D6 xd = F;
    for (int i = 0; i < 6; ++i) xd.d[i] = -F.d[i] / Fp.v;
    xd.v = chi;
    stumpff_d(alpha * xd * xd, c0, c1, c2, c3);
    const D6 f = mk(1.0) - xd * xd * c2 / r0n;
    const D6 g = mk(dt) - (1.0 / smu) * (xd * xd * xd * c3);
    for (int i = 0; i < 3; ++i) {
        const D6 r = f * r0[i] + g * v0[i];
        for (int k = 0; k < 6; ++k) P[i][k] = r.d[k];
    }
}

// RA/Dec of an ecliptic direction (equator of J2000 by the obliquity) and
// d(ra, dec)/d(d_ecl).
__device__ __forceinline__ void radec(const double d[3], double ce, double se, double& ra, double& dec, double J[6]) {
    const double q[3] = {d[0], ce * d[1] - se * d[2], se * d[1] + ce * d[2]};
    const double rho2 = q[0] * q[0] + q[1] * q[1], rho = sqrt(rho2), n2 = rho2 + q[2] * q[2];
    ra = atan2(q[1], q[0]);
    if (ra < 0.0) ra += 6.283185307179586476925286766559;
    dec = atan2(q[2], rho);
    const double da[3] = {-q[1] / rho2, q[0] / rho2, 0.0};
    const double dd[3] = {-q[0] * q[2] / (n2 * rho), -q[1] * q[2] / (n2 * rho), rho / n2};
    J[0] = da[0]; J[1] = ce * da[1] + se * da[2]; J[2] = -se * da[1] + ce * da[2];
    J[3] = dd[0]; J[4] = ce * dd[1] + se * dd[2]; J[5] = -se * dd[1] + ce * dd[2];
}

struct SunGlobal {
    EphemArgs E;
    __device__ __forceinline__ void eval(double t, double pos[3], double vel[3]) const {
        cheb_body(E.coef, 0, E.deg1, t, E.t_start, E.seg_days, E.inv_seg, 0, E.n_seg - 1, pos, vel);
    }
};

// Light-time hop of the state (x, v) at t_obs seen from o: direction d,
// light time, emission velocity, the heliocentric start (r0, v0) and the
// converged universal anomaly of the final hop.
__device__ __forceinline__ int hop(const AdjParams& p, const SunGlobal& sun, double t_obs, const double xs[3],
                                   const double vs[3], const double o[3], double d[3], double& tau, double ve[3],
                                   double r0[3], double v0[3], double& chi) {
    double S[3], Sd[3];
    sun.eval(t_obs, S, Sd);
    for (int i = 0; i < 3; ++i) { r0[i] = xs[i] - S[i]; v0[i] = vs[i] - Sd[i]; }
    const int st = lighttime(sun, p.eph.gm[0], p.smu, p.c_light, p.lt_tol, p.lt_iter, t_obs, r0, v0, t_obs, o, d,
                             tau, ve);
    // universal anomaly of the final hop (warm-started solve)
    double r[3], v[3];
    chi = __builtin_nan("");
    kepler_uv(p.eph.gm[0], p.smu, r0, v0, -tau, chi, r, v);
    return st;
}

// dL/d(x, v) at t_obs from dL/d(ra, dec) through the sky projection and
// the light-time hop (implicit tau: dx_e = P dz - v_e (u . dx_e) / c).
__device__ void hop_vjp(const AdjParams& p, const SunGlobal& sun, double t_obs, const double xs[3], const double vs[3],
                        const double o[3], double gra, double gdec, double lx[3], double lv[3]) {
    double d[3], tau, ve[3], r0[3], v0[3], chi;
    hop(p, sun, t_obs, xs, vs, o, d, tau, ve, r0, v0, chi);
    double ra, dec, J[6];
    radec(d, p.cos_eps, p.sin_eps, ra, dec, J);
    double gd[3];
    for (int i = 0; i < 3; ++i) gd[i] = gra * J[i] + gdec * J[3 + i];
    const double dn = sqrt(dot3(d, d));
    const double u[3] = {d[0] / dn, d[1] / dn, d[2] / dn};
    const double cu = p.c_light + dot3(u, ve);
    const double vg = dot3(ve, gd);
    double gP[3];
    for (int i = 0; i < 3; ++i) gP[i] = gd[i] - u[i] * vg / cu;
    double P[3][6];
    hop_jacobian(p.eph.gm[0], p.smu, r0, v0, -tau, chi, P);
    for (int k = 0; k < 3; ++k) {
        lx[k] = gP[0] * P[0][k] + gP[1] * P[1][k] + gP[2] * P[2][k];
        lv[k] = gP[0] * P[0][3 + k] + gP[1] * P[1][3 + k] + gP[2] * P[2][3 + k];
    }
}

// ---------------------------------------------------------------- forward
__device__ __forceinline__ void save_ckpt(const AdjParams& p, int c, int j, const Lane& L, double hw) {
    double* ck = p.ckpt + ((size_t)c * p.n_obj + j) * kCkptDoubles;
    for (int i = 0; i < 3; ++i) { ck[i] = L.x0[i]; ck[3 + i] = L.v0[i]; }
    ck[6] = hw;
    ck[7] = L.active ? 0.0 : (double)(L.status ? L.status : 1);
}

__global__ __launch_bounds__(64) void k_adjoint_fwd(const AdjParams p) {
    extern __shared__ double smem[];
    const int lane = threadIdx.x;
    const EphemArgs& E = p.eph;
    const int bstride = p.max_win_segs * 3 * E.deg1;
    double* coefL = smem;
    double* ephW = smem + (size_t)E.n_body * bstride;
    const long gi = (long)blockIdx.x * 64 + lane;
    const bool valid = gi < p.n_obj;
    const int j = valid ? p.perm[gi] : 0;
    const SunGlobal sun{E};
    Lane L;
    L.status = 0;
    L.active = valid;
    for (int i = 0; i < 3; ++i) { L.x0[i] = valid ? p.x0[6 * j + i] : (i == 0 ? 1.0 : 0.0); L.v0[i] = valid ? p.x0[6 * j + 3 + i] : 0.0; L.F0[i] = 0.0; }
    double hw = wave_min(L.active ? p.h_pref[j] : kInf);
    if (!(hw < kInf)) hw = p.h_init;
    double t = p.t0;
    bool haveF0 = false;
    long wsteps = 0;
    const int K = p.k_obs;
    int kobs = 0;
    const double* tob = p.t_obs + (size_t)j * K;
    auto sky_of = [&](int k, const double X[3], const double V[3]) {
        double d[3], tau, ve[3], r0[3], v0[3], chi;
        hop(p, sun, tob[k], X, V, p.obs_pos + ((size_t)j * K + k) * 3, d, tau, ve, r0, v0, chi);
        double ra, dec, J[6];
        radec(d, p.cos_eps, p.sin_eps, ra, dec, J);
        p.sky_out[((size_t)j * K + k) * 2] = ra;
        p.sky_out[((size_t)j * K + k) * 2 + 1] = dec;
    };
    // observations at the start epoch
    if (L.active) while (kobs < K && tob[kobs] <= t) { sky_of(kobs, L.x0, L.v0); ++kobs; }
    if (valid) save_ckpt(p, 0, j, L, hw);
    for (int c = 0; c < p.n_ckpt; ++c) {
        for (int w = p.seg_win[c]; w < p.seg_win[c + 1]; ++w) {
            const Window W = p.win[w];
            __syncthreads();
            stage_window(E, W.seg_lo, W.seg_hi, bstride, lane, 64, coefL);
            __syncthreads();
            integrate_window(p, W, coefL, bstride, ephW, L, t, hw, haveF0, wsteps,
                             [&](double ts, double h, const double D[7][3], const double*) {
                                 if (!L.active) return;
                                 const double te = ts + h;
                                 while (kobs < K && (h > 0 ? tob[kobs] <= te : tob[kobs] >= te)) {
                                     double X[3], V[3];
                                     dense_state(p.rc, L.x0, L.v0, L.F0, D, h, (tob[kobs] - ts) / h, X, V);
                                     sky_of(kobs, X, V);
                                     ++kobs;
                                 }
                             });
        }
        if (valid) save_ckpt(p, c + 1, j, L, hw);
    }
    if (valid) {
        p.status[j] = L.status;
        if (L.status)
            for (int k = 0; k < K; ++k) { p.sky_out[((size_t)j * K + k) * 2] = __builtin_nan(""); p.sky_out[((size_t)j * K + k) * 2 + 1] = __builtin_nan(""); }
    }
}

// ---------------------------------------------------------------- backward
__global__ __launch_bounds__(64) void k_adjoint_bwd(const AdjParams p) {
    extern __shared__ double smem[];
    const int lane = threadIdx.x;
    const EphemArgs& E = p.eph;
    const RadauConst& rc = p.rc;
    const int bstride = p.max_win_segs * 3 * E.deg1;
    double* coefL = smem;
    double* ephW = smem + (size_t)E.n_body * bstride;
    const long gi_raw = (long)blockIdx.x * 64 + lane;
    const bool valid = gi_raw < p.n_obj;
    const size_t gi = valid ? (size_t)gi_raw : 0;     // scratch slot (invalid lanes read slot 0, never write)
    const int j = valid ? p.perm[gi] : 0;
    const size_t N = p.n_obj;
    const SunGlobal sun{E};
    const int K = p.k_obs;
    const double* tob = p.t_obs + (size_t)j * K;
    const double* gsky = p.dL_dsky + (size_t)j * K * 2;
    const bool ok_final = valid && p.status[j] == 0;
    double lx[3] = {0.0, 0.0, 0.0}, lv[3] = {0.0, 0.0, 0.0};
    int kb = K - 1;
    bool overflow_steps = false;

    for (int c = p.n_ckpt - 1; c >= 0; --c) {
        // ---- recompute segment c, storing steps and node Jacobians
        Lane L;
        double hw = 0.0;
        if (valid) {
            const double* ck = p.ckpt + ((size_t)c * N + j) * kCkptDoubles;
            for (int i = 0; i < 3; ++i) { L.x0[i] = ck[i]; L.v0[i] = ck[3 + i]; L.F0[i] = 0.0; }
            hw = ck[6];
            L.active = ck[7] == 0.0;
            L.status = 0;
        } else {
            for (int i = 0; i < 3; ++i) { L.x0[i] = (i == 0 ? 1.0 : 0.0); L.v0[i] = 0.0; L.F0[i] = 0.0; }
            L.active = false;
            L.status = 0;
        }
        hw = wave_max(valid ? hw : 0.0);     // the same value in every valid lane
        double t = p.win[p.seg_win[c]].t_a;
        bool haveF0 = false;
        long wsteps = 0;
        int ns = 0;
        for (int w = p.seg_win[c]; w < p.seg_win[c + 1]; ++w) {
            const Window W = p.win[w];
            __syncthreads();
            stage_window(E, W.seg_lo, W.seg_hi, bstride, lane, 64, coefL);
            __syncthreads();
            integrate_window(p, W, coefL, bstride, ephW, L, t, hw, haveF0, wsteps,
                             [&](double ts, double h, const double D[7][3], const double* eph) {
                                 if (ns >= p.s_max) { overflow_steps = true; return; }
                                 if (!valid) { ++ns; return; }
                                 double* sp = p.steps + (size_t)ns * kStepDoubles * N;
                                 sp[0 * N + gi] = ts;
                                 sp[1 * N + gi] = h;
                                 for (int i = 0; i < 3; ++i) {
                                     sp[(2 + i) * N + gi] = L.x0[i];
                                     sp[(5 + i) * N + gi] = L.v0[i];
                                     sp[(8 + i) * N + gi] = L.F0[i];
                                 }
                                 for (int m = 0; m < 7; ++m)
                                     for (int i = 0; i < 3; ++i) sp[(11 + 3 * m + i) * N + gi] = D[m][i];
                                 double* jp = p.jac + (size_t)ns * 8 * kJacDoubles * N;
                                 const double hh = h * h;
                                 for (int n = 0; n < 8; ++n) {
                                     double X[3], V[3];
                                     if (n == 0) {
                                         for (int i = 0; i < 3; ++i) { X[i] = L.x0[i]; V[i] = L.v0[i]; }
                                     } else {
                                         for (int i = 0; i < 3; ++i) {
                                             double ax = rc.half_s2[n] * L.F0[i], av = rc.s[n] * L.F0[i];
                                             for (int m = 0; m < 7; ++m) {
                                                 ax = fma(rc.A[n][m], D[m][i], ax);
                                                 av = fma(rc.B[n][m], D[m][i], av);
                                             }
                                             X[i] = fma(hh, ax, fma(rc.s[n] * h, L.v0[i], L.x0[i]));
                                             V[i] = fma(h, av, L.v0[i]);
                                         }
                                     }
                                     double Jx[9], Jv[9];
                                     accel_jac(eph + n * E.n_body * 6, E, X, V, Jx, Jv);
                                     for (int q = 0; q < 9; ++q) {
                                         jp[((size_t)n * kJacDoubles + q) * N + gi] = Jx[q];
                                         jp[((size_t)n * kJacDoubles + 9 + q) * N + gi] = Jv[q];
                                     }
                                 }
                                 ++ns;
                             });
        }
        // ---- reverse sweep over the stored steps
        for (int s = ns - 1; s >= 0; --s) {
            const double* sp = p.steps + (size_t)s * kStepDoubles * N;
            const double ts = valid ? sp[gi] : 0.0;
            const double h = valid ? sp[N + gi] : 1.0;
            double x0[3], v0[3], F0[3], D[7][3];
            for (int i = 0; i < 3; ++i) {
                x0[i] = valid ? sp[(2 + i) * N + gi] : 0.0;
                v0[i] = valid ? sp[(5 + i) * N + gi] : 0.0;
                F0[i] = valid ? sp[(8 + i) * N + gi] : 0.0;
            }
            for (int m = 0; m < 7; ++m)
                for (int i = 0; i < 3; ++i) D[m][i] = valid ? sp[(11 + 3 * m + i) * N + gi] : 0.0;
            const double hh = h * h;
            // output cotangents: the step end and the observations inside
            double G[8][3];
            double sA = 0.0, sB = 0.0;
            for (int m = 0; m < 7; ++m) { sA += rc.A[8][m]; sB += rc.B[8][m]; }
            for (int i = 0; i < 3; ++i) {
                G[0][i] = hh * (rc.half_s2[8] - sA) * lx[i] + h * (1.0 - sB) * lv[i];
                for (int m = 0; m < 7; ++m) G[m + 1][i] = hh * rc.A[8][m] * lx[i] + h * rc.B[8][m] * lv[i];
            }
            double gx0[3], gv0[3];
            for (int i = 0; i < 3; ++i) { gx0[i] = lx[i]; gv0[i] = h * lx[i] + lv[i]; }
            if (ok_final) {
                while (kb >= 0 && (h > 0 ? tob[kb] > ts : tob[kb] < ts)) {
                    const double sig = (tob[kb] - ts) / h;
                    double X[3], V[3];
                    dense_state(rc, x0, v0, F0, D, h, sig, X, V);
                    double lX[3], lV[3];
                    hop_vjp(p, sun, tob[kb], X, V, p.obs_pos + ((size_t)j * K + kb) * 3, gsky[2 * kb], gsky[2 * kb + 1],
                            lX, lV);
                    double al[7], be[7];
                    dense_weights(rc, sig, al, be);
                    double sa = 0.0, sb = 0.0;
                    for (int m = 0; m < 7; ++m) { sa += al[m]; sb += be[m]; }
                    for (int i = 0; i < 3; ++i) {
                        G[0][i] += hh * (0.5 * sig * sig - sa) * lX[i] + h * (sig - sb) * lV[i];
                        for (int m = 0; m < 7; ++m) G[m + 1][i] += hh * al[m] * lX[i] + h * be[m] * lV[i];
                        gx0[i] += lX[i];
                        gv0[i] += sig * h * lX[i] + lV[i];
                    }
                    --kb;
                }
            }
            // stage cotangents: mu_m = G_m + sum_n [h^2 alpha_m(s_n) Jx_n^T mu_n + h beta_m(s_n) Jv_n^T mu_n]
            const double* jp = p.jac + (size_t)s * 8 * kJacDoubles * N;
            double mu[7][3];
            for (int m = 0; m < 7; ++m) for (int i = 0; i < 3; ++i) mu[m][i] = G[m + 1][i];
            double wsum[3], usum[3], m0[3];
            double pc = 1e300, pcl;
            int it = 0;
            do {
                pcl = pc;
                ++it;
                double nm[7][3];
                for (int m = 0; m < 7; ++m) for (int i = 0; i < 3; ++i) nm[m][i] = G[m + 1][i];
                for (int i = 0; i < 3; ++i) { wsum[i] = 0.0; usum[i] = 0.0; m0[i] = G[0][i]; }
                for (int n = 1; n <= 7; ++n) {
                    double wn[3], un[3];
                    for (int c2 = 0; c2 < 3; ++c2) {
                        double a = 0.0, b = 0.0;
                        for (int r = 0; r < 3; ++r) {
                            a = fma(jp[((size_t)n * kJacDoubles + 3 * r + c2) * N + gi], mu[n - 1][r], a);
                            b = fma(jp[((size_t)n * kJacDoubles + 9 + 3 * r + c2) * N + gi], mu[n - 1][r], b);
                        }
                        wn[c2] = a; un[c2] = b;
                    }
                    double sAn = 0.0, sBn = 0.0;
                    for (int m = 0; m < 7; ++m) { sAn += rc.A[n][m]; sBn += rc.B[n][m]; }
                    for (int i = 0; i < 3; ++i) {
                        for (int m = 0; m < 7; ++m) nm[m][i] += hh * rc.A[n][m] * wn[i] + h * rc.B[n][m] * un[i];
                        m0[i] += hh * (rc.half_s2[n] - sAn) * wn[i] + h * (rc.s[n] - sBn) * un[i];
                        wsum[i] += wn[i];
                        usum[i] += rc.s[n] * h * wn[i] + un[i];
                    }
                }
                double dm = 0.0, mm = 0.0;
                for (int m = 0; m < 7; ++m)
                    for (int i = 0; i < 3; ++i) {
                        dm = fmax(dm, fabs(nm[m][i] - mu[m][i]));
                        mm = fmax(mm, fabs(nm[m][i]));
                        mu[m][i] = nm[m][i];
                    }
                pc = wave_max((ok_final && mm > 0.0) ? dm / mm : 0.0);
            } while (!(pc < 1e-16) && !(it > 2 && pcl <= pc) && it < 2 * p.max_iter);
            // wsum/usum/m0 hold the sums of the last sweep, whose mu differs
            // from the converged one by the last change only
            double J0x[9], J0v[9];
            for (int q = 0; q < 9; ++q) {
                J0x[q] = jp[(size_t)q * N + gi];
                J0v[q] = jp[(size_t)(9 + q) * N + gi];
            }
            for (int i = 0; i < 3; ++i) {
                double a = 0.0, b = 0.0;
                for (int r = 0; r < 3; ++r) { a = fma(J0x[3 * r + i], m0[r], a); b = fma(J0v[3 * r + i], m0[r], b); }
                lx[i] = gx0[i] + wsum[i] + a;
                lv[i] = gv0[i] + usum[i] + b;
            }
        }
    }
    // observations at the start epoch
    if (ok_final) {
        while (kb >= 0) {
            double lX[3], lV[3];
            const double xs[3] = {p.x0[6 * j], p.x0[6 * j + 1], p.x0[6 * j + 2]};
            const double vs[3] = {p.x0[6 * j + 3], p.x0[6 * j + 4], p.x0[6 * j + 5]};
            hop_vjp(p, sun, tob[kb], xs, vs, p.obs_pos + ((size_t)j * K + kb) * 3, gsky[2 * kb], gsky[2 * kb + 1], lX, lV);
            for (int i = 0; i < 3; ++i) { lx[i] += lX[i]; lv[i] += lV[i]; }
            --kb;
        }
    }
    if (valid) {
        const bool good = ok_final && !overflow_steps;
        for (int i = 0; i < 3; ++i) {
            p.grad[6 * j + i] = good ? lx[i] : 0.0;
            p.grad[6 * j + 3 + i] = good ? lv[i] : 0.0;
        }
        if (overflow_steps && p.status[j] == 0) p.status[j] = KETE_ST_MAX_STEPS;
    }
}

}  // namespace

size_t adjoint_lds_bytes(const AdjParams& p) {
    return ((size_t)p.eph.n_body * p.max_win_segs * 3 * p.eph.deg1 + (size_t)kNodes * p.eph.n_body * 6) *
           sizeof(double);
}

hipError_t launch_adjoint(const AdjParams& p, int mode, hipStream_t s) {
    const int grid = (int)((p.n_obj + 63) / 64);
    if (grid == 0) return hipSuccess;
    if (mode == KETE_ADJ_FWD)
        hipLaunchKernelGGL(k_adjoint_fwd, dim3(grid), dim3(64), adjoint_lds_bytes(p), s, p);
    else
        hipLaunchKernelGGL(k_adjoint_bwd, dim3(grid), dim3(64), adjoint_lds_bytes(p), s, p);
    return hipGetLastError();
}

size_t adjoint_step_doubles() { return kStepDoubles + 8 * kJacDoubles; }

}  // namespace kete
