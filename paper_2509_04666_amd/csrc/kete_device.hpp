// Device-side building blocks shared by the gfx950 kernels: Chebyshev
// evaluation, the universal-variable Kepler hop and the light-time loop.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kete_mi.h"

namespace kete {

constexpr int kWave = 64;

// Ephemeris description passed by value to kernels.  gm/kgr live in the
// kernel-argument segment, so per-body reads are uniform scalar loads.
struct EphemArgs {
    const double* coef;      // [n_body][n_seg][3][deg1]
    int32_t n_body, n_seg, deg1, has_gr;
    double t_start, seg_days, inv_seg;
    double gm[KETE_MAX_BODIES];
    double kgr[KETE_MAX_BODIES];   // gm/c^2 for bodies with the Eq. A.3 term, else 0
    // Slot order of the grouped integrator's perturber table: bodies with
    // the Eq. A.3 term first (n_gr of them), then the others, each group
    // in body order.  slot_of holds 4 bits per body.
    int32_t n_gr, pad_;
    unsigned long long slot_of;    // slot of body b: 4 bits at 4 b
    unsigned long long body_at;    // body in slot s: 4 bits at 4 s
    // Bodies with the Eq. A.4 term: body index, grouped-table slot,
    // k = (3/2) J2 mu R^2 and the unit pole.
    int32_t n_j2, pad2_;
    int32_t j2_body[KETE_MAX_J2], j2_slot[KETE_MAX_J2];
    double j2k[KETE_MAX_J2];
    double j2p[KETE_MAX_J2][3];
};

__host__ __device__ inline int body_slot(const EphemArgs& E, int b) { return (int)((E.slot_of >> (4 * b)) & 15ull); }
__host__ __device__ inline int slot_body(const EphemArgs& E, int s) { return (int)((E.body_at >> (4 * s)) & 15ull); }

__device__ __forceinline__ double dot3(const double* a, const double* b) {
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

// Segment index of time t (floor rule: a joint belongs to the later
// segment), clamped to [lo, hi].
__device__ __forceinline__ int seg_index(double t, double t_start, double inv_seg, int lo, int hi) {
    int k = (int)floor((t - t_start) * inv_seg);
    return k < lo ? lo : (k > hi ? hi : k);
}

// Clenshaw recurrence for sum_n c_n T_n(tau) and its tau-derivative.
__device__ __forceinline__ void clenshaw(const double* __restrict__ c, int deg1, double tau,
                                         double& p, double& dp) {
    double b1 = 0.0, b2 = 0.0, d1 = 0.0, d2 = 0.0;
    const double t2 = tau + tau;
    for (int k = deg1 - 1; k >= 1; --k) {
        double b0 = fma(t2, b1, c[k] - b2);
        double d0 = fma(t2, d1, 2.0 * b1 - d2);
        b2 = b1; b1 = b0; d2 = d1; d1 = d0;
    }
    p = fma(tau, b1, c[0] - b2);
    dp = fma(tau, d1, b1 - d2);
}

// The same two recurrences with the coefficient count fixed at compile
// time (DEG1 > 0): every coefficient load is issued before the chain
// starts.  DEG1 = 0 falls back to the runtime loops.
template <int DEG1>
__device__ __forceinline__ void clenshaw_n(const double* __restrict__ c, int deg1, double tau, double& p, double& dp) {
    if constexpr (DEG1 == 0) {
        clenshaw(c, deg1, tau, p, dp);
    } else {
        static_assert(DEG1 >= 3, "compile-time chains need degree 2 or more");
        double cc[DEG1];
#pragma unroll
        for (int k = 0; k < DEG1; ++k) cc[k] = c[k];
        const double t2 = tau + tau;
        // the first two steps from zero start values, written out: the same
        // numbers without the multiplications by zero
        double b2 = cc[DEG1 - 1], b1 = fma(t2, b2, cc[DEG1 - 2]);
        double d2 = 0.0, d1 = 2.0 * b2;
#pragma unroll
        for (int k = DEG1 - 3; k >= 1; --k) {
            const double b0 = fma(t2, b1, cc[k] - b2);
            const double d0 = fma(t2, d1, 2.0 * b1 - d2);
            b2 = b1; b1 = b0; d2 = d1; d1 = d0;
        }
        p = fma(tau, b1, cc[0] - b2);
        dp = fma(tau, d1, b1 - d2);
    }
}

// Clenshaw recurrence for the value only.
__device__ __forceinline__ double clenshaw_value(const double* __restrict__ c, int deg1, double tau) {
    double b1 = 0.0, b2 = 0.0;
    const double t2 = tau + tau;
    for (int k = deg1 - 1; k >= 1; --k) {
        const double b0 = fma(t2, b1, c[k] - b2);
        b2 = b1; b1 = b0;
    }
    return fma(tau, b1, c[0] - b2);
}

template <int DEG1>
__device__ __forceinline__ double clenshaw_value_n(const double* __restrict__ c, int deg1, double tau) {
    if constexpr (DEG1 == 0) {
        return clenshaw_value(c, deg1, tau);
    } else {
        static_assert(DEG1 >= 3, "compile-time chains need degree 2 or more");
        double cc[DEG1];
#pragma unroll
        for (int k = 0; k < DEG1; ++k) cc[k] = c[k];
        const double t2 = tau + tau;
        double b2 = cc[DEG1 - 1], b1 = fma(t2, b2, cc[DEG1 - 2]);
#pragma unroll
        for (int k = DEG1 - 3; k >= 1; --k) {
            const double b0 = fma(t2, b1, cc[k] - b2);
            b2 = b1; b1 = b0;
        }
        return fma(tau, b1, cc[0] - b2);
    }
}

// Position and velocity of one body from a segment table laid out as
// [seg][3][deg1] starting at segment `seg_base` (global or LDS).
__device__ __forceinline__ void cheb_body(const double* __restrict__ tab, int seg_base, int deg1,
                                          double t, double t_start, double seg_days, double inv_seg,
                                          int lo, int hi, double pos[3], double vel[3]) {
    int k = seg_index(t, t_start, inv_seg, lo, hi);
    double t0 = t_start + (double)k * seg_days;
    double tau = 2.0 * (t - t0) * inv_seg - 1.0;
    const double* c = tab + (size_t)(k - seg_base) * 3 * deg1;
    double sc = 2.0 * inv_seg;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        double p, dp;
        clenshaw(c + i * deg1, deg1, tau, p, dp);
        pos[i] = p;
        vel[i] = dp * sc;
    }
}

// A body's motion near one time t0 as a cubic in t - t0: position,
// velocity, acceleration and jerk of its Chebyshev segment at t0 (the
// segment's polynomial differentiated three times).  It differs from the
// segment's own value by the fourth-order term, which for the Sun's
// barycentric wobble (the inner planets' pull dominates its high
// derivatives) is below 1e-17 au within kCubicSpan of t0 but grows as
// |t - t0|^4 beyond: 3e-13 au at one day (and a segment's polynomial
// carried across the segment's end departs from the next segment's).  A
// user whose times may leave the span asks covers(t) and re-expands with
// center(t) (the light-time loop does this once for a body beyond about
// 10 au).  Evaluations load nothing, so a light-time loop that takes the
// Sun from the cubic waits on no memory between hops.
constexpr double kCubicSpan = 0.0625;        // days
struct SunCubic {
    double t0, s[3], v[3], a[3], j[3];
    // the body row of the segment table the cubic comes from (as cheb_body)
    const double* tab;
    int seg_base, deg1, lo, hi;
    double t_start, seg_days, inv_seg;
    __device__ void eval(double t, double pos[3], double vel[3]) const;
    __device__ bool covers(double t) const { return fabs(t - t0) <= kCubicSpan; }
    __device__ void center(double t);
};

// The cubic of the table row at t, into S (whose table fields are set).
// T_n and its first three derivatives follow the Chebyshev recurrence
// T_{n+1} = 2x T_n - T_{n-1} differentiated:
//   T'_{n+1}   = 2 T_n   + 2x T'_n   - T'_{n-1}
//   T''_{n+1}  = 4 T'_n  + 2x T''_n  - T''_{n-1}
//   T'''_{n+1} = 6 T''_n + 2x T'''_n - T'''_{n-1}.
// Terms n >= 2 go in chunks of kChunk: a chunk's coefficient loads (all
// three coordinates) are issued together, and only one chunk is held in
// registers at a time (small chunks where registers are scarce).
template <int kChunk = 7>
__device__ __forceinline__ void sun_cubic_at(SunCubic& S, double t) {
    static_assert((KETE_MAX_DEGREE - 1) % kChunk == 0, "terms 2..KETE_MAX_DEGREE split into whole chunks");
    const int deg1 = S.deg1;
    const int k = seg_index(t, S.t_start, S.inv_seg, S.lo, S.hi);
    const double x = 2.0 * (t - (S.t_start + (double)k * S.seg_days)) * S.inv_seg - 1.0;
    const double* c = S.tab + (size_t)(k - S.seg_base) * 3 * deg1;
    const double x2 = x + x;
    double p[3], d1[3], d2[3], d3[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const double c0 = c[i * deg1];
        const double c1 = deg1 > 1 ? c[i * deg1 + 1] : 0.0;
        p[i] = fma(c1, x, c0);
        d1[i] = c1;
        d2[i] = 0.0;
        d3[i] = 0.0;
    }
    double t_a = 1.0, t_b = x;                      // T_{n-2}, T_{n-1}
    double u_a = 0.0, u_b = 1.0;                    // T'
    double w_a = 0.0, w_b = 0.0;                    // T''
    double z_a = 0.0, z_b = 0.0;                    // T'''
#pragma unroll 1
    for (int n0 = 2; n0 < deg1; n0 += kChunk) {
        double cc[3][kChunk];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int m = 0; m < kChunk; ++m) cc[i][m] = n0 + m < deg1 ? c[i * deg1 + n0 + m] : 0.0;
#pragma unroll
        for (int m = 0; m < kChunk; ++m) {
            const double tn = fma(x2, t_b, -t_a);
            const double un = fma(x2, u_b, fma(2.0, t_b, -u_a));
            const double wn = fma(x2, w_b, fma(4.0, u_b, -w_a));
            const double zn = fma(x2, z_b, fma(6.0, w_b, -z_a));
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                p[i] = fma(cc[i][m], tn, p[i]);
                d1[i] = fma(cc[i][m], un, d1[i]);
                d2[i] = fma(cc[i][m], wn, d2[i]);
                d3[i] = fma(cc[i][m], zn, d3[i]);
            }
            t_a = t_b; t_b = tn; u_a = u_b; u_b = un; w_a = w_b; w_b = wn; z_a = z_b; z_b = zn;
        }
    }
    const double sc = 2.0 * S.inv_seg;
    S.t0 = t;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        S.s[i] = p[i];
        S.v[i] = d1[i] * sc;
        S.a[i] = d2[i] * (sc * sc);
        S.j[i] = d3[i] * (sc * sc * sc);
    }
}

// Re-expansion inside a light-time loop: one term at a time, which keeps
// the loop's register count down (it runs for distant bodies only).
__device__ __forceinline__ void SunCubic::center(double t) { sun_cubic_at<1>(*this, t); }

__device__ __forceinline__ void SunCubic::eval(double t, double pos[3], double vel[3]) const {
    const double h = t - t0;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        pos[i] = fma(h, fma(h, fma(h, j[i] * (1.0 / 6.0), 0.5 * a[i]), v[i]), s[i]);
        vel[i] = fma(h, fma(h, 0.5 * j[i], a[i]), v[i]);
    }
}

// The table fields of a cubic for body row `tab` (layout as cheb_body).
__device__ __forceinline__ SunCubic sun_table(const double* __restrict__ tab, int seg_base, int deg1, double t_start,
                                              double seg_days, double inv_seg, int lo, int hi) {
    SunCubic S;
    S.tab = tab;
    S.seg_base = seg_base;
    S.deg1 = deg1;
    S.lo = lo;
    S.hi = hi;
    S.t_start = t_start;
    S.seg_days = seg_days;
    S.inv_seg = inv_seg;
    return S;
}

// The cubic of a table row about t.
__device__ __forceinline__ SunCubic sun_cubic(const double* __restrict__ tab, int seg_base, int deg1, double t,
                                              double t_start, double seg_days, double inv_seg, int lo, int hi) {
    SunCubic S = sun_table(tab, seg_base, deg1, t_start, seg_days, inv_seg, lo, hi);
    sun_cubic_at(S, t);
    return S;
}

// Stumpff functions c0..c3 of z: series on |z| <= 0.1 after quartering
// the argument, then c_k(4z) from c_k(z):
//   c0' = 2 c0^2 - 1, c1' = c0 c1, c2' = c1^2 / 2, c3' = (c2 + c0 c3) / 4.
__device__ __forceinline__ void stumpff(double z, double& c0, double& c1, double& c2, double& c3) {
    int n = 0;
    while (fabs(z) > 0.1 && n < 64) { z *= 0.25; ++n; }
    // c2 = sum (-z)^j/(2j+2)!, c3 = sum (-z)^j/(2j+3)!
    c2 = 1.0 / 2.0 - z * (1.0 / 24.0 - z * (1.0 / 720.0 - z * (1.0 / 40320.0 - z * (1.0 / 3628800.0
         - z * (1.0 / 479001600.0 - z * (1.0 / 87178291200.0 - z * (1.0 / 20922789888000.0)))))));
    c3 = 1.0 / 6.0 - z * (1.0 / 120.0 - z * (1.0 / 5040.0 - z * (1.0 / 362880.0 - z * (1.0 / 39916800.0
         - z * (1.0 / 6227020800.0 - z * (1.0 / 1307674368000.0 - z * (1.0 / 355687428096000.0)))))));
    c0 = 1.0 - z * c2;
    c1 = 1.0 - z * c3;
    for (; n > 0; --n) {
        double n0 = 2.0 * c0 * c0 - 1.0;
        double n1 = c0 * c1;
        double n2 = 0.5 * c1 * c1;
        double n3 = 0.25 * (c2 + c0 * c3);
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
}

// Iteration cap of one universal-variable solve unless the caller sets one.
constexpr int kKeplerIterDefault = 60;

// Two-body hop about a fixed centre: (r0, v0) -> (r, v) after dt.
// Universal anomaly chi solves
//   F(chi) = r0 chi c1 + s0 chi^2 c2 + chi^3 c3 - sqrt(mu) dt = 0,
// z = alpha chi^2, alpha = 2/r0 - v0^2/mu, s0 = r0.v0/sqrt(mu), with
// Laguerre-Conway iterations (order 5); then the Lagrange f, g functions.
// The solve has converged when the update is within 4 ulps of chi, when F
// is exactly zero, or when the update stops shrinking while already below
// 1e-12 |chi| (the rounding floor of F); it fails after max_iter updates
// without that.  `chi` carries a warm start in and the solution out (pass
// NaN for none).  Returns 0 or KETE_ST_KEPLER_NOCONV (the last iterate is
// still returned).
__device__ __forceinline__ int kepler_uv(double mu, double smu, const double r0[3], const double v0[3],
                                         double dt, double& chi, double r[3], double v[3],
                                         int max_iter = kKeplerIterDefault) {
    if (dt == 0.0) {
        for (int i = 0; i < 3; ++i) { r[i] = r0[i]; v[i] = v0[i]; }
        chi = 0.0;
        return 0;
    }
    const double r0n = sqrt(dot3(r0, r0));
    const double s0 = dot3(r0, v0) / smu;
    const double alpha = 2.0 / r0n - dot3(v0, v0) / mu;
    const double target = smu * dt;
    double x = (chi == chi) ? chi : target / r0n;
    double c0, c1, c2, c3, z;
    int it = 0, ok = 0;
    double adx_prev = 1e300;
    for (; it < max_iter; ++it) {
        z = alpha * x * x;
        stumpff(z, c0, c1, c2, c3);
        double F = r0n * x * c1 + s0 * x * x * c2 + x * x * x * c3 - target;
        double Fp = r0n * c0 + s0 * x * c1 + x * x * c2;
        double Fpp = s0 * c0 + (1.0 - alpha * r0n) * x * c1;
        double disc = fabs(16.0 * Fp * Fp - 20.0 * F * Fpp);
        double den = Fp + copysign(sqrt(disc), Fp);
        double dx = 5.0 * F / den;
        x -= dx;
        if (!(x == x)) break;
        const double adx = fabs(dx);
        if (adx <= 8.881784197001252e-16 * fabs(x) || F == 0.0 || (adx >= adx_prev && adx <= 1e-12 * fabs(x))) {
            ok = 1;
            break;
        }
        adx_prev = adx;
    }
    chi = x;
    z = alpha * x * x;
    stumpff(z, c0, c1, c2, c3);
    const double f = 1.0 - x * x * c2 / r0n;
    const double g = dt - x * x * x * c3 / smu;
    for (int i = 0; i < 3; ++i) r[i] = f * r0[i] + g * v0[i];
    const double rn = sqrt(dot3(r, r));
    const double fd = -smu * x * c1 / (rn * r0n);
    const double gd = 1.0 - x * x * c2 / rn;
    for (int i = 0; i < 3; ++i) v[i] = fd * r0[i] + gd * v0[i];
    return ok ? 0 : KETE_ST_KEPLER_NOCONV;
}

// Predicted integration step of a body (days) for sorting bodies into
// wavefronts: a fixed fraction of the shortest local time scale r^2 / |r x v|
// (the inverse angular rate, sqrt(r^3 / mu) on a circle) its two-body orbit
// about the Sun (state x, v relative to it, gravitational parameter mu)
// reaches over the interval [dt_lo, dt_hi] around the state's epoch
// (dt_lo <= 0 <= dt_hi): the perihelion distance when the orbit passes
// perihelion inside the interval, otherwise the smaller of the distances at
// its ends.  t_min receives the time (relative to the epoch) of that
// smallest distance.  Only orders the bodies; the integrator's own step
// control decides every step.
__device__ __forceinline__ double predicted_step(const double x[3], const double v[3], double mu, double dt_lo,
                                                 double dt_hi, double* t_min = nullptr) {
    const double pi2 = 6.283185307179586;
    const double rn = sqrt(dot3(x, x)), rv = dot3(x, v), v2 = dot3(v, v);
    const double hx = x[1] * v[2] - x[2] * v[1], hy = x[2] * v[0] - x[0] * v[2], hz = x[0] * v[1] - x[1] * v[0];
    const double hm = sqrt(hx * hx + hy * hy + hz * hz);
    double ev[3];
    for (int i = 0; i < 3; ++i) ev[i] = ((v2 - mu / rn) * x[i] - rv * v[i]) / mu;
    const double e = sqrt(dot3(ev, ev));
    const double alpha = 2.0 / rn - v2 / mu;
    bool peri;
    double tp = 0.0;                                  // a perihelion passage inside the interval
    if (alpha > 0.0) {
        // mean anomaly from e cos E = 1 - r / a, e sin E = r.v / sqrt(mu a)
        const double es = rv * sqrt(alpha / mu), M0 = atan2(es, 1.0 - rn * alpha) - es;
        const double n = sqrt(mu * alpha * alpha * alpha);
        const double next = (M0 <= 0.0 ? -M0 : pi2 - M0) / n, prev = (M0 >= 0.0 ? M0 : pi2 + M0) / n;
        peri = next <= dt_hi || prev <= -dt_lo;
        tp = next <= dt_hi ? next : -prev;
    } else {
        peri = (rv < 0.0 && dt_hi > 0.0) || (rv > 0.0 && dt_lo < 0.0);
        tp = rv < 0.0 ? dt_hi : dt_lo;
    }
    const double q = hm * hm / (mu * (1.0 + e));      // perihelion distance
    double rmin = q;
    if (!peri) {
        rmin = rn;
        tp = 0.0;
        const double smu = sqrt(mu);
        for (int k = 0; k < 2; ++k) {
            const double dt = k ? dt_hi : dt_lo;
            if (dt == 0.0) continue;
            double chi = __builtin_nan(""), r1[3], v1[3];
            kepler_uv(mu, smu, x, v, dt, chi, r1, v1);
            const double r1n = sqrt(dot3(r1, r1));
            if (r1n < rmin) { rmin = r1n; tp = dt; }
        }
        if (!(rmin > 0.0)) rmin = q;
    }
    if (t_min) *t_min = tp;
    return 0.05 * rmin * rmin / hm;
}

// Sun position at arbitrary times of one batch, from its coefficient
// segments [lo, hi] held at `tab` (LDS or global).
struct SunTable {
    const double* tab;
    int lo, hi, deg1;
    double t_start, seg_days, inv_seg;
    __device__ __forceinline__ void eval(double t, double pos[3], double vel[3]) const {
        cheb_body(tab, lo, deg1, t, t_start, seg_days, inv_seg, lo, hi, pos, vel);
    }
    __device__ bool covers(double) const { return true; }
    __device__ void center(double) const {}
};

// Light-time corrected direction of a body from an observer (Newtonian,
// barycentric frame, no aberration): heliocentric state (r0, v0) at t_ref,
// emission point x_e = S(t_obs - tau) + hop(r0, v0, t_obs - tau - t_ref),
// tau the root of h(tau) = |x_e - o| / c - tau.  The first guess takes the
// body along its epoch velocity in a straight line to t_obs; each hop then
// gives h and its slope h' = -(1 + u.v_e / c) (u the unit direction, v_e
// the barycentric emission velocity), and Newton's update -h / h' is taken
// until it is at most lt_tol (at most lt_iter updates).  The fixed point is
// the one the plain iteration tau <- |x_e - o| / c reaches; Newton reaches
// it in two or three hops where the plain iteration from zero takes six,
// since its error shrinks quadratically instead of by |v_e| / c a hop.
// Outputs d = x_e - o, the tau of that last hop (so that |d| / c - tau is
// within lt_tol) and the barycentric emission velocity.  Returns
// KETE_ST_KEPLER_NOCONV when any of its hops ended on the iteration cap
// kepler_iter without converging, else 0.
template <class SunT>
__device__ __forceinline__ int lighttime(SunT& sun, double mu, double smu, double c_light,
                                         double lt_tol, int lt_iter, double t_ref,
                                         const double r0[3], const double v0[3], double t_obs,
                                         const double o[3], double d[3], double& tau, double ve[3],
                                         double* chi_out = nullptr, int kepler_iter = kKeplerIterDefault) {
    double Se[3], Sde[3], r[3], v[3];
    double chi = __builtin_nan("");
    {
        sun.eval(t_obs, Se, Sde);
        const double dt = t_obs - t_ref;
        for (int i = 0; i < 3; ++i) d[i] = Se[i] + r0[i] + v0[i] * dt - o[i];
        tau = sqrt(dot3(d, d)) / c_light;
    }
    int st = 0;
    // a Sun model that holds near one time only (SunCubic) is centred on
    // the first guess when that lies outside it, and once more on the
    // solution if the loop ends outside it
#pragma unroll 1
    for (int pass = 0; pass < 2; ++pass) {
        if (!sun.covers(t_obs - tau)) sun.center(t_obs - tau);
        for (int k = 0;; ++k) {
            const double te = t_obs - tau;
            st |= kepler_uv(mu, smu, r0, v0, te - t_ref, chi, r, v, kepler_iter);
            sun.eval(te, Se, Sde);
            for (int i = 0; i < 3; ++i) {
                d[i] = Se[i] + r[i] - o[i];
                ve[i] = Sde[i] + v[i];
            }
            if (k == lt_iter) break;
            const double dn = sqrt(dot3(d, d));
            const double step = (dn / c_light - tau) / (1.0 + dot3(d, ve) / (dn * c_light));
            if (fabs(step) <= lt_tol) break;
            tau += step;
        }
        if (sun.covers(t_obs - tau)) break;
    }
    if (chi_out) *chi_out = chi;
    return st;
}

// A value known to be equal in every lane, marked as wave-uniform so that
// control flow depending on it compiles to scalar branches.
__device__ __forceinline__ double uniform(double x) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffffll));
    const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Wave-wide reductions over the 64 lanes (results are wave-uniform).
__device__ __forceinline__ double wave_max(double x) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) x = fmax(x, __shfl_xor(x, off, kWave));
    return uniform(x);
}
__device__ __forceinline__ double wave_min(double x) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) x = fmin(x, __shfl_xor(x, off, kWave));
    return uniform(x);
}

// LDS visibility between lanes of one wavefront (no block barrier).
// The lanes of a wavefront issue their LDS accesses together and the LDS
// serves one wavefront's accesses in order, so wavefront-scope fences
// suffice: they keep the compiler from moving LDS accesses across the
// call and, unlike wider scopes, make no wait for outstanding global
// loads and stores.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

}  // namespace kete
