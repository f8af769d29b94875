// Gradient of sky-position residuals with respect to the initial state.
//
// Forward: the collocation integrator of the propagation kernels (8-lane
// group per object, wave-shared steps) takes its own steps; checkpoint c
// is the state at the first step start at or after t0 + c ckpt_days, and
// observations at per-object times are read off the step's collocation
// polynomial, hopped with light time to the emission point (Sect. 2) and
// turned into RA/Dec.
//
// Backward: the discrete adjoint of that forward map.  Checkpoint
// segments are processed last to first: the segment's steps are
// recomputed from its checkpoint (same windows and step sequence, bit for
// bit) while each step's start, size and force Jacobians at its 8 nodes
// are stored; the steps are then swept in reverse, solving the linear
// stage equations of the step's transpose by fixed-point iteration.  The
// recompute of the next segment runs on a second stream during a sweep.  The light-time hop's
// Jacobian comes from one forward-mode (six-direction dual number)
// evaluation of the universal-variable solution at its converged anomaly
// plus the implicit light-time term.
#include <math.h>

#include "kete_adjoint.hpp"
#include "kete_radau.hpp"

#include <mutex>

namespace kete {
namespace {

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
    __device__ bool covers(double) const { return true; }
    __device__ void center(double) const {}
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
    return lighttime(sun, p.eph.gm[0], p.smu, p.c_light, p.lt_tol, p.lt_iter, t_obs, r0, v0, t_obs, o, d, tau, ve,
                     &chi, p.kepler_iter);
}

// The same hop from the light time and universal anomaly the forward
// converged to: one warm-started Kepler evaluation, no light-time loop.
__device__ __forceinline__ void hop_known(const AdjParams& p, const SunGlobal& sun, double t_obs, const double xs[3],
                                          const double vs[3], const double o[3], double tau, double& chi,
                                          double d[3], double ve[3], double r0[3], double v0[3]) {
    double S[3], Sd[3], r[3], v[3], Se[3], Sde[3];
    sun.eval(t_obs, S, Sd);
    for (int i = 0; i < 3; ++i) { r0[i] = xs[i] - S[i]; v0[i] = vs[i] - Sd[i]; }
    kepler_uv(p.eph.gm[0], p.smu, r0, v0, -tau, chi, r, v, p.kepler_iter);
    sun.eval(t_obs - tau, Se, Sde);
    for (int i = 0; i < 3; ++i) {
        d[i] = Se[i] + r[i] - o[i];
        ve[i] = Sde[i] + v[i];
    }
}

// dL/d(x, v) at t_obs from dL/d(ra, dec) through the sky projection and
// the light-time hop (implicit tau: dx_e = P dz - v_e (u . dx_e) / c),
// given the forward's light time and universal anomaly.
__device__ void hop_vjp(const AdjParams& p, const SunGlobal& sun, double t_obs, const double xs[3], const double vs[3],
                        const double o[3], double tau, double chi, double gra, double gdec, double lx[3],
                        double lv[3]) {
    double d[3], ve[3], r0[3], v0[3];
    hop_known(p, sun, t_obs, xs, vs, o, tau, chi, d, ve, r0, v0);
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
// Both passes integrate each object as an 8-lane group (one lane per
// collocation node, 8 objects per wavefront, wave-shared steps) with the
// step loop of the propagation kernels.

// Checkpoint c of object j at time t: state, the step size to resume
// with, a failure flag, the force at the state (with whether it was
// evaluated yet), and the last accepted step with its node increments, so
// that a recompute repeats the forward's steps exactly (extrapolated
// corrector starts included).  Lanes 0..7 of the group write the first
// eight values, lanes 0..3 the force, lanes 0..6 their node's increment
// and lane 7 the step and the time.
__device__ __forceinline__ void save_ckpt_g8(const AdjParams& p, int c, int j, int gl, const G8State& S, double t) {
    double* ck = p.ckpt + ((size_t)c * p.n_obj + j) * kCkptDoubles;
    const double v = gl < 6 ? state_component(S.x0, S.v0, gl)
                            : gl == 6 ? S.hw : (S.active ? 0.0 : (double)(S.status ? S.status : 1));
    ck[gl] = v;
    const double f = gl == 0 ? S.F0[0] : gl == 1 ? S.F0[1] : gl == 2 ? S.F0[2] : (S.haveF0 ? 1.0 : 0.0);
    if (gl < 4) ck[8 + gl] = f;
    if (gl < 7) {
#pragma unroll
        for (int i = 0; i < 3; ++i) ck[12 + 3 * gl + i] = S.Dp[i];
    } else {
        ck[33] = S.hprev;
        ck[34] = t;
    }
}


__device__ __forceinline__ void init_lane_state(const AdjParams& p, bool valid, int j, G8State& S) {
    S.status = 0;
    S.active = valid;
    for (int i = 0; i < 3; ++i) {
        S.x0[i] = valid ? p.x0[6 * j + i] : (i == 0 ? 1.0 : 0.0);
        S.v0[i] = valid ? p.x0[6 * j + 3 + i] : 0.0;
        S.F0[i] = 0.0;
    }
    S.hp_new = kInf;
    S.haveF0 = false;
}

template <int NB, int NGR, int DEG1>
__global__ __launch_bounds__(64, 3) void k_adjoint_fwd(const AdjParams p) {
    extern __shared__ double smem[];
    const int lane = threadIdx.x;
    const int gl = lane & (kGroup - 1);
    const int node = gl < 7 ? gl + 1 : 7;
    const EphemArgs& E = p.eph;
    const int bstride = p.max_win_segs * 3 * E.deg1;
    double* coefL = smem;
    double* e8 = smem + (((size_t)E.n_body * bstride + 1) & ~(size_t)1);
    g8_table_init(E, lane, e8);
    NodeRow R;
    load_node_row(p.rc, node, R);
    // dense-output rows, read from LDS at the observations inside a step
    __shared__ double dcoef[kDenseCoefDoubles];
    for (int i = lane; i < kDenseCoefDoubles; i += 64) dcoef[i] = p.dense_coef[i];
    __syncthreads();
    const long gi = ((long)blockIdx.x * 64 + lane) / kGroup;
    const bool valid = gi < p.n_obj;
    const int j = valid ? p.perm[gi] : 0;
    G8State S;
    init_lane_state(p, valid, j, S);
    S.hw = groups_min(valid ? p.h_pref[j] : kInf);
    if (!(S.hw < kInf)) S.hw = p.h_init;
    S.t = p.t0;
    G8Count C;
    const int K = p.k_obs;
    int kobs = 0;
    const double* tob = p.t_obs + (size_t)j * K;
    auto store_obs = [&](int k, const double X[3], const double V[3]) {
        if (gl < 6) p.obs_state[((size_t)j * K + k) * 6 + gl] = state_component(X, V, gl);
    };
    // observations at the start epoch
    if (valid) while (kobs < K && tob[kobs] <= S.t) { store_obs(kobs, S.x0, S.v0); ++kobs; }
    // Checkpoint c (1 .. C - 1) is the state at the first accepted step
    // start at or after t0 + c ckpt_days (wave-uniform: the wavefront's
    // objects share their steps), so steps are not cut at checkpoints.
    int c_next = 1;
    auto visit = [&](double ts, double h, const double dn[3], const G8State& St) {
        while (c_next < p.n_ckpt && ts >= p.t0 + c_next * p.ckpt_days) {
            if (valid) save_ckpt_g8(p, c_next, j, gl, St, ts);
            ++c_next;
        }
        const double te = ts + h;
        auto pending = [&]() {
            return valid && St.active && kobs < K && (h > 0 ? tob[kobs] <= te : tob[kobs] >= te);
        };
        bool pend = pending();
        if (__ballot(pend) == 0ull) return;
        // the step's node increments into the group's exchange rows
        double* xg = g8_xch(e8, E.n_body, lane / kGroup);
        wave_lds_sync();
        xg[gl] = dn[0];
        xg[8 + gl] = dn[1];
        xg[16 + gl] = dn[2];
        wave_lds_sync();
        while (__ballot(pend) != 0ull) {
            if (pend) {
                double X[3], V[3];
                dense_state_rows(dcoef, xg, St.x0, St.v0, St.F0, h, (tob[kobs] - ts) / h, X, V);
                store_obs(kobs, X, V);
                ++kobs;
            }
            pend = pending();
        }
    };
    if (valid) save_ckpt_g8(p, 0, j, gl, S, S.t);
    // windows on the fixed grid (aligned_window), so a recompute that starts
    // at a checkpoint cuts its steps where this run did
    const int wsegs = p.max_win_segs - 1;
    int lo = 1, hi = 0;                          // nothing staged yet
    while (S.t < p.t_end) {
        const Window W = aligned_window(S.t, p.t_end, E.t_start, E.seg_days, E.inv_seg, E.n_seg, wsegs);
        ensure_window(E, W.seg_lo, W.seg_hi, lo, hi, coefL, bstride);
        g8_integrate<NB, NGR, DEG1, kGroup, kStartExtrapolateHeld>(p, R, node, gl, lane / kGroup, lane, coefL, bstride,
                                                                   e8, lo, hi, W.t_b, S, C, visit);
    }
    // checkpoints no step start reached: the end state
    for (; c_next <= p.n_ckpt; ++c_next)
        if (valid) save_ckpt_g8(p, c_next, j, gl, S, p.t_end);
    if (valid && gl == 0) p.status[j] = S.status;
}

// Sky position of every observation from its stored state (forward), one
// lane per (object, observation); failed objects get NaN, and so does an
// observation whose hop ends on the Kepler iteration cap (its light time
// is stored as NaN for k_obs_status).
__global__ __launch_bounds__(256) void k_obs_sky(const AdjParams p) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)p.n_obj * p.k_obs) return;
    const int64_t j = i / p.k_obs;
    double* out = p.sky_out + 2 * i;
    if (p.status[j] != 0) { out[0] = out[1] = __builtin_nan(""); return; }
    const SunGlobal sun{p.eph};
    const double* st = p.obs_state + 6 * i;
    double d[3], tau, ve[3], r0[3], v0[3], chi;
    if (hop(p, sun, p.t_obs[i], st, st + 3, p.obs_pos + 3 * i, d, tau, ve, r0, v0, chi)) {
        out[0] = out[1] = __builtin_nan("");
        p.obs_hop[2 * i] = p.obs_hop[2 * i + 1] = __builtin_nan("");
        return;
    }
    double ra, dec, J[6];
    radec(d, p.cos_eps, p.sin_eps, ra, dec, J);
    out[0] = ra;
    out[1] = dec;
    p.obs_hop[2 * i] = tau;
    p.obs_hop[2 * i + 1] = chi;
}

// Objects with an observation whose hop failed (NaN light time) get
// KETE_ST_KEPLER_NOCONV, so the backward gives them a zero gradient.  A
// kernel of its own: k_obs_sky's lanes of one object read the status
// they would otherwise be writing.
__global__ void k_obs_status(const AdjParams p) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= p.n_obj || p.status[j] != 0) return;
    for (int k = 0; k < p.k_obs; ++k) {
        const double tau = p.obs_hop[2 * (j * p.k_obs + k)];
        if (!(tau == tau)) { p.status[j] = KETE_ST_KEPLER_NOCONV; return; }
    }
}

// dL/d(state) of every observation (backward), one lane per observation.
__global__ __launch_bounds__(256) void k_obs_vjp(const AdjParams p) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)p.n_obj * p.k_obs) return;
    const int64_t j = i / p.k_obs;
    double* g = p.obs_grad + 6 * i;
    if (p.status[j] != 0) { for (int c = 0; c < 6; ++c) g[c] = 0.0; return; }
    const SunGlobal sun{p.eph};
    const double* st = p.obs_state + 6 * i;
    double lX[3], lV[3];
    hop_vjp(p, sun, p.t_obs[i], st, st + 3, p.obs_pos + 3 * i, p.obs_hop[2 * i], p.obs_hop[2 * i + 1],
            p.dL_dsky[2 * i], p.dL_dsky[2 * i + 1], lX, lV);
    for (int c = 0; c < 3; ++c) { g[c] = lX[c]; g[3 + c] = lV[c]; }
}

// ---------------------------------------------------------------- backward
// Constants of the reverse sweep held by lane gl of a group.  Lane m - 1
// (m = 1..7) owns stage m: cA[n-1] = A_m(s_n), cB[n-1] = B_m(s_n) and the
// step-end weights gA = A_m(1), gB = B_m(1); lane 7 owns the step start:
// s_n^2/2 - sum_m A_m(s_n), s_n - sum_m B_m(s_n), and the same at s = 1.
struct AdjCols {
    double cA[7], cB[7], gA, gB;
};
constexpr int kAdjColDoubles = 16;
static_assert(sizeof(AdjCols) == kAdjColDoubles * sizeof(double), "AdjCols is 16 doubles");
static_assert(kAdjTabDoubles == kGroup * (kAdjColDoubles + 18), "table size");

__device__ __forceinline__ void load_adj_cols(const RadauConst& rc, int gl, AdjCols& c) {
#pragma unroll
    for (int n = 1; n <= 8; ++n) {
        double sA = 0.0, sB = 0.0, a = 0.0, b = 0.0;
#pragma unroll
        for (int m = 0; m < 7; ++m) {
            sA += rc.A[n][m];
            sB += rc.B[n][m];
            a = (gl == m) ? rc.A[n][m] : a;
            b = (gl == m) ? rc.B[n][m] : b;
        }
        if (gl == 7) { a = rc.half_s2[n] - sA; b = rc.s[n] - sB; }
        if (n < 8) { c.cA[n - 1] = a; c.cB[n - 1] = b; }
        else { c.gA = a; c.gB = b; }
    }
}

// Per-node constants of the 8 lanes of a group (LDS rows, indexed by gl).
__device__ __forceinline__ void fill_node_rows(const RadauConst& rc, int tid, NodeRow* rows) {
    if (tid < kGroup) {
        NodeRow r;
        load_node_row(rc, tid < 7 ? tid + 1 : 7, r);
        rows[tid] = r;
    }
}

// Backward, first half for checkpoint segment c: recompute the segment from
// its checkpoint with the forward's grouping, windows and step sequence
// (one wavefront per block: the checkpoints' times differ between
// wavefronts), storing each step's start and size and this lane's node
// Jacobians (lane 7: node 0).  The step count (plus kSegOverflow when the
// step store was too small) goes to seg_ns[wave].
constexpr int kSegOverflow = 1 << 30;
static_assert(kAdjLanes == kGroup, "adjoint wavefronts hold 8 objects");

template <int NB, int NGR, int DEG1>
__global__ __launch_bounds__(64, 2) void k_adj_recompute(const AdjParams p, const int c) {
    extern __shared__ double smem[];
    const int lane = threadIdx.x;
    const int gl = lane & (kGroup - 1);
    const int node = gl < 7 ? gl + 1 : 7;
    const int jnode = gl < 7 ? gl + 1 : 0;          // node whose Jacobians this lane keeps
    const EphemArgs& E = p.eph;
    const long wave = blockIdx.x;
    const long gi_raw = wave * kGroup + lane / kGroup;
    const bool valid = gi_raw < p.n_obj;
    const size_t gi = valid ? (size_t)gi_raw : 0;   // scratch slot (invalid groups read slot 0, never write)
    const int j = valid ? p.perm[gi] : 0;
    const size_t N = p.n_obj;
    // this checkpoint's time and the next one's (the same for every object
    // of the wavefront); a segment with no step start stores nothing
    const double t_c = groups_max(valid ? p.ckpt[((size_t)c * N + j) * kCkptDoubles + 34] : -kInf);
    const double t_stop = groups_max(valid ? p.ckpt[((size_t)(c + 1) * N + j) * kCkptDoubles + 34] : -kInf);
    if (!(t_c < t_stop)) {
        if (lane == 0) p.seg_ns[wave] = 0;
        return;                                     // the whole block: one wavefront
    }
    const int bstride = p.max_win_segs * 3 * E.deg1;
    double* coefL = smem;
    double* e8 = smem + (((size_t)E.n_body * bstride + 1) & ~(size_t)1);
    g8_table_init(E, lane, e8);
    __shared__ NodeRow rows[kGroup];
    fill_node_rows(p.rc, lane, rows);
    __syncthreads();
    const NodeRow& R = rows[gl];
    bool overflow_steps = false;
    G8State S;
    init_lane_state(p, false, j, S);
    double hw = 0.0, hprev = -kInf;
    bool have_f0 = false;
    if (valid) {
        const double* ck = p.ckpt + ((size_t)c * N + j) * kCkptDoubles;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            S.x0[i] = ck[i]; S.v0[i] = ck[3 + i]; S.F0[i] = ck[8 + i];
            S.Dp[i] = gl < 7 ? ck[12 + 3 * gl + i] : 0.0;
        }
        hw = ck[6];
        S.active = ck[7] == 0.0;
        have_f0 = ck[11] != 0.0;
        hprev = ck[33];
    }
    S.hw = groups_max(valid ? hw : 0.0);        // the same value in every valid group
    S.hprev = groups_max(hprev);                // likewise (invalid groups give -inf)
    S.haveF0 = __ballot(have_f0) != 0ull;       // as in the forward at this checkpoint
    S.t = t_c;
    G8Count Cn;
    int ns = 0;
        auto store = [&](double ts, double h, const double dn[3], const G8State& St) {
            if (ns >= p.s_max) { overflow_steps = true; return; }
            double D[7][3];
            g8_exchange(g8_xch(e8, E.n_body, lane / kGroup), gl, dn, D);
            if (valid) {
                double* sp = p.steps + (size_t)ns * kStepDoubles * N;
                if (gl == 6) sp[gi] = ts;
                if (gl == 7) sp[N + gi] = h;
                // state at this lane's Jacobian node
                double X[3], V[3];
                const double hh = h * h;
                #pragma unroll
                for (int i = 0; i < 3; ++i) {
                    if (jnode == 0) { X[i] = St.x0[i]; V[i] = St.v0[i]; continue; }
                    double ax = R.hs2 * St.F0[i], av = R.s * St.F0[i];
                    #pragma unroll
                    for (int m = 0; m < 7; ++m) { ax = fma(R.A[m], D[m][i], ax); av = fma(R.B[m], D[m][i], av); }
                    X[i] = fma(hh, ax, fma(R.s * h, St.v0[i], St.x0[i]));
                    V[i] = fma(h, av, St.v0[i]);
                }
                double Jx[9], Jv[9];
                accel_jac8<NB, NGR>(e8 + jnode * g8_row(E.n_body), E, X, V, Jx, Jv);
                double* jp = p.jac + (size_t)ns * 8 * kJacDoubles * N;
                #pragma unroll
                for (int q = 0; q < 9; ++q) {
                    jp[((size_t)q * N + gi) * 8 + jnode] = Jx[q];
                    jp[((size_t)(9 + q) * N + gi) * 8 + jnode] = Jv[q];
                }
            }
            ++ns;
        };
    // the forward's windows (aligned_window) from the checkpoint on, until
    // the step start where the forward took the next checkpoint
    const int wsegs = p.max_win_segs - 1;
    int lo = 1, hi = 0;                          // nothing staged yet
    while (S.t < t_stop) {
        const Window W = aligned_window(S.t, p.t_end, E.t_start, E.seg_days, E.inv_seg, E.n_seg, wsegs);
        ensure_window(E, W.seg_lo, W.seg_hi, lo, hi, coefL, bstride);
        g8_integrate<NB, NGR, DEG1, kGroup, kStartExtrapolateHeld>(p, R, node, gl, lane / kGroup, lane, coefL, bstride,
                                                                   e8, lo, hi, W.t_b, S, Cn, store, true, t_stop);
    }
    if (lane == 0 && wave * kGroup < p.n_obj) p.seg_ns[wave] = min(ns, p.s_max) | (overflow_steps ? kSegOverflow : 0);
}

// Constant rows of the reverse sweep, for the 8 lanes of a group: the
// stage columns (AdjCols) and the dense-output rows alpha(sig) =
// sum_k dr[k] sig^(k+2) + dr[16] sig^2, beta(sig) = sum_k dr[8+k] sig^(k+1)
// + dr[17] sig of stage m = lane + 1 (lanes 0..6), and minus the sum over
// the stages for lane 7.  One block of 64 threads.
__global__ void k_adj_tables(const AdjParams p) {
    const int lane = threadIdx.x;
    if (lane >= kGroup) return;
    const RadauConst& rc = p.rc;
    AdjCols q;
    load_adj_cols(rc, lane, q);
    double* col = p.adj_tab + lane * kAdjColDoubles;
    for (int n = 0; n < 7; ++n) { col[n] = q.cA[n]; col[7 + n] = q.cB[n]; }
    col[14] = q.gA;
    col[15] = q.gB;
    double* dr = p.adj_tab + kGroup * kAdjColDoubles + lane * 18;
    for (int k = 0; k < 8; ++k) {
        double a = 0.0, b = 0.0, sa = 0.0, sb = 0.0;
        for (int m = 0; m < 7; ++m) {
            sa += rc.Ap[m][k]; sb += rc.Bp[m][k];
            if (m == lane) { a = rc.Ap[m][k]; b = rc.Bp[m][k]; }
        }
        dr[k] = lane < 7 ? a : -sa;
        dr[8 + k] = lane < 7 ? b : -sb;
    }
    dr[16] = lane < 7 ? 0.0 : 0.5;
    dr[17] = lane < 7 ? 0.0 : 1.0;
}

// Backward, second half for checkpoint segment c: the reverse sweep over
// the stored steps, one 8-lane group per object (lane m - 1 holds the
// stage cotangent mu_m, lane 7 the step-start term), carrying the state
// cotangent (lx, lv), the next observation and the overflow flag from
// segment c + 1 in adj_state; segment 0 adds the observations at the start
// epoch and writes the gradient.
__global__ __launch_bounds__(64) void k_adj_sweep(const AdjParams p, const int c) {
    const int lane = threadIdx.x;
    const int gl = lane & (kGroup - 1);
    const int jnode = gl < 7 ? gl + 1 : 0;
    const RadauConst& rc = p.rc;
    // exchange slots of the reverse sweep: [group][node lane][6] (W, U)
    __shared__ double xw_all[kWave * 6];
    double* xw = xw_all + (lane / kGroup) * kGroup * 6;
    __shared__ AdjCols cols[kGroup];
    __shared__ double drow[kGroup][18];      // own dense-output row (see below)
    {
        // the constant rows, computed once per call by k_adj_tables
        const double* src = p.adj_tab;
        double* dst = &cols[0].cA[0];
        for (int i = lane; i < kAdjTabDoubles; i += kWave)
            (i < kGroup * kAdjColDoubles ? dst[i] : drow[0][i - kGroup * kAdjColDoubles]) = src[i];
    }
    __syncthreads();
    const AdjCols& Q = cols[gl];
    const double* dr = drow[gl];
    const long wave = blockIdx.x;
    const long gi_raw = wave * kGroup + lane / kGroup;
    const bool valid = gi_raw < p.n_obj;
    const size_t gi = valid ? (size_t)gi_raw : 0;
    const int j = valid ? p.perm[gi] : 0;
    const size_t N = p.n_obj;
    const int K = p.k_obs;
    const double* tob = p.t_obs + (size_t)j * K;
    const bool ok_final = valid && p.status[j] == 0;
    double lx[3] = {0.0, 0.0, 0.0}, lv[3] = {0.0, 0.0, 0.0};
    int kb = K - 1;
    bool overflow_steps = false;
    double* as = p.adj_state + (size_t)j * kAdjStateDoubles;
    if (c < p.n_ckpt - 1 && valid) {
#pragma unroll
        for (int i = 0; i < 3; ++i) { lx[i] = as[i]; lv[i] = as[3 + i]; }
        kb = (int)as[6];
        overflow_steps = as[7] != 0.0;
    }
    const int sn = p.seg_ns[wave];
    const int ns = sn & (kSegOverflow - 1);
    overflow_steps = overflow_steps || (sn & kSegOverflow) != 0;
    for (int st = ns - 1; st >= 0; --st) {
        const double* sp = p.steps + (size_t)st * kStepDoubles * N;
        const double ts = sp[gi];
        const double h = valid ? sp[N + gi] : 1.0;
        const double hh = h * h;
        // output cotangents: the step end and the observations inside
        double G[3], gx0[3], gv0[3];
        #pragma unroll
        for (int i = 0; i < 3; ++i) {
            G[i] = hh * Q.gA * lx[i] + h * Q.gB * lv[i];
            gx0[i] = lx[i];
            gv0[i] = h * lx[i] + lv[i];
        }
        auto pending = [&]() { return ok_final && kb >= 0 && (h > 0 ? tob[kb] > ts : tob[kb] < ts); };
        bool pend = pending();
        while (__ballot(pend) != 0ull) {
            if (pend) {
                const double sig = (tob[kb] - ts) / h;
                const double* og = p.obs_grad + ((size_t)j * K + kb) * 6;
                const double lX[3] = {og[0], og[1], og[2]}, lV[3] = {og[3], og[4], og[5]};
                // this lane's dense-output weights at sig
                double a = dr[7], b = dr[15];
                #pragma unroll
                for (int k = 6; k >= 0; --k) { a = fma(a, sig, dr[k]); b = fma(b, sig, dr[8 + k]); }
                a = (a + dr[16]) * sig * sig;
                b = (b + dr[17]) * sig;
                #pragma unroll
                for (int i = 0; i < 3; ++i) {
                    G[i] += hh * a * lX[i] + h * b * lV[i];
                    gx0[i] += lX[i];
                    gv0[i] += sig * h * lX[i] + lV[i];
                }
                --kb;
            }
            pend = pending();
        }
        // this lane's Jacobians
        const double* jp = p.jac + (size_t)st * 8 * kJacDoubles * N;
        double Jx[9], Jv[9];
        #pragma unroll
        for (int q = 0; q < 9; ++q) {
            Jx[q] = valid ? jp[((size_t)q * N + gi) * 8 + jnode] : 0.0;
            Jv[q] = valid ? jp[((size_t)(9 + q) * N + gi) * 8 + jnode] : 0.0;
        }
        // stage cotangents: mu_m = G_m + sum_n [h^2 A_m(s_n) Jx_n^T mu_n + h B_m(s_n) Jv_n^T mu_n],
        // lane m - 1 holding mu_m; lane 7 accumulates the step-start term m0
        double mu[3] = {G[0], G[1], G[2]};
        double wsum[3], usum[3], m0[3] = {0.0, 0.0, 0.0};
        double pc = 1e300, pcl;
        int it = 0;
        do {
            pcl = pc;
            ++it;
            double W[3] = {0.0, 0.0, 0.0}, U[3] = {0.0, 0.0, 0.0};
            if (gl < 7) {
                #pragma unroll
                for (int c2 = 0; c2 < 3; ++c2) {
                    double a = 0.0, b = 0.0;
                    #pragma unroll
                    for (int r = 0; r < 3; ++r) { a = fma(Jx[3 * r + c2], mu[r], a); b = fma(Jv[3 * r + c2], mu[r], b); }
                    W[c2] = a; U[c2] = b;
                }
            }
            *reinterpret_cast<double2*>(xw + 6 * gl) = make_double2(W[0], W[1]);
            *reinterpret_cast<double2*>(xw + 6 * gl + 2) = make_double2(W[2], U[0]);
            *reinterpret_cast<double2*>(xw + 6 * gl + 4) = make_double2(U[1], U[2]);
            wave_lds_sync();
            double nm[3] = {G[0], G[1], G[2]};
            #pragma unroll
            for (int i = 0; i < 3; ++i) { wsum[i] = 0.0; usum[i] = 0.0; }
            #pragma unroll
            for (int n = 1; n <= 7; ++n) {
                const double* x = xw + 6 * (n - 1);
                const double2 w01 = *reinterpret_cast<const double2*>(x);
                const double2 w2u0 = *reinterpret_cast<const double2*>(x + 2);
                const double2 u12 = *reinterpret_cast<const double2*>(x + 4);
                const double wn[3] = {w01.x, w01.y, w2u0.x}, un[3] = {w2u0.y, u12.x, u12.y};
                #pragma unroll
                for (int i = 0; i < 3; ++i) {
                    nm[i] += hh * Q.cA[n - 1] * wn[i] + h * Q.cB[n - 1] * un[i];
                    wsum[i] += wn[i];
                    usum[i] += rc.s[n] * h * wn[i] + un[i];
                }
            }
            wave_lds_sync();
            double dm = 0.0, mm = 0.0;
            if (gl < 7) {
                #pragma unroll
                for (int i = 0; i < 3; ++i) {
                    dm = fmax(dm, fabs(nm[i] - mu[i]));
                    mm = fmax(mm, fabs(nm[i]));
                    mu[i] = nm[i];
                }
            } else {
                #pragma unroll
                for (int i = 0; i < 3; ++i) m0[i] = nm[i];
            }
#pragma unroll
            for (int off = 1; off < kGroup; off <<= 1) {
                dm = fmax(dm, __shfl_xor(dm, off, kWave));
                mm = fmax(mm, __shfl_xor(mm, off, kWave));
            }
            // the ratio only steers the stopping rule: the reciprocal estimate suffices
            pc = groups_max((ok_final && mm > 0.0) ? dm * __builtin_amdgcn_rcp(mm) : 0.0);
        } while (!(pc < 1e-16) && !(it > 2 && pcl <= pc) && it < 2 * p.max_iter);
        // step-start Jacobians (lane 7) applied to m0, shared with the group
        double a0[3], b0[3];
        #pragma unroll
        for (int i = 0; i < 3; ++i) {
            double a = 0.0, b = 0.0;
            #pragma unroll
            for (int r = 0; r < 3; ++r) { a = fma(Jx[3 * r + i], m0[r], a); b = fma(Jv[3 * r + i], m0[r], b); }
            a0[i] = __shfl(a, 7, kGroup);
            b0[i] = __shfl(b, 7, kGroup);
        }
        #pragma unroll
        for (int i = 0; i < 3; ++i) {
            lx[i] = gx0[i] + wsum[i] + a0[i];
            lv[i] = gv0[i] + usum[i] + b0[i];
        }
    }
    if (c > 0) {
        if (valid) {
            const double v = gl < 6 ? state_component(lx, lv, gl) : gl == 6 ? (double)kb : (overflow_steps ? 1.0 : 0.0);
            as[gl] = v;
        }
        return;
    }
    // observations at the start epoch
    if (ok_final) {
        while (kb >= 0) {
            const double* og = p.obs_grad + ((size_t)j * K + kb) * 6;
            #pragma unroll
            for (int i = 0; i < 3; ++i) { lx[i] += og[i]; lv[i] += og[3 + i]; }
            --kb;
        }
    }
    if (valid) {
        const bool good = ok_final && !overflow_steps;
        if (gl < 6) p.grad[6 * j + gl] = good ? state_component(lx, lv, gl) : 0.0;
        if (gl == 0 && overflow_steps && p.status[j] == 0) p.status[j] = KETE_ST_MAX_STEPS;
    }
}

}  // namespace

size_t adjoint_lds_bytes(const AdjParams& p) {
    return ((((size_t)p.eph.n_body * p.max_win_segs * 3 * p.eph.deg1 + 1) & ~(size_t)1) +
            (size_t)g8_wave_doubles(p.eph.n_body)) * sizeof(double);
}


// A second stream per device for the backward recomputes: created once, at
// the default priority, not synchronizing with the null stream.
static hipError_t aux_stream(hipStream_t* out) {
    static std::mutex m;
    static hipStream_t st[64] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> g(m);
    if (!st[dev] && (e = hipStreamCreateWithFlags(&st[dev], hipStreamNonBlocking)) != hipSuccess) return e;
    *out = st[dev];
    return hipSuccess;
}

// The backward's five ordering events, created once per host thread and
// recorded again by every call (a wait uses the record made before it).
struct AdjEvents {
    hipEvent_t ev[5] = {};
    int next = 0;
};
static thread_local AdjEvents g_adj_events;
static hipError_t pooled_event(hipEvent_t* out) {
    AdjEvents& a = g_adj_events;
    const int i = a.next++ % 5;
    if (!a.ev[i]) {
        const hipError_t e = hipEventCreateWithFlags(&a.ev[i], hipEventDisableTiming);
        if (e != hipSuccess) return e;
    }
    *out = a.ev[i];
    return hipSuccess;
}

// The dense-output rows of the constants into device memory for the forward.
__global__ void k_adj_dense_coef(const AdjParams p) {
    const int i = threadIdx.x;
    if (i < 56) p.dense_coef[i] = p.rc.Ap[i / 8][i % 8];
    else if (i < kDenseCoefDoubles) p.dense_coef[i] = p.rc.Bp[(i - 56) / 8][(i - 56) % 8];
}

hipError_t launch_adjoint(const AdjParams& p, int mode, hipStream_t s) {
    const int64_t waves = ((int64_t)p.n_obj + kGroup - 1) / kGroup;
    const int grid = (int)waves;
    if (grid == 0) return hipSuccess;
    const int64_t n_o = (int64_t)p.n_obj * p.k_obs;
    const unsigned go = (unsigned)((n_o + 255) / 256);
    const size_t lds = adjoint_lds_bytes(p);
    const int nb = p.eph.n_body, ngr = p.eph.n_gr, d1 = p.eph.deg1;
    if (mode == KETE_ADJ_FWD) {
        hipLaunchKernelGGL(k_adj_dense_coef, dim3(1), dim3(128), 0, s, p);
        if (nb == 10 && ngr == 3 && d1 == 13) hipLaunchKernelGGL((k_adjoint_fwd<10, 3, 13>), dim3(grid), dim3(64), lds, s, p);
        else if (nb == 3 && ngr == 2 && d1 == 13)
            hipLaunchKernelGGL((k_adjoint_fwd<3, 2, 13>), dim3(grid), dim3(64), lds, s, p);
        else hipLaunchKernelGGL((k_adjoint_fwd<0, 0, 0>), dim3(grid), dim3(64), lds, s, p);
        if (n_o > 0) {
            hipLaunchKernelGGL(k_obs_sky, dim3(go), dim3(256), 0, s, p);
            hipLaunchKernelGGL(k_obs_status, dim3((unsigned)((p.n_obj + 255) / 256)), dim3(256), 0, s, p);
        }
        return hipGetLastError();
    }
    if (n_o > 0) hipLaunchKernelGGL(k_obs_vjp, dim3(go), dim3(256), 0, s, p);
    hipLaunchKernelGGL(k_adj_tables, dim3(1), dim3(64), 0, s, p);
    // The sweeps run on s, last segment first.  The recompute of segment c
    // needs only its checkpoint, so it runs on a second stream ahead of the
    // sweeps, into one of two step stores: the store of segment c is free
    // once the sweep of segment c + 2 has read it.
    hipStream_t r = nullptr;
    hipError_t e;
    if ((e = aux_stream(&r)) != hipSuccess) return e;
    const int C = p.n_ckpt;
    hipEvent_t ready[2] = {nullptr, nullptr}, freed[2] = {nullptr, nullptr}, start = nullptr;
    g_adj_events.next = 0;
    if ((e = pooled_event(&start)) != hipSuccess) return e;
    for (int b = 0; b < 2; ++b) {
        if ((e = pooled_event(&ready[b])) != hipSuccess || (e = pooled_event(&freed[b])) != hipSuccess) return e;
    }
    // the recomputes start after everything already queued on s (the forward's checkpoints)
    if ((e = hipEventRecord(start, s)) != hipSuccess || (e = hipStreamWaitEvent(r, start, 0)) != hipSuccess) return e;
    const size_t store = (size_t)p.s_max * kStepRecDoubles * p.n_obj;
    const size_t ns_len = (size_t)((p.n_obj + kAdjLanes - 1) / kAdjLanes);
    auto in_store = [&](int b) {
        AdjParams q = p;
        q.steps = p.steps + b * store;
        q.jac = q.steps + (size_t)p.s_max * kStepDoubles * p.n_obj;
        q.seg_ns = p.seg_ns + b * ns_len;
        return q;
    };
    auto recompute = [&](int c) -> hipError_t {
        const int b = c & 1;
        if (c + 2 < C && (e = hipStreamWaitEvent(r, freed[b], 0)) != hipSuccess) return e;
        const AdjParams q = in_store(b);
        if (nb == 10 && ngr == 3 && d1 == 13)
            hipLaunchKernelGGL((k_adj_recompute<10, 3, 13>), dim3(grid), dim3(64), lds, r, q, c);
        else if (nb == 3 && ngr == 2 && d1 == 13)
            hipLaunchKernelGGL((k_adj_recompute<3, 2, 13>), dim3(grid), dim3(64), lds, r, q, c);
        else hipLaunchKernelGGL((k_adj_recompute<0, 0, 0>), dim3(grid), dim3(64), lds, r, q, c);
        return hipEventRecord(ready[b], r);
    };
    if ((e = recompute(C - 1)) != hipSuccess) return e;
    for (int c = C - 1; c >= 0; --c) {
        const int b = c & 1;
        if ((e = hipStreamWaitEvent(s, ready[b], 0)) != hipSuccess) return e;
        // the next recompute is queued before this sweep, into the other store
        if (c > 0 && (e = recompute(c - 1)) != hipSuccess) return e;
        hipLaunchKernelGGL(k_adj_sweep, dim3(grid), dim3(64), 0, s, in_store(b), c);
        if ((e = hipEventRecord(freed[b], s)) != hipSuccess) return e;
    }
    return hipGetLastError();
}


}  // namespace kete
