/*
 * kete_oracle.c -- plain, slow, FP64 CPU oracle for the known-object
 * prediction path.
 *
 * TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load or call this library.  The
 * GPU product path never links, imports or executes it, and the two share
 * no code (no headers, helpers, tables or generated constants).
 *
 * Everything here is written for a reader checking it against the paper
 * (Kete: Predicting Known Minor Bodies in Images, arXiv 2509.04666):
 *   - perturber positions from Chebyshev segments (Sect. 3.2: planets are
 *     read from precomputed kernels rather than integrated), evaluated by
 *     the direct T_k / T_k' recurrences;
 *   - acceleration: Newtonian sum over registered masses (Eq. A.1, with
 *     the attractive sign written out) plus the eps = 0 post-Newtonian term
 *     (Eq. A.3) for flagged bodies and the J2 oblateness term (App. A.3,
 *     Eq. A.4) for bodies given a J2, radius and pole;
 *   - integrator: Gauss-Radau 15th order in Everhart's b/g form with the
 *     IAS15 corrector-convergence test and the predictor removed (App. A.6:
 *     the b coefficients start from zero at every step), IAS15-style step
 *     control, landing exactly on each requested epoch (Sect. 2);
 *   - universal-variable Kepler hop and Newtonian light-time fixed point
 *     (Sect. 2: two-body motion inside a batch with light delay);
 *   - brute-force field-of-view membership: inside iff every inward normal
 *     has a positive dot product with the object direction (Sect. 3.1);
 *   - forward-mode variational equations (6x6 state transition matrix)
 *     and the sky-residual loss gradient built from them;
 *   - apparent V magnitude per pair in the H-G system (Sect. 3.3).
 *
 * Compile with -O2 -ffp-contract=off (no fast-math).  OpenMP, when
 * enabled, only distributes independent objects over threads.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ERANGE (-2)
#define ORC_ECAPACITY (-3)

/* per-object status */
#define ORC_ST_OK 0
#define ORC_ST_NONFINITE 1
#define ORC_ST_STEP_UNDERFLOW 2
#define ORC_ST_MAX_STEPS 3
#define ORC_ST_KEPLER_NOCONV 4
#define ORC_ST_ERANGE 5

#define ORC_C_AU_PER_DAY 173.14463267424034
#define ORC_MAXD 21          /* 3 position coordinates + 6 variations x 3 */

typedef struct {
    int32_t n_body, n_seg, degree, pad;
    double t_start, seg_days;
    const double *coef;      /* [n_body][n_seg][3][degree+1] */
    const double *gm;        /* [n_body] au^3/day^2 */
    const uint32_t *flags;   /* [n_body], bit0: post-Newtonian term */
    const double *j2;        /* [n_body][5] or NULL: J2, radius (au), unit pole
                                (integration frame); J2 = 0: no term */
} orc_ephem;

typedef struct {
    double eps;              /* step-control tolerance on |b6|/|a| */
    double h_init;           /* first trial step (days) */
    double h_min;            /* smallest allowed step magnitude */
    double safety;           /* IAS15 safety factor (0.25) */
    double c_light;          /* speed of light, au/day (0 = default) */
    int32_t max_iter;        /* corrector iteration cap (12) */
    int32_t n_threads;       /* OpenMP threads (0 = runtime default) */
    int64_t max_steps;       /* per object */
    double h_max;            /* largest allowed step magnitude (0 = none) */
    int32_t extrapolate;     /* 1: start each step's corrector from the previous step's
                                acceleration polynomial (RADAU's predictor, which App. A.6
                                removes); 0: from zero, as the paper does (default) */
    int32_t pad;
} orc_opts;

/* ------------------------------------------------------------------ */
/* Chebyshev ephemeris (Sect. 3.2: planets from precomputed segments).  */
/* ------------------------------------------------------------------ */

/* Position and velocity of `body` at time t.  The segment is
 * k = floor((t - t_start)/seg_days); a time exactly on a joint uses the
 * later segment, the final end point uses the last segment.  Times
 * outside [t_start, t_end] are an error: an ephemeris limits the span. */
int orc_cheb(const orc_ephem *E, int body, double t, double pos[3], double vel[3])
{
    double t_end = E->t_start + E->n_seg * E->seg_days;
    if (!(t >= E->t_start && t <= t_end)) return ORC_ERANGE;
    int64_t k = (int64_t)floor((t - E->t_start) / E->seg_days);
    if (k >= E->n_seg) k = E->n_seg - 1;
    if (k < 0) k = 0;
    double t0 = E->t_start + (double)k * E->seg_days;
    double tau = 2.0 * (t - t0) / E->seg_days - 1.0;
    int m = E->degree + 1;
    for (int c = 0; c < 3; c++) {
        const double *a = E->coef + (((int64_t)body * E->n_seg + k) * 3 + c) * m;
        /* T_0 = 1, T_1 = tau, T_{n+1} = 2 tau T_n - T_{n-1};
         * T'_0 = 0, T'_1 = 1, T'_{n+1} = 2 T_n + 2 tau T'_n - T'_{n-1}. */
        double Tm1 = 1.0, T = tau, dTm1 = 0.0, dT = 1.0;
        double p = a[0], dp = 0.0;
        if (m > 1) { p += a[1] * T; dp += a[1] * dT; }
        for (int n = 2; n < m; n++) {
            double Tn = 2.0 * tau * T - Tm1;
            double dTn = 2.0 * T + 2.0 * tau * dT - dTm1;
            p += a[n] * Tn;
            dp += a[n] * dTn;
            Tm1 = T; T = Tn; dTm1 = dT; dT = dTn;
        }
        pos[c] = p;
        if (vel) vel[c] = dp * 2.0 / E->seg_days;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Acceleration (Eq. A.1 Newtonian sum, Eq. A.3 relativistic term).     */
/* ------------------------------------------------------------------ */

static double dot3(const double *a, const double *b) { return a[0]*b[0] + a[1]*b[1] + a[2]*b[2]; }

/* J2 term of body m (App. A.3, Eq. A.4) written as the paper gives it:
 * in the body's equatorial frame (z along the pole p, x and y any
 * right-handed completion), with the relative position rho = x_m - x
 * taken with the sign of Eq. A.2's Newtonian term mu rho / |rho|^3,
 *   a = psi [(1 - 5 z^2/r^2) x, (1 - 5 z^2/r^2) y, (3 - 5 z^2/r^2) z],
 *   psi = (3/2) J2 mu R^2 / r^5,
 * then rotated back.  With jx, adds da/dx (= -da/drho), derived in the
 * same frame: da_i/drho_j = dpsi/drho_j c_i rho_i - psi dq/drho_j rho_i
 * + psi c_i delta_ij, q = 5 z^2/r^2, c = (1 - q, 1 - q, 3 - q). */
static void orc_j2_term(const double *j2, double mu, const double pb[3], const double x[3], double a[3],
                        double *jx)
{
    double J2 = j2[0], R = j2[1];
    double pz[3] = { j2[2], j2[3], j2[4] };
    /* x axis: the unit axis least aligned with the pole, made orthogonal */
    int ax = 0;
    if (fabs(pz[1]) < fabs(pz[ax])) ax = 1;
    if (fabs(pz[2]) < fabs(pz[ax])) ax = 2;
    double px[3] = { -pz[ax] * pz[0], -pz[ax] * pz[1], -pz[ax] * pz[2] };
    px[ax] += 1.0;
    double nx = sqrt(dot3(px, px));
    for (int i = 0; i < 3; i++) px[i] /= nx;
    double py[3] = { pz[1] * px[2] - pz[2] * px[1], pz[2] * px[0] - pz[0] * px[2], pz[0] * px[1] - pz[1] * px[0] };
    const double *Rw[3] = { px, py, pz };            /* rows: frame axes in the integration frame */
    double rw[3] = { pb[0] - x[0], pb[1] - x[1], pb[2] - x[2] };
    double rho[3];
    for (int i = 0; i < 3; i++) rho[i] = dot3(Rw[i], rw);
    double r2 = dot3(rho, rho), r = sqrt(r2);
    double psi = 1.5 * J2 * mu * R * R / (r2 * r2 * r);
    double q = 5.0 * rho[2] * rho[2] / r2;
    double c[3] = { 1.0 - q, 1.0 - q, 3.0 - q };
    double af[3];
    for (int i = 0; i < 3; i++) af[i] = psi * c[i] * rho[i];
    for (int i = 0; i < 3; i++) a[i] += af[0] * Rw[0][i] + af[1] * Rw[1][i] + af[2] * Rw[2][i];
    if (jx) {
        double Jf[9];                                  /* d af / d rho in the body frame */
        for (int i = 0; i < 3; i++)
            for (int j = 0; j < 3; j++) {
                double dpsi = -5.0 * psi * rho[j] / r2;
                double dq = (j == 2 ? 10.0 * rho[2] / r2 : 0.0) - 10.0 * rho[2] * rho[2] * rho[j] / (r2 * r2);
                Jf[3*i + j] = dpsi * c[i] * rho[i] - psi * dq * rho[i] + (i == j ? psi * c[i] : 0.0);
            }
        /* da/dx = Rw^T Jf Rw (d rho / dx = -Rw, so a minus sign) */
        for (int i = 0; i < 3; i++)
            for (int j = 0; j < 3; j++) {
                double s = 0.0;
                for (int k = 0; k < 3; k++)
                    for (int l = 0; l < 3; l++) s += Rw[k][i] * Jf[3*k + l] * Rw[l][j];
                jx[3*i + j] -= s;
            }
    }
}

/* a = sum_m [ -mu_m r / |r|^3  +  (flagged) mu_m/(c^2 |r|^3) ((4 mu_m/|r| - |w|^2) r + 4 (r.w) w)
 *            + (J2 given) Eq. A.4 ]
 * with r = x - x_m and w = v - v_m.  Optional Jacobians jx = da/dx and
 * jv = da/dv (row-major 3x3). */
int orc_accel_jac(const orc_ephem *E, double c_light, double t, const double x[3], const double v[3],
                  double a[3], double *jx, double *jv)
{
    double c2 = c_light * c_light;
    a[0] = a[1] = a[2] = 0.0;
    if (jx) memset(jx, 0, 9 * sizeof(double));
    if (jv) memset(jv, 0, 9 * sizeof(double));
    for (int b = 0; b < E->n_body; b++) {
        double pb[3], vb[3];
        int st = orc_cheb(E, b, t, pb, vb);
        if (st) return st;
        double mu = E->gm[b];
        double r[3] = { x[0] - pb[0], x[1] - pb[1], x[2] - pb[2] };
        double r2 = dot3(r, r);
        double rn = sqrt(r2);
        double ir3 = 1.0 / (r2 * rn);
        for (int i = 0; i < 3; i++) a[i] -= mu * ir3 * r[i];
        if (jx) {
            double ir5 = ir3 / r2;
            for (int i = 0; i < 3; i++)
                for (int j = 0; j < 3; j++)
                    jx[3*i + j] += mu * (3.0 * r[i] * r[j] * ir5 - (i == j ? ir3 : 0.0));
        }
        if (E->flags[b] & 1u) {
            double w[3] = { v[0] - vb[0], v[1] - vb[1], v[2] - vb[2] };
            double w2 = dot3(w, w), rw = dot3(r, w);
            double k = mu / c2;
            double s1 = 4.0 * mu / rn - w2;
            for (int i = 0; i < 3; i++) a[i] += k * ir3 * (s1 * r[i] + 4.0 * rw * w[i]);
            if (jx) {
                double ir4 = 1.0 / (r2 * r2), ir5 = ir3 / r2, ir6 = ir4 / r2;
                for (int i = 0; i < 3; i++)
                    for (int j = 0; j < 3; j++) {
                        double d = (i == j) ? 1.0 : 0.0;
                        /* d/dr of k[(4 mu r/r^4) - w^2 r/r^3 + 4 (r.w) w / r^3] */
                        double t1 = 4.0 * mu * (d * ir4 - 4.0 * r[i] * r[j] * ir6);
                        double t2 = -w2 * (d * ir3 - 3.0 * r[i] * r[j] * ir5);
                        double t3 = 4.0 * (w[i] * w[j] * ir3 - 3.0 * rw * w[i] * r[j] * ir5);
                        jx[3*i + j] += k * (t1 + t2 + t3);
                    }
            }
            if (jv) {
                for (int i = 0; i < 3; i++)
                    for (int j = 0; j < 3; j++) {
                        double d = (i == j) ? 1.0 : 0.0;
                        double t1 = -2.0 * r[i] * w[j] * ir3;
                        double t2 = 4.0 * (w[i] * r[j] + rw * d) * ir3;
                        jv[3*i + j] += k * (t1 + t2);
                    }
            }
        }
        if (E->j2 && E->j2[5 * b] != 0.0) orc_j2_term(E->j2 + 5 * b, mu, pb, x, a, jx);
    }
    return ORC_OK;
}

int orc_accel(const orc_ephem *E, double c_light, double t, const double x[3], const double v[3], double a[3])
{
    return orc_accel_jac(E, c_light, t, x, v, a, NULL, NULL);
}

/* ------------------------------------------------------------------ */
/* Gauss-Radau 15 (Everhart) with IAS15 convergence, no predictor.      */
/* ------------------------------------------------------------------ */

static double orc_hn[8];          /* node spacings, h_0 = 0 */
static double orc_cc[7][7];       /* s*prod_{j<=k}(s-h_j) = sum_m cc[k][m] s^{m+1} */
static int orc_nodes_ready = 0;

static double legendre(int n, double x)
{
    double p0 = 1.0, p1 = x;
    if (n == 0) return p0;
    for (int k = 1; k < n; k++) {
        double p2 = ((2.0 * k + 1.0) * x * p1 - k * p0) / (k + 1.0);
        p0 = p1; p1 = p2;
    }
    return p1;
}

/* The 8 Radau nodes on [0,1] are 0 and the 7 other roots of
 * P_7(x) + P_8(x) (x = 2s - 1).  Found by a sign scan and bisection.
 * Built into locals and published once; every entry point calls this
 * before any parallel region, so threads only ever read the tables. */
static void orc_init_nodes(void)
{
#ifdef _OPENMP
#pragma omp critical(orc_nodes)
#endif
    {
        if (!orc_nodes_ready) {
            double roots[8]; int nr = 0;
            const int NS = 20000;
            double xa = -1.0 + 1e-7, fa = legendre(7, xa) + legendre(8, xa);
            for (int i = 1; i <= NS && nr < 7; i++) {
                double xb = -1.0 + 1e-7 + (2.0 - 1e-7) * i / NS;
                double fb = legendre(7, xb) + legendre(8, xb);
                if (fa == 0.0 || (fa < 0) != (fb < 0)) {
                    double lo = xa, hi = xb, flo = fa;
                    for (int it = 0; it < 200; it++) {
                        double mid = 0.5 * (lo + hi);
                        double fm = legendre(7, mid) + legendre(8, mid);
                        if ((fm < 0) == (flo < 0)) { lo = mid; flo = fm; } else hi = mid;
                        if (hi - lo <= 0.0) break;
                    }
                    roots[nr++] = 0.5 * (lo + hi);
                }
                xa = xb; fa = fb;
            }
            double hn[8], cc[7][7];
            hn[0] = 0.0;
            for (int i = 0; i < 7; i++) hn[i + 1] = 0.5 * (roots[i] + 1.0);
            /* monomial coefficients of the Newton basis polynomials */
            double p[8] = {0};
            memset(cc, 0, sizeof(cc));
            p[0] = 1.0;                        /* omega_0(s) = s */
            for (int m = 0; m < 7; m++) cc[0][m] = p[m];
            for (int k = 1; k < 7; k++) {
                double q[8] = {0};
                for (int m = 0; m <= k; m++) q[m] = (m > 0 ? p[m - 1] : 0.0) - hn[k] * p[m];
                memcpy(p, q, sizeof(p));
                for (int m = 0; m < 7; m++) cc[k][m] = p[m];
            }
            memcpy(orc_hn, hn, sizeof(hn));
            memcpy(orc_cc, cc, sizeof(cc));
            orc_nodes_ready = 1;
        }
    }
}

void orc_radau_nodes(double out[8])
{
    orc_init_nodes();
    for (int i = 0; i < 8; i++) out[i] = orc_hn[i];
}

typedef int (*orc_force_fn)(void *ctx, double t, const double *x, const double *v, double *a);

typedef struct {
    int D;                     /* coordinates integrated */
    int D_ctrl;                /* leading coordinates used for convergence / step control */
    orc_force_fn force;
    void *ctx;
    double eps, h_min, h_max, safety;
    int max_iter;
    int64_t max_steps;
    /* accepted-step recording (for frozen-step finite differences) */
    double *rec; int64_t rec_cap; int64_t rec_n;
    /* replay: when set, steps are taken from this list without control */
    const double *replay; int64_t replay_n; int64_t replay_i;
    /* counters */
    int64_t n_steps, n_iter, n_reject, n_force, n_pred;
    /* corrector start from the last accepted step (extrapolate = 1) */
    int extrapolate;
    double b_prev[7][ORC_MAXD], h_prev;      /* h_prev = 0: no accepted step yet */
} orc_radau;

/* Largest ratio of a new step to the previous accepted one for which the
 * corrector starts from the extrapolated polynomial. */
#define ORC_PRED_MAX_RATIO 3.0

/* The acceleration polynomial of a step, a(s) = a0 + sum_k b_k s^(k+1) on
 * s in [0, 1], re-expanded about the step's end for a next step q times
 * as long: with s = 1 + q sigma,
 *   a = a(1) + sum_k b'_k sigma^(k+1),  b'_k = q^(k+1) sum_{j>=k} C(j+1, k+1) b_j
 * (the binomial expansion of (1 + q sigma)^(j+1)).  One coordinate. */
void orc_predict_b(const double b[7], double q, double bn[7])
{
    double qk = q;
    for (int k = 0; k < 7; k++) {
        double s = 0.0;
        for (int j = k; j < 7; j++) {
            /* C(j+1, k+1) */
            double c = 1.0;
            for (int i = 1; i <= k + 1; i++) c = c * (double)(j + 2 - i) / (double)i;
            s += c * b[j];
        }
        bn[k] = qk * s;
        qk *= q;
    }
}

/* Advance (t, x, v) to t_target exactly.  *h_io carries the desired step
 * size from call to call.  Returns a per-object status. */
static int orc_radau_advance(orc_radau *R, double *t, double *x, double *v, double t_target, double *h_io)
{
    if (!orc_nodes_ready) orc_init_nodes();
    const int D = R->D;
    double a0[ORC_MAXD], F[ORC_MAXD], xs[ORC_MAXD], vs[ORC_MAXD];
    double b[7][ORC_MAXD], g[7][ORC_MAXD];
    while (*t != t_target) {
        double dir = (t_target > *t) ? 1.0 : -1.0;
        double h;
        if (R->replay) {
            if (R->replay_i >= R->replay_n) return ORC_ST_MAX_STEPS;
            h = R->replay[R->replay_i];
        } else {
            h = dir * fabs(*h_io);
            if (R->h_max > 0 && fabs(h) > R->h_max) h = dir * R->h_max;
        }
        int landed = 0;
        if (fabs(h) >= fabs(t_target - *t)) { h = t_target - *t; landed = 1; }
        if (!R->replay && !landed && fabs(h) < R->h_min) return ORC_ST_STEP_UNDERFLOW;
        if (R->n_steps >= R->max_steps) return ORC_ST_MAX_STEPS;

        int st = R->force(R->ctx, *t, x, v, a0);
        R->n_force++;
        if (st) return ORC_ST_ERANGE;
        for (int k = 0; k < 7; k++)
            for (int c = 0; c < D; c++) b[k][c] = g[k][c] = 0.0;   /* no predictor */
        double q = R->h_prev != 0.0 ? h / R->h_prev : 0.0;
        if (R->extrapolate && q > 0.0 && q <= ORC_PRED_MAX_RATIO) {
            /* start from the previous step's polynomial, re-expanded (b), and
             * the divided differences that give the same polynomial (g):
             * b_m = sum_{k>=m} cc[k][m] g_k, solved from g_6 = b_6 down */
            for (int c = 0; c < D; c++) {
                double bo[7], bn[7];
                for (int k = 0; k < 7; k++) bo[k] = R->b_prev[k][c];
                orc_predict_b(bo, q, bn);
                for (int k = 0; k < 7; k++) b[k][c] = bn[k];
                for (int m = 6; m >= 0; m--) {
                    double s = bn[m];
                    for (int k = m + 1; k < 7; k++) s -= orc_cc[k][m] * g[k][c];
                    g[m][c] = s;
                }
            }
            R->n_pred++;
        }

        double pc_err = 1e300, pc_last = 2e300;
        int it = 0;
        double maxF7 = 0.0;
        for (;;) {
            if (pc_err < 1e-16) break;
            if (it > 2 && pc_last <= pc_err) break;
            if (it >= R->max_iter) break;
            pc_last = pc_err;
            it++;
            double max_dg6 = 0.0;
            maxF7 = 0.0;
            for (int n = 1; n <= 7; n++) {
                double s = orc_hn[n];
                for (int c = 0; c < D; c++) {
                    double xp = a0[c] / 2.0 + s * (b[0][c] / 6.0 + s * (b[1][c] / 12.0 + s * (b[2][c] / 20.0
                               + s * (b[3][c] / 30.0 + s * (b[4][c] / 42.0 + s * (b[5][c] / 56.0 + s * b[6][c] / 72.0))))));
                    xs[c] = x[c] + s * h * v[c] + (s * h) * (s * h) * xp;
                    double vp = a0[c] + s * (b[0][c] / 2.0 + s * (b[1][c] / 3.0 + s * (b[2][c] / 4.0
                               + s * (b[3][c] / 5.0 + s * (b[4][c] / 6.0 + s * (b[5][c] / 7.0 + s * b[6][c] / 8.0))))));
                    vs[c] = v[c] + s * h * vp;
                }
                st = R->force(R->ctx, *t + s * h, xs, vs, F);
                R->n_force++;
                if (st) return ORC_ST_ERANGE;
                for (int c = 0; c < D; c++) {
                    /* divided difference over the nodes 0, h_1, ..., h_n */
                    double tmp = (F[c] - a0[c]) / s;
                    for (int k = 0; k < n - 1; k++) tmp = (tmp - g[k][c]) / (s - orc_hn[k + 1]);
                    double dg = tmp - g[n - 1][c];
                    g[n - 1][c] = tmp;
                    for (int m = 0; m < n; m++) b[m][c] += orc_cc[n - 1][m] * dg;
                    if (n == 7 && c < R->D_ctrl) {
                        if (fabs(dg) > max_dg6) max_dg6 = fabs(dg);
                        if (fabs(F[c]) > maxF7) maxF7 = fabs(F[c]);
                    }
                }
            }
            pc_err = (maxF7 > 0.0) ? max_dg6 / maxF7 : 0.0;
        }
        R->n_iter += it;

        /* IAS15 step control on the highest coefficient. */
        double maxb6 = 0.0;
        for (int c = 0; c < R->D_ctrl; c++) if (fabs(b[6][c]) > maxb6) maxb6 = fabs(b[6][c]);
        double eb = (maxF7 > 0.0) ? maxb6 / maxF7 : 0.0;
        double h_new;
        if (eb > 0.0 && isfinite(eb)) h_new = h * pow(R->eps / eb, 1.0 / 7.0);
        else h_new = h / R->safety;

        if (!R->replay && fabs(h_new) < R->safety * fabs(h)) {
            /* reject: retry from the same state with the smaller step */
            R->n_reject++;
            *h_io = fabs(h_new);
            continue;
        }

        for (int c = 0; c < D; c++) {
            double xe = a0[c] / 2.0 + b[0][c] / 6.0 + b[1][c] / 12.0 + b[2][c] / 20.0 + b[3][c] / 30.0
                        + b[4][c] / 42.0 + b[5][c] / 56.0 + b[6][c] / 72.0;
            double ve = a0[c] + b[0][c] / 2.0 + b[1][c] / 3.0 + b[2][c] / 4.0 + b[3][c] / 5.0
                        + b[4][c] / 6.0 + b[5][c] / 7.0 + b[6][c] / 8.0;
            x[c] = x[c] + h * v[c] + h * h * xe;
            v[c] = v[c] + h * ve;
        }
        for (int c = 0; c < D; c++) if (!isfinite(x[c]) || !isfinite(v[c])) return ORC_ST_NONFINITE;
        *t = landed ? t_target : *t + h;
        R->n_steps++;
        for (int k = 0; k < 7; k++)
            for (int c = 0; c < D; c++) R->b_prev[k][c] = b[k][c];
        R->h_prev = h;
        if (R->replay) R->replay_i++;
        if (R->rec) { if (R->rec_n < R->rec_cap) R->rec[R->rec_n] = h; R->rec_n++; }
        if (landed) {
            if (fabs(h_new) < fabs(*h_io)) *h_io = fabs(h_new);
        } else {
            double cap = fabs(h) / R->safety;
            *h_io = fabs(h_new) > cap ? cap : fabs(h_new);
        }
    }
    return ORC_ST_OK;
}

/* ------------------------------------------------------------------ */
/* Force callbacks.                                                     */
/* ------------------------------------------------------------------ */

typedef struct { const orc_ephem *E; double c_light; int variational; } orc_nbody_ctx;

/* Coordinates: [0..2] position; with variations, [3+3k .. 5+3k] is the
 * position part of column k of the state transition matrix. */
static int orc_nbody_force(void *ctx_, double t, const double *x, const double *v, double *a)
{
    orc_nbody_ctx *ctx = (orc_nbody_ctx *)ctx_;
    if (!ctx->variational) return orc_accel_jac(ctx->E, ctx->c_light, t, x, v, a, NULL, NULL);
    double jx[9], jv[9];
    int st = orc_accel_jac(ctx->E, ctx->c_light, t, x, v, a, jx, jv);
    if (st) return st;
    for (int k = 0; k < 6; k++) {
        const double *dx = x + 3 + 3 * k, *dv = v + 3 + 3 * k;
        for (int i = 0; i < 3; i++)
            a[3 + 3*k + i] = jx[3*i] * dx[0] + jx[3*i+1] * dx[1] + jx[3*i+2] * dx[2]
                           + jv[3*i] * dv[0] + jv[3*i+1] * dv[1] + jv[3*i+2] * dv[2];
    }
    return ORC_OK;
}

/* Heliocentric two-body motion with variations (used for the Jacobian of
 * the light-time hop). */
typedef struct { double mu; } orc_kep_ctx;
static int orc_twobody_force(void *ctx_, double t, const double *x, const double *v, double *a)
{
    (void)t; (void)v;
    double mu = ((orc_kep_ctx *)ctx_)->mu;
    double r2 = dot3(x, x), rn = sqrt(r2), ir3 = 1.0 / (r2 * rn), ir5 = ir3 / r2;
    for (int i = 0; i < 3; i++) a[i] = -mu * ir3 * x[i];
    for (int k = 0; k < 6; k++) {
        const double *dx = x + 3 + 3 * k;
        double rd = dot3(x, dx);
        for (int i = 0; i < 3; i++) a[3 + 3*k + i] = mu * (3.0 * x[i] * rd * ir5 - dx[i] * ir3);
    }
    return ORC_OK;
}

static void orc_opts_fill(const orc_opts *o, orc_radau *R)
{
    R->eps = o->eps > 0 ? o->eps : 1e-9;
    R->h_min = o->h_min > 0 ? o->h_min : 1e-9;
    R->h_max = o->h_max > 0 ? o->h_max : 0.0;
    R->safety = o->safety > 0 ? o->safety : 0.25;
    R->max_iter = o->max_iter > 0 ? o->max_iter : 12;
    R->max_steps = o->max_steps > 0 ? o->max_steps : 10000000;
    R->extrapolate = o->extrapolate != 0;
}

static double orc_c(const orc_opts *o) { return (o && o->c_light > 0) ? o->c_light : ORC_C_AU_PER_DAY; }

/* Propagate n_obj states from t0 to each t_out[e] (monotone in one
 * direction), chaining epoch to epoch.  x_out is [n_out][n_obj][6].
 * stats (optional) receives [steps, iterations, rejections, force evals,
 * steps started from the extrapolated polynomial]. */
int orc_propagate(const orc_ephem *E, const orc_opts *o, int64_t n_obj, const double *x0, double t0,
                  int64_t n_out, const double *t_out, double *x_out, int32_t *status, int64_t *stats)
{
    if (n_obj < 0 || n_out < 0) return ORC_EINVAL;
    orc_init_nodes();
    int64_t s_steps = 0, s_iter = 0, s_rej = 0, s_force = 0, s_pred = 0;
#ifdef _OPENMP
    int nt = o->n_threads > 0 ? o->n_threads : omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 4) num_threads(nt) reduction(+:s_steps, s_iter, s_rej, s_force, s_pred)
#endif
    for (int64_t j = 0; j < n_obj; j++) {
        orc_nbody_ctx ctx = { E, orc_c(o), 0 };
        orc_radau R; memset(&R, 0, sizeof(R));
        R.D = 3; R.D_ctrl = 3; R.force = orc_nbody_force; R.ctx = &ctx;
        orc_opts_fill(o, &R);
        double x[3], v[3], t = t0, h = o->h_init > 0 ? o->h_init : 1.0;
        for (int i = 0; i < 3; i++) { x[i] = x0[6*j + i]; v[i] = x0[6*j + 3 + i]; }
        int st = ORC_ST_OK;
        for (int64_t e = 0; e < n_out; e++) {
            if (st == ORC_ST_OK) st = orc_radau_advance(&R, &t, x, v, t_out[e], &h);
            double *dst = x_out + (e * n_obj + j) * 6;
            for (int i = 0; i < 3; i++) {
                dst[i] = st ? NAN : x[i];
                dst[3 + i] = st ? NAN : v[i];
            }
        }
        if (status) status[j] = st;
        s_steps += R.n_steps; s_iter += R.n_iter; s_rej += R.n_reject; s_force += R.n_force; s_pred += R.n_pred;
    }
    if (stats) { stats[0] = s_steps; stats[1] = s_iter; stats[2] = s_rej; stats[3] = s_force; stats[4] = s_pred; }
    return ORC_OK;
}

/* The accepted step sizes of one object integrated from t0 to t1 on its
 * own (rec[0..*n) signed days, at most cap recorded; *n is the full count).
 * For studying how well objects that share a wavefront's steps match. */
int orc_step_trace(const orc_ephem *E, const orc_opts *o, const double x0[6], double t0, double t1,
                   double *rec, int64_t cap, int64_t *n)
{
    orc_init_nodes();
    orc_nbody_ctx ctx = { E, orc_c(o), 0 };
    orc_radau R; memset(&R, 0, sizeof(R));
    R.D = 3; R.D_ctrl = 3; R.force = orc_nbody_force; R.ctx = &ctx;
    orc_opts_fill(o, &R);
    R.rec = rec; R.rec_cap = cap;
    double x[3], v[3], t = t0, h = o->h_init > 0 ? o->h_init : 1.0;
    for (int i = 0; i < 3; i++) { x[i] = x0[i]; v[i] = x0[3 + i]; }
    int st = orc_radau_advance(&R, &t, x, v, t1, &h);
    *n = R.rec_n;
    return st;
}

/* ------------------------------------------------------------------ */
/* Universal-variable Kepler hop (Sect. 2: two-body motion in a batch). */
/* ------------------------------------------------------------------ */

/* Stumpff functions C(z) = (1 - cos sqrt z)/z, S(z) = (sqrt z - sin sqrt z)/z^{3/2},
 * continued to z < 0 with the hyperbolic functions; series for |z| <= 0.1. */
static void stumpff(double z, double *C, double *S)
{
    if (z > 0.1) {
        double sz = sqrt(z);
        *C = (1.0 - cos(sz)) / z;
        *S = (sz - sin(sz)) / (z * sz);
    } else if (z < -0.1) {
        double sz = sqrt(-z);
        *C = (cosh(sz) - 1.0) / (-z);
        *S = (sinh(sz) - sz) / ((-z) * sz);
    } else {
        /* C = sum (-z)^k/(2k+2)!, S = sum (-z)^k/(2k+3)! */
        double c = 0.0, s = 0.0, term_c = 0.5, term_s = 1.0 / 6.0;
        for (int k = 0; k < 12; k++) {
            c += term_c; s += term_s;
            term_c *= -z / ((2.0 * k + 3.0) * (2.0 * k + 4.0));
            term_s *= -z / ((2.0 * k + 4.0) * (2.0 * k + 5.0));
        }
        *C = c; *S = s;
    }
}

/* Newton iterations one Kepler solve may take before it is reported as
 * not converged (a test can lower it to force that report). */
static int orc_kep_max_iter = 200;
void orc_set_kepler_max_iter(int n) { orc_kep_max_iter = n > 0 ? n : 200; }

/* Two-body state at dt from (r0, v0) about a fixed centre with parameter mu.
 * Solves sqrt(mu) dt = sigma0 chi^2 C + (1 - alpha r0) chi^3 S + r0 chi for
 * the universal anomaly chi (alpha = 2/r0 - v0^2/mu, sigma0 = r0.v0/sqrt(mu))
 * by Newton's method inside a bisection bracket, then applies the
 * Lagrange f, g coefficients.  Returns 0 or ORC_ST_KEPLER_NOCONV. */
int orc_kepler(double mu, const double r0[3], const double v0[3], double dt, double r[3], double v[3])
{
    double rn0 = sqrt(dot3(r0, r0));
    double smu = sqrt(mu);
    double sig0 = dot3(r0, v0) / smu;
    double alpha = 2.0 / rn0 - dot3(v0, v0) / mu;
    double target = smu * dt;
    if (dt == 0.0) { for (int i = 0; i < 3; i++) { r[i] = r0[i]; v[i] = v0[i]; } return 0; }
#define KEPF(chi, Fv, Fp) do { double z_ = alpha * (chi) * (chi), C_, S_; stumpff(z_, &C_, &S_); \
        Fv = sig0 * (chi) * (chi) * C_ + (1.0 - alpha * rn0) * (chi) * (chi) * (chi) * S_ + rn0 * (chi) - target; \
        Fp = sig0 * (chi) * (1.0 - z_ * S_) + (1.0 - alpha * rn0) * (chi) * (chi) * C_ + rn0; } while (0)
    double chi = target / rn0;
    if (alpha > 0 && fabs(dt) * sqrt(mu * alpha * alpha * alpha) > 1.0) chi = target * alpha;
    /* bracket: F is increasing in chi (F' = |r| > 0) */
    double lo, hi, Flo, Fhi, Fv, Fp;
    KEPF(chi, Fv, Fp);
    if (Fv == 0.0) goto done;
    {
        double step = fabs(chi) > 0 ? fabs(chi) : 1e-3;
        if (Fv < 0) {
            lo = chi; Flo = Fv; hi = chi + step;
            KEPF(hi, Fhi, Fp);
            while (Fhi < 0) { lo = hi; Flo = Fhi; step *= 2.0; hi = hi + step; KEPF(hi, Fhi, Fp); if (!isfinite(Fhi)) return ORC_ST_KEPLER_NOCONV; }
        } else {
            hi = chi; Fhi = Fv; lo = chi - step;
            KEPF(lo, Flo, Fp);
            while (Flo > 0) { hi = lo; Fhi = Flo; step *= 2.0; lo = lo - step; KEPF(lo, Flo, Fp); if (!isfinite(Flo)) return ORC_ST_KEPLER_NOCONV; }
        }
        (void)Flo; (void)Fhi;
        int it;
        for (it = 0; it < orc_kep_max_iter; it++) {
            KEPF(chi, Fv, Fp);
            if (Fv == 0.0) break;
            if (Fv < 0) lo = chi; else hi = chi;
            double nx = chi - Fv / Fp;
            if (!(nx > lo && nx < hi)) nx = 0.5 * (lo + hi);
            double dchi = nx - chi;
            chi = nx;
            if (fabs(dchi) <= 4.0 * 2.220446049250313e-16 * fabs(chi)) break;
        }
        if (it == orc_kep_max_iter) return ORC_ST_KEPLER_NOCONV;
    }
done:;
    double z = alpha * chi * chi, C, S;
    stumpff(z, &C, &S);
    double f = 1.0 - chi * chi * C / rn0;
    double g = dt - chi * chi * chi * S / smu;
    for (int i = 0; i < 3; i++) r[i] = f * r0[i] + g * v0[i];
    double rn = sqrt(dot3(r, r));
    double fd = smu * chi * (z * S - 1.0) / (rn * rn0);
    double gd = 1.0 - chi * chi * C / rn;
    for (int i = 0; i < 3; i++) v[i] = fd * r0[i] + gd * v0[i];
#undef KEPF
    return 0;
}

/* ------------------------------------------------------------------ */
/* Light-time corrected direction (Sect. 2: correction for light delay). */
/* ------------------------------------------------------------------ */

/* From the barycentric state st at t_ref, the emission point seen from
 * observer o at t_obs: tau_0 = 0, tau_{k+1} = |x_e(t_obs - tau_k) - o|/c,
 * x_e(t) = S(t) + kepler(st - S(t_ref), t - t_ref); stop when the update is
 * below 1e-15 day (at most 10 updates).  Newtonian, no aberration.
 * Outputs d = x_e - o, tau and the emission state xe[6] (barycentric). */
int orc_lighttime(const orc_ephem *E, double c_light, double t_ref, const double st[6], double t_obs,
                  const double o[3], double d[3], double *tau_out, double xe_out[6])
{
    double S[3], Sd[3];
    if (orc_cheb(E, 0, t_ref, S, Sd)) return ORC_ST_ERANGE;
    double r0[3] = { st[0] - S[0], st[1] - S[1], st[2] - S[2] };
    double v0[3] = { st[3] - Sd[0], st[4] - Sd[1], st[5] - Sd[2] };
    double mu = E->gm[0];
    double tau = 0.0, xe[3] = {0}, ve[3] = {0};
    for (int k = 0; k <= 10; k++) {
        double te = t_obs - tau, r[3], v[3], Se[3], Sde[3];
        if (orc_kepler(mu, r0, v0, te - t_ref, r, v)) return ORC_ST_KEPLER_NOCONV;
        if (orc_cheb(E, 0, te, Se, Sde)) return ORC_ST_ERANGE;
        for (int i = 0; i < 3; i++) { xe[i] = Se[i] + r[i]; ve[i] = Sde[i] + v[i]; }
        double dd[3] = { xe[0] - o[0], xe[1] - o[1], xe[2] - o[2] };
        double tn = sqrt(dot3(dd, dd)) / c_light;
        double dtau = tn - tau;
        tau = tn;
        if (fabs(dtau) <= 1e-15) break;
    }
    /* final emission point at the converged tau */
    {
        double te = t_obs - tau, r[3], v[3], Se[3], Sde[3];
        if (orc_kepler(mu, r0, v0, te - t_ref, r, v)) return ORC_ST_KEPLER_NOCONV;
        if (orc_cheb(E, 0, te, Se, Sde)) return ORC_ST_ERANGE;
        for (int i = 0; i < 3; i++) { xe[i] = Se[i] + r[i]; ve[i] = Sde[i] + v[i]; }
    }
    for (int i = 0; i < 3; i++) d[i] = xe[i] - o[i];
    if (tau_out) *tau_out = tau;
    if (xe_out) for (int i = 0; i < 3; i++) { xe_out[i] = xe[i]; xe_out[3 + i] = ve[i]; }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Brute-force field-of-view membership (Sect. 3.1).                    */
/* ------------------------------------------------------------------ */

/* For every batch b, every frame f of the batch and every object j with
 * status 0: d = light-time direction of j from the frame's observer at the
 * frame time, hopping from the batch epoch t_ref[b] (state
 * x_epoch[b][j]); (f, s, j) is a pair when all four inward normals of
 * sub-frame s have n.d > 0.  Also returns the signed angular distance to
 * the nearest edge, asin(min_i n_i.d/|d|).  Output order: batch, frame
 * (as listed), object, sub-frame; the caller sorts.  *n_pairs receives the
 * total even when it exceeds cap.  An object any of whose light-time hops
 * fails has no pairs at all; status_out (when not NULL) gets its status
 * code, 0 for the others. */
int orc_fov(const orc_ephem *E, double c_light, int64_t n_obj, const double *x_epoch, const int32_t *status,
            int64_t n_batch, const double *t_ref, const int64_t *batch_off, const int64_t *frame_order,
            const double *ft, const double *fobs, int32_t n_sub, const double *normals,
            int64_t cap, int32_t *pf, int32_t *ps, int32_t *po, double *edge, int64_t *n_pairs, int32_t n_threads,
            int32_t *status_out)
{
    if (c_light <= 0) c_light = ORC_C_AU_PER_DAY;
    int64_t total = 0;
    int64_t n_frames_all = batch_off[n_batch];
    /* per sorted-frame counts first, so the output order is deterministic */
    int64_t *cnt = (int64_t *)calloc((size_t)(n_frames_all + 1), sizeof(int64_t));
    int32_t *failed = (int32_t *)calloc((size_t)(n_obj > 0 ? n_obj : 1), sizeof(int32_t));
    if (!cnt || !failed) { free(cnt); free(failed); return ORC_EINVAL; }
    int any_failed = 0, recount = 0;
    for (int pass = 0; pass < 2; pass++) {
#ifdef _OPENMP
        int nt = n_threads > 0 ? n_threads : omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nt)
#endif
        for (int64_t q = 0; q < n_frames_all; q++) {
            int64_t b = 0;
            while (batch_off[b + 1] <= q) b++;
            int64_t f = frame_order[q];
            int64_t k = pass ? cnt[q] : 0;
            for (int64_t j = 0; j < n_obj; j++) {
                if (status && status[j]) continue;
                if (pass == 1 || recount) {
                    int fj;
#ifdef _OPENMP
#pragma omp atomic read
#endif
                    fj = failed[j];
                    if (fj) continue;
                }
                const double *st = x_epoch + (b * n_obj + j) * 6;
                double d[3], tau;
                int lst = orc_lighttime(E, c_light, t_ref[b], st, ft[f], fobs + 3 * f, d, &tau, NULL);
                if (lst) {
#ifdef _OPENMP
#pragma omp atomic write
#endif
                    failed[j] = lst;
                    continue;
                }
                double dn = sqrt(dot3(d, d));
                for (int s = 0; s < n_sub; s++) {
                    const double *nn = normals + ((f * n_sub + s) * 4) * 3;
                    int inside = 1;
                    double mn = 1e300;
                    for (int i = 0; i < 4; i++) {
                        double p = dot3(nn + 3 * i, d);
                        if (!(p > 0.0)) inside = 0;
                        if (p / dn < mn) mn = p / dn;
                    }
                    if (!inside) continue;
                    if (pass == 0) k++;
                    else {
                        if (k < cap) { pf[k] = (int32_t)f; ps[k] = s; po[k] = (int32_t)j; if (edge) edge[k] = asin(mn); }
                        k++;
                    }
                }
            }
            if (pass == 0) cnt[q] = k;
        }
        if (pass == 0 && !recount) {
            for (int64_t j = 0; j < n_obj; j++) if (failed[j]) any_failed = 1;
            if (any_failed) {
                /* count again without the failed objects' pairs */
                recount = 1;
                pass = -1;
                continue;
            }
        }
        if (pass == 0) {
            /* exclusive scan */
            int64_t run = 0;
            for (int64_t q = 0; q < n_frames_all; q++) { int64_t c = cnt[q]; cnt[q] = run; run += c; }
            total = run;
        }
    }
    free(cnt);
    if (status_out) for (int64_t j = 0; j < n_obj; j++) status_out[j] = failed[j];
    free(failed);
    *n_pairs = total;
    return total > cap ? ORC_ECAPACITY : ORC_OK;
}

/* Light-time direction of every object (state at t_ref) from one observer
 * at t_obs: d [n][3], tau [n].  A helper for edge and sampling tests. */
int orc_directions(const orc_ephem *E, double c_light, int64_t n, const double *states, double t_ref,
                   double t_obs, const double o[3], double *d, double *tau)
{
    if (c_light <= 0) c_light = ORC_C_AU_PER_DAY;
    for (int64_t j = 0; j < n; j++) {
        int st = orc_lighttime(E, c_light, t_ref, states + 6 * j, t_obs, o, d + 3 * j, tau ? tau + j : NULL, NULL);
        if (st) return st;
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Sky residual loss and its gradient through the variational equations. */
/* ------------------------------------------------------------------ */

#define ORC_OBLIQ (84381.448 / 3600.0 * 3.14159265358979323846 / 180.0)

/* RA/Dec of an ecliptic direction after rotation to the equator by the
 * J2000 obliquity, and the Jacobian d(ra,dec)/d(d_ecl) (2x3). */
static void orc_radec(const double d[3], double *ra, double *dec, double J[6])
{
    double ce = cos(ORC_OBLIQ), se = sin(ORC_OBLIQ);
    double q[3] = { d[0], ce * d[1] - se * d[2], se * d[1] + ce * d[2] };
    double rho2 = q[0] * q[0] + q[1] * q[1], rho = sqrt(rho2), n2 = rho2 + q[2] * q[2];
    *ra = atan2(q[1], q[0]);
    if (*ra < 0) *ra += 2.0 * 3.14159265358979323846;
    *dec = atan2(q[2], rho);
    if (J) {
        double da[3] = { -q[1] / rho2, q[0] / rho2, 0.0 };
        double dd[3] = { -q[0] * q[2] / (n2 * rho), -q[1] * q[2] / (n2 * rho), rho / n2 };
        /* chain through q = R d: dq/dd = R, so row . R */
        J[0] = da[0]; J[1] = ce * da[1] + se * da[2]; J[2] = -se * da[1] + ce * da[2];
        J[3] = dd[0]; J[4] = ce * dd[1] + se * dd[2]; J[5] = -se * dd[1] + ce * dd[2];
    }
}

static double wrap_pi(double a)
{
    const double TWO_PI = 2.0 * 3.14159265358979323846;
    a = fmod(a, TWO_PI);
    if (a > 3.14159265358979323846) a -= TWO_PI;
    if (a <= -3.14159265358979323846) a += TWO_PI;
    return a;
}

/* Sky residual of one observation: r = ((ra - ra_obs) cos dec,
 * dec - dec_obs), the RA difference taken in (-pi, pi]. */
void orc_sky_residual(double ra, double dec, double ra_obs, double dec_obs, double r[2])
{
    r[0] = wrap_pi(ra - ra_obs) * cos(dec);
    r[1] = dec - dec_obs;
}

/* orc_radec for the tests: out = {ra, dec}, J = d(ra, dec)/d(d) (2x3). */
void orc_radec_of(const double d[3], double out[2], double J[6])
{
    orc_radec(d, &out[0], &out[1], J);
}

/* One object: integrate with (optionally) the 6x6 variational equations
 * from t0 through its k observation times (ascending), hop with light
 * time to each emission point, compute RA/Dec and the residual
 * r = ((ra - ra_obs) cos dec, dec - dec_obs) and L = sum |r|^2.
 * With want_grad, grad = dL/dx0 = sum_k Phi_k^T J_hop^T J_sky^T dL/dsky_k,
 * where the hop Jacobian at fixed tau comes from the heliocentric
 * two-body variational equations and the implicit tau dependence is
 * dx_e = P - v_e (u.P)/(c + u.v_e).  Steps can be recorded / replayed. */
static int orc_sky_one(const orc_ephem *E, const orc_opts *o, const double x0[6], double t0, int k,
                       const double *t_obs, const double *obs_pos, const double *radec_obs,
                       double *radec_out, double *loss, double *grad, int want_grad,
                       double *rec, int64_t rec_cap, int64_t *rec_n, const double *replay, int64_t replay_n)
{
    double c_light = orc_c(o);
    orc_nbody_ctx ctx = { E, c_light, want_grad };
    orc_radau R; memset(&R, 0, sizeof(R));
    R.D = want_grad ? 21 : 3; R.D_ctrl = 3; R.force = orc_nbody_force; R.ctx = &ctx;
    orc_opts_fill(o, &R);
    R.rec = rec; R.rec_cap = rec_cap;
    R.replay = replay; R.replay_n = replay_n;
    double x[ORC_MAXD] = {0}, v[ORC_MAXD] = {0};
    for (int i = 0; i < 3; i++) { x[i] = x0[i]; v[i] = x0[3 + i]; }
    if (want_grad) {
        /* column k of Phi: d(x, v)/d(x0_k); columns 0..2 start as unit
         * positions, 3..5 as unit velocities */
        for (int c = 0; c < 6; c++) {
            if (c < 3) x[3 + 3 * c + c] = 1.0; else v[3 + 3 * c + (c - 3)] = 1.0;
        }
    }
    double t = t0, h = o->h_init > 0 ? o->h_init : 1.0, L = 0.0;
    double g6[6] = {0};
    for (int q = 0; q < k; q++) {
        int st = orc_radau_advance(&R, &t, x, v, t_obs[q], &h);
        if (st) return st;
        double stv[6] = { x[0], x[1], x[2], v[0], v[1], v[2] };
        double d[3], tau, xe[6];
        st = orc_lighttime(E, c_light, t_obs[q], stv, t_obs[q], obs_pos + 3 * q, d, &tau, xe);
        if (st) return st;
        double ra, dec, J[6];
        orc_radec(d, &ra, &dec, J);
        radec_out[2 * q] = ra; radec_out[2 * q + 1] = dec;
        double dra = wrap_pi(ra - radec_obs[2 * q]);
        double res[2];
        orc_sky_residual(ra, dec, radec_obs[2 * q], radec_obs[2 * q + 1], res);
        double r1 = res[0], r2 = res[1];
        L += r1 * r1 + r2 * r2;
        if (!want_grad) continue;
        /* dL/d(ra, dec) */
        double gra = 2.0 * r1 * cos(dec);
        double gdec = 2.0 * r1 * (-dra * sin(dec)) + 2.0 * r2;
        /* dL/dd (ecliptic direction) */
        double gd[3];
        for (int i = 0; i < 3; i++) gd[i] = gra * J[i] + gdec * J[3 + i];
        /* heliocentric state at t_obs and the hop's two-body variational solution */
        double S[3], Sd[3];
        orc_cheb(E, 0, t_obs[q], S, Sd);
        double hx[ORC_MAXD] = {0}, hv[ORC_MAXD] = {0};
        for (int i = 0; i < 3; i++) { hx[i] = stv[i] - S[i]; hv[i] = stv[3 + i] - Sd[i]; }
        for (int c = 0; c < 6; c++) { if (c < 3) hx[3 + 3 * c + c] = 1.0; else hv[3 + 3 * c + (c - 3)] = 1.0; }
        orc_kep_ctx kc = { E->gm[0] };
        orc_radau H; memset(&H, 0, sizeof(H));
        H.D = 21; H.D_ctrl = 3; H.force = orc_twobody_force; H.ctx = &kc;
        orc_opts_fill(o, &H);
        double th = 0.0, hh = tau > 0 ? tau : 1e-3;
        int sth = orc_radau_advance(&H, &th, hx, hv, -tau, &hh);
        if (sth) return sth;
        /* P = d x_e / d(x_k, v_k) at fixed tau: rows = position part of each column */
        double P[3][6];
        for (int c = 0; c < 6; c++) for (int i = 0; i < 3; i++) P[i][c] = hx[3 + 3 * c + i];
        double dn = sqrt(dot3(d, d));
        double u[3] = { d[0] / dn, d[1] / dn, d[2] / dn };
        double uv = dot3(u, xe + 3);
        /* dL/dP = gd - u (v_e . gd)/(c + u.v_e) */
        double vg = dot3(xe + 3, gd);
        double gP[3];
        for (int i = 0; i < 3; i++) gP[i] = gd[i] - u[i] * vg / (c_light + uv);
        /* dL/d(x_k, v_k) */
        double gk[6];
        for (int c = 0; c < 6; c++) gk[c] = gP[0] * P[0][c] + gP[1] * P[1][c] + gP[2] * P[2][c];
        /* Phi_k: rows 0..2 from positions, 3..5 from velocities */
        for (int c = 0; c < 6; c++) {
            double s = 0.0;
            for (int i = 0; i < 3; i++) s += gk[i] * x[3 + 3 * c + i] + gk[3 + i] * v[3 + 3 * c + i];
            g6[c] += s;
        }
    }
    *loss = L;
    if (grad) for (int c = 0; c < 6; c++) grad[c] = g6[c];
    if (rec_n) *rec_n = R.rec_n;
    return 0;
}

/* Batch form: loss[j], radec[j][k][2] and (want_grad) grad[j][6]. */
int orc_sky_grad(const orc_ephem *E, const orc_opts *o, int64_t n_obj, const double *x0, double t0, int32_t k,
                 const double *t_obs, const double *obs_pos, const double *radec_obs,
                 double *radec_out, double *loss, double *grad, int32_t want_grad, int32_t *status)
{
    orc_init_nodes();
#ifdef _OPENMP
    int nt = o->n_threads > 0 ? o->n_threads : omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 4) num_threads(nt)
#endif
    for (int64_t j = 0; j < n_obj; j++) {
        int st = orc_sky_one(E, o, x0 + 6 * j, t0, k, t_obs + (int64_t)k * j, obs_pos + (int64_t)3 * k * j,
                             radec_obs + (int64_t)2 * k * j, radec_out + (int64_t)2 * k * j, loss + j,
                             grad ? grad + 6 * j : NULL, want_grad, NULL, 0, NULL, NULL, 0);
        if (status) status[j] = st;
    }
    return 0;
}

/* Finite-difference harness: the loss of one object with the integrator
 * step sequence either recorded (replay == NULL) or frozen to `replay`. */
int orc_loss_steps(const orc_ephem *E, const orc_opts *o, const double x0[6], double t0, int32_t k,
                   const double *t_obs, const double *obs_pos, const double *radec_obs,
                   double *loss, double *rec, int64_t rec_cap, int64_t *rec_n,
                   const double *replay, int64_t replay_n)
{
    double radec[2 * 256];
    if (k > 256) return ORC_EINVAL;
    return orc_sky_one(E, o, x0, t0, k, t_obs, obs_pos, radec_obs, radec, loss, NULL, 0,
                       rec, rec_cap, rec_n, replay, replay_n);
}

/* Membership predicate alone: inside[s] = all_i (n_{s,i} . d > 0). */
int orc_inside(int32_t n_sub, const double *normals, const double d[3], int32_t *inside, double *edge)
{
    double dn = sqrt(dot3(d, d));
    for (int s = 0; s < n_sub; s++) {
        int in = 1; double mn = 1e300;
        for (int i = 0; i < 4; i++) {
            double p = dot3(normals + (s * 4 + i) * 3, d);
            if (!(p > 0.0)) in = 0;
            if (p / dn < mn) mn = p / dn;
        }
        inside[s] = in;
        if (edge) edge[s] = asin(mn);
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Apparent V magnitude in the H-G system (Sect. 3.3: optical           */
/* magnitudes follow Bowell et al. 1989, the MPC and Horizons form).    */
/* ------------------------------------------------------------------ */

/* V = H + 5 log10(r_H Delta) - 2.5 log10((1 - G) Phi_1 + G Phi_2), with
 * Phi_i = exp(-A_i tan(alpha/2)^B_i), A = (3.33, 1.87), B = (0.63, 1.22);
 * r_H and Delta in au, alpha the phase angle in radians. */
double orc_hg_mag(double H, double G, double r_h, double delta, double alpha)
{
    double t = tan(0.5 * alpha);
    double phi1 = exp(-3.33 * pow(t, 0.63));
    double phi2 = exp(-1.87 * pow(t, 1.22));
    return H + 5.0 * log10(r_h * delta) - 2.5 * log10((1.0 - G) * phi1 + G * phi2);
}

/* Magnitude of every pair (frame pf[i], object po[i]): the emission point
 * of the object seen from the frame's observer (orc_lighttime from the
 * state x_epoch[b][j] of the frame's batch b), r = emission point less the
 * Sun at the emission time, d = emission point less the observer;
 * r_H = |r|, Delta = |d|, phase angle alpha = angle between -r and -d
 * (object to Sun, object to observer), taken here by acos of the cosine.
 * geom (optional) receives {r_H, Delta, alpha} per pair. */
int orc_pair_mags(const orc_ephem *E, double c_light, int64_t n_obj, const double *x_epoch,
                  int64_t n_batch, const double *t_ref, const int64_t *batch_off, const int64_t *frame_order,
                  int64_t n_frames, const double *frames_t, const double *frames_obs,
                  int64_t n_pairs, const int32_t *pf, const int32_t *po, const double *H, const double *G,
                  double *v_mag, double *geom)
{
    int64_t *fb = malloc(sizeof(int64_t) * (size_t)(n_frames > 0 ? n_frames : 1));
    if (!fb) return ORC_EINVAL;
    for (int64_t f = 0; f < n_frames; f++) fb[f] = -1;
    for (int64_t b = 0; b < n_batch; b++)
        for (int64_t q = batch_off[b]; q < batch_off[b + 1]; q++) fb[frame_order[q]] = b;
    int rc = ORC_OK;
    for (int64_t i = 0; i < n_pairs; i++) {
        int64_t f = pf[i], j = po[i];
        if (f < 0 || f >= n_frames || j < 0 || j >= n_obj || fb[f] < 0) { rc = ORC_EINVAL; break; }
        int64_t b = fb[f];
        double d[3], tau, xe[6], S[3], Sd[3];
        int st = orc_lighttime(E, c_light, t_ref[b], x_epoch + 6 * (b * n_obj + j), frames_t[f],
                               frames_obs + 3 * f, d, &tau, xe);
        if (!st) st = orc_cheb(E, 0, frames_t[f] - tau, S, Sd);
        if (st) {
            v_mag[i] = NAN;
            if (geom) geom[3 * i] = geom[3 * i + 1] = geom[3 * i + 2] = NAN;
            continue;
        }
        double r[3] = { xe[0] - S[0], xe[1] - S[1], xe[2] - S[2] };
        double rh = sqrt(dot3(r, r)), dl = sqrt(dot3(d, d));
        double c = dot3(r, d) / (rh * dl);
        double alpha = acos(c > 1.0 ? 1.0 : (c < -1.0 ? -1.0 : c));
        v_mag[i] = orc_hg_mag(H[j], G[j], rh, dl, alpha);
        if (geom) { geom[3 * i] = rh; geom[3 * i + 1] = dl; geom[3 * i + 2] = alpha; }
    }
    free(fb);
    return rc;
}

/* State and 6x6 state transition matrix Phi[i][c] = d state_i(t1) / d state_c(t0)
 * of one object, from the variational equations integrated alongside. */
int orc_stm(const orc_ephem *E, const orc_opts *o, const double x0[6], double t0, double t1,
            double out[6], double phi[36])
{
    orc_nbody_ctx ctx = { E, orc_c(o), 1 };
    orc_radau R; memset(&R, 0, sizeof(R));
    R.D = 21; R.D_ctrl = 3; R.force = orc_nbody_force; R.ctx = &ctx;
    orc_opts_fill(o, &R);
    double x[ORC_MAXD] = {0}, v[ORC_MAXD] = {0};
    for (int i = 0; i < 3; i++) { x[i] = x0[i]; v[i] = x0[3 + i]; }
    for (int c = 0; c < 6; c++) { if (c < 3) x[3 + 3 * c + c] = 1.0; else v[3 + 3 * c + (c - 3)] = 1.0; }
    double t = t0, h = o->h_init > 0 ? o->h_init : 1.0;
    int st = orc_radau_advance(&R, &t, x, v, t1, &h);
    if (st) return st;
    for (int i = 0; i < 3; i++) { out[i] = x[i]; out[3 + i] = v[i]; }
    for (int c = 0; c < 6; c++)
        for (int i = 0; i < 3; i++) { phi[6 * i + c] = x[3 + 3 * c + i]; phi[6 * (3 + i) + c] = v[3 + 3 * c + i]; }
    return 0;
}
