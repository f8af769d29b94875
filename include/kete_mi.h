/*
 * kete_mi.h -- C ABI of the MI355X (gfx950) known-object prediction path.
 *
 * The path follows Sect. 2 of "Kete: Predicting Known Minor Bodies in
 * Images" (arXiv 2509.04666): frames are grouped into time batches; the
 * small bodies are integrated with the n-body force model (App. A, Eqs.
 * A.1, A.3 and A.4, perturbers read from Chebyshev segments as in Sect. 3.2) to
 * the mid time of every batch; inside a batch each body is moved by
 * two-body motion with a light-delay correction to every frame; a body is
 * in a frame when every inward great-circle normal of the frame has a
 * positive dot product with its direction (Sect. 3.1).
 *
 * Conventions for every entry point:
 *   - units: au, TDB days, au/day; frame: ecliptic J2000; origin: solar
 *     system barycentre; all floating point is IEEE binary64;
 *   - "device" pointers are HIP device memory owned by the caller; "host"
 *     pointers are ordinary CPU memory owned by the caller; the library
 *     never frees caller memory and keeps no pointer after returning;
 *   - scratch memory is the caller's `workspace` (device, 256-byte
 *     aligned) of at least the size returned by the matching
 *     *_workspace_size query; the library allocates no device memory;
 *   - work is enqueued on `stream` (a hipStream_t, NULL = default stream)
 *     and runs asynchronously unless a function says otherwise;
 *   - the return value is KETE_OK or a negative KETE_E* code; a text
 *     description of the last error on the calling thread is available
 *     from kete_last_error();
 *   - per-object numerical failures are reported in `status` (KETE_ST_*),
 *     never as a call error; failed objects get NaN states, are skipped
 *     by the field-of-view test and get a zero gradient.
 */
#ifndef KETE_MI_H
#define KETE_MI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- codes */
#define KETE_OK          0
#define KETE_EINVAL     (-1)   /* null pointer, bad size or unsorted epochs */
#define KETE_ERANGE     (-2)   /* a time outside the ephemeris coverage */
#define KETE_ECAPACITY  (-3)   /* output buffer too small; required size reported */
#define KETE_EDEVICE    (-4)   /* HIP runtime failure */
#define KETE_EWORKSPACE (-5)   /* workspace smaller than the query result */

#define KETE_ST_OK             0
#define KETE_ST_NONFINITE      1   /* state became NaN/Inf */
#define KETE_ST_STEP_UNDERFLOW 2   /* step below h_min (close encounter) */
#define KETE_ST_MAX_STEPS      3   /* more than max_steps steps */
#define KETE_ST_KEPLER_NOCONV  4   /* universal-variable solve did not converge */

#define KETE_MAX_BODIES  16        /* perturbers, body 0 = Sun */
#define KETE_MAX_J2      4         /* bodies with the App. A.3 oblateness term */
#define KETE_MAX_DEGREE  15        /* Chebyshev degree */
#define KETE_MAX_SUB     128       /* sub-frames per frame */
#define KETE_MAX_OBJ     (1 << 25) /* objects per call */

/* ---------------------------------------------------------------- types */

/* Perturber ephemeris as uniform Chebyshev segments (Sect. 3.2: planet
 * positions are read from precomputed kernels instead of integrated).
 * Segment k of body b covers [t_start + k seg_days, t_start + (k+1) seg_days]
 * and gives position_c(t) = sum_n coef[b][k][c][n] T_n(tau) with
 * tau = 2 (t - t_k)/seg_days - 1; velocities are the derivative series.
 * A time exactly on a joint uses the later segment; times outside
 * [t_start, t_start + n_seg seg_days] are KETE_ERANGE. */
typedef struct {
    int32_t n_body;          /* 1..KETE_MAX_BODIES, body 0 is the Sun */
    int32_t n_seg;           /* >= 1 */
    int32_t degree;          /* 0..KETE_MAX_DEGREE */
    int32_t reserved;
    double t_start;          /* TDB day */
    double seg_days;         /* > 0 */
    const double *coef;      /* device [n_body][n_seg][3][degree+1] */
    const double *gm;        /* host [n_body], au^3/day^2 (Eq. A.1 mu_m) */
    const uint32_t *flags;   /* host [n_body], bit0: add the Eq. A.3 term */
    const double *j2;        /* host [n_body][5] or NULL: {J2, radius rho_m (au),
                                pole (unit vector in the integration frame)}
                                of the App. A.3 Eq. A.4 term; J2 = 0 for none,
                                at most KETE_MAX_J2 bodies */
} kete_ephem_t;

/* Options.  kete_default_opts() fills every field; zero means "default"
 * for the optional ones. */
typedef struct {
    double eps;              /* step control: |b6|/|a| target (1e-9) */
    double h_init;           /* first trial step in days (1.0) */
    double h_min;            /* smallest step before KETE_ST_STEP_UNDERFLOW (1e-8) */
    double h_max;            /* largest step, 0 = unlimited */
    double c_light;          /* speed of light in au/day (173.144632674...) */
    double batch_span;       /* frame batch span in days (3.0, Sect. 2) */
    double cell_chord;       /* FoV sky-grid cell size (chord units; 0 = auto: 0.10) */
    double lt_tol;           /* light-time convergence: last update in days (1e-15) */
    int32_t max_steps;       /* per object per call (2,000,000) */
    int32_t max_iter;        /* corrector iterations per step (12) */
    int32_t n_buckets;       /* step-size buckets (octaves of the predicted step), 1 = none (16) */
    int32_t block;           /* integrator threads per block: 64/128/256, 0 = auto (0: 256 for the
                                grouped integrators reading epochs off the step polynomials,
                                else 128) */
    int32_t rebucket_epochs; /* epochs per integrator launch, 0 = all (0) */
    int32_t window_segs;     /* Chebyshev segments per staged window, 0 = auto (0: for the grouped
                                integrators reading epochs off the step polynomials the most, up
                                to 6, with which three blocks share a compute unit's LDS; for the
                                adjoint 3; else 2) */
    int32_t lt_iter;         /* light-time updates at most (10) */
    int32_t fov_block;       /* FoV threads per block: 64/128/256 (128) */
    int32_t adj_seg_steps;   /* adjoint: steps stored per checkpoint segment (32) */
    int32_t persist_waves;   /* batched runs: resident waves per compute unit (8) */
    int32_t lanes_per_body;  /* integrator lanes per object: 1, 7 (9 per wavefront) or 8 (7) */
    int32_t zero_start;      /* 1: every corrector starts from zero increments, as in App. A.6;
                                0: grouped integrators start from the previous step's
                                collocation polynomial extrapolated (0) */
    int32_t land_epochs;     /* 1: the integration lands on every output epoch (Sect. 2);
                                0: grouped integrators land only on the last epoch of each
                                launch and read the others off the collocation polynomial
                                of the step that spans them (0) */
    int32_t kepler_iter;     /* iterations of one universal-variable solve before the hop is
                                KETE_ST_KEPLER_NOCONV (60; 0 = default) */
} kete_opts_t;

/* Frames (Sect. 3.1): an instantaneous observation at time t from the
 * observer position obs, made of n_sub convex spherical quadrilaterals
 * given by their inward unit normals.  Within a quadrilateral normals 0
 * and 1 bound opposite edges, and so do normals 2 and 3 (every rectangle
 * or rotated rectangle has this form).  A direction d is inside
 * sub-frame s when n_{s,i} . d > 0 for all four i.  Each quadrilateral
 * must be smaller than a hemisphere. */
typedef struct {
    int64_t n_frames;
    int32_t n_sub;           /* 1..KETE_MAX_SUB */
    int32_t reserved;
    const double *t;         /* device [n_frames], exposure mid time */
    const double *obs;       /* device [n_frames][3], barycentric observer */
    const double *normals;   /* device [n_frames][n_sub][4][3] */
} kete_frames_t;

/* One job of a batched run: n_obj bodies (rows obj_off.. of the
 * concatenated state array) starting at the common epoch t0, integrated
 * through n_epoch epochs (entries epoch_off.. of the concatenated epoch
 * array, strictly monotone away from t0); their states at epoch e are
 * written to x_out[xout_off + (e n_obj + j) 6 ..] (doubles). */
typedef struct {
    int64_t obj_off;
    int64_t epoch_off;
    int64_t xout_off;
    int32_t n_obj;
    int32_t n_epoch;
    double t0;
} kete_job_t;

/* A batched run: jobs plus the frames each job checks.  Frames of all
 * jobs are concatenated; the batches of all jobs are listed in one array
 * (batch b belongs to job batch_job[b] and uses that job's epoch
 * batch_epoch[b], whose time is t_ref[b]); frame_order / batch_off index
 * the frames of each batch as in kete_fov_check.  The *_host arrays are
 * host copies used to plan; every other pointer is device memory. */
typedef struct {
    int32_t n_jobs;
    int32_t reserved;
    int64_t n_bodies;               /* rows of x0 */
    int64_t n_epochs;               /* entries of epochs */
    int64_t n_batch;
    const kete_job_t *jobs_host;    /* host [n_jobs] */
    const kete_job_t *jobs;         /* device [n_jobs] */
    const double *x0;               /* device [n_bodies][6] */
    const double *epochs;           /* device [n_epochs] */
    const double *epochs_host;      /* host [n_epochs] or NULL (orders the tile queue) */
    const int32_t *batch_job_host;  /* host [n_batch] */
    const int32_t *batch_epoch_host;/* host [n_batch] */
    const int32_t *batch_off_host;  /* host [n_batch + 1] */
    const double *t_ref;            /* device [n_batch] */
    const int32_t *batch_off;       /* device [n_batch + 1] */
    const int32_t *frame_order;     /* device [n_frames] */
    kete_frames_t frames;           /* device */
} kete_batch_t;

/* ---------------------------------------------------------------- calls */

void kete_default_opts(kete_opts_t *opts);

/* Text of the last error raised on the calling thread ("" if none). */
const char *kete_last_error(void);

/* Library version string. */
const char *kete_version(void);

/* Frame batching (Sect. 2: batches of frames span at most batch_span
 * days; each batch is integrated to its mid time).  Host-only.  Sorts
 * frames by (t, index); a batch starts at its first frame and contains
 * every following frame within `span` days of that first frame; the batch
 * epoch is (t_first + t_last)/2.
 *   t           host [n_frames]
 *   frame_order host out [n_frames]: frame indices in batch order
 *   batch_off   host out [n_frames + 1]: batch b is frame_order[off[b]..off[b+1])
 *   t_ref       host out [n_frames]: batch epochs (first *n_batch used)
 *   n_batch     host out
 * Returns KETE_EINVAL for n_frames < 0, null pointers or non-finite t. */
int kete_make_batches(const double *t, int64_t n_frames, double span,
                      int32_t *frame_order, int32_t *batch_off, double *t_ref,
                      int64_t *n_batch);

/* Bytes of workspace needed by kete_propagate_nbody. */
size_t kete_propagate_workspace_size(int64_t n_obj, int64_t n_out, const kete_opts_t *opts);

/* n-body propagation of massless bodies (Sect. 2, App. A): every object
 * starts at the common epoch t0 and is integrated through the epochs
 * t_out[0..n_out) (strictly monotone, all after t0 or all before t0),
 * and its state at each epoch is written.  Force: Eq. A.1 (attractive)
 * plus Eq. A.3 for bodies with flags bit0 and Eq. A.4 (App. A.3) for
 * bodies given a J2.
 * Integrator: Gauss-Radau collocation with 8 nodes (the method of
 * App. A.6, predictor removed), IAS15 step control.  By default 7 lanes
 * share an object's force sums and the 9 objects of a wavefront share its
 * step size (objects are grouped by a predicted step size); states at
 * epochs inside a step are read off the step's collocation polynomial and
 * only the last epoch of a launch is landed on (opts lanes_per_body,
 * land_epochs).
 *   x0      device [n_obj][6]  (x, y, z, vx, vy, vz)
 *   t_out   host   [n_out]
 *   x_out   device [n_out][n_obj][6]
 *   status  device [n_obj]  (KETE_ST_*)
 *   stats   device [8] int64 or NULL: accumulated counters
 *           {wave steps, wave iterations, rejections, lane-steps,
 *            lane-iterations, Chebyshev chains with derivative, value-only
 *            chains, lane-steps started from an extrapolated corrector}
 * Errors: KETE_EINVAL, KETE_ERANGE (t0 or an epoch outside the ephemeris),
 * KETE_EWORKSPACE, KETE_EDEVICE. */
int kete_propagate_nbody(const kete_ephem_t *eph, const double *x0, double t0, int64_t n_obj,
                         const double *t_out, int64_t n_out, double *x_out, int32_t *status,
                         int64_t *stats, const kete_opts_t *opts,
                         void *workspace, size_t ws_bytes, void *stream);

/* Bytes of workspace needed by kete_fov_check. */
size_t kete_fov_workspace_size(int64_t n_obj, int64_t n_frames, int64_t n_batch, int32_t n_sub,
                               int64_t pairs_cap, const kete_opts_t *opts);

/* Field-of-view membership for a batched frame list (Sect. 2 and 3.1).
 * For batch b with epoch t_ref[b], each object j with status[j] == 0 is
 * moved from x_epoch[b][j] by heliocentric two-body motion (universal
 * variables, mu = gm[0]) to the emission time t_f - tau of every frame f of
 * the batch, tau being the Newtonian light time from the frame's observer
 * (iterated to lt_tol); (f, s, j) is a pair when all four normals of
 * sub-frame s have a positive dot product with the direction.  Objects
 * are binned on the sky so that only bodies that can reach a frame within
 * the batch are tested exactly.  An object one of whose hops ends on
 * the Kepler iteration cap (opts->kepler_iter) without converging loses all
 * of its pairs and gets KETE_ST_KEPLER_NOCONV in status (when given).
 *   x_epoch     device [n_batch][n_obj][6]
 *   status      device [n_obj] or NULL: in, objects to skip (non-zero);
 *               out, KETE_ST_KEPLER_NOCONV for objects whose hop failed
 *   t_ref       device [n_batch]
 *   batch_off   device [n_batch + 1]
 *   frame_order device [n_frames]
 *   pf, ps, po  device [pairs_cap]: frame, sub-frame, object of each pair,
 *               sorted by (frame, sub-frame, object)
 *   n_pairs     host out: number of pairs
 * The workspace holds up to max(65536, 16 n_frames, pairs_cap / 2)
 * exact-test candidates (the pairs that the linear-motion bound leaves
 * undecided).  Synchronizes `stream` once to read the counts.  Returns
 * KETE_ECAPACITY (outputs unspecified) when the pairs or the candidates
 * do not fit; *n_pairs then holds a pairs_cap to retry with, large
 * enough for both as far as they were counted. */
int kete_fov_check(const kete_ephem_t *eph, const double *x_epoch, int32_t *status,
                   int64_t n_obj, int64_t n_batch, const double *t_ref, const int32_t *batch_off,
                   const int32_t *frame_order, const kete_frames_t *frames, const kete_opts_t *opts,
                   int32_t *pf, int32_t *ps, int32_t *po, int64_t pairs_cap, int64_t *n_pairs,
                   void *workspace, size_t ws_bytes, void *stream);

/* Counters of the last kete_fov_check on the calling thread: out[0]
 * (object, frame) pairs that passed the cap test, out[1] exact light-time
 * tests, out[2] objects handled by the brute-force path, out[3] frame
 * records scanned by the per-cell join (per wavefront). */
void kete_fov_last_stats(int64_t out[4]);

/* The same counters followed by out[4] exact-test candidates listed,
 * out[5] (object, batch) items on the wide path, out[6] hops that ended on
 * the Kepler iteration cap, out[7] 0. */
void kete_fov_last_counts(int64_t out[8]);

/* Bytes of workspace needed by kete_pair_magnitudes (0 for a bad size):
 * a frame-to-batch map and one 192-byte record per frame. */
size_t kete_magnitudes_workspace_size(int64_t n_frames);

/* Apparent V magnitude of every (frame, object) pair in the H-G system
 * (Sect. 3.3, which takes the system of Bowell et al. 1989):
 *   V = H + 5 log10(r_H Delta) - 2.5 log10((1 - G) Phi_1 + G Phi_2),
 *   Phi_i = exp(-A_i tan(alpha/2)^B_i), A = (3.33, 1.87), B = (0.63, 1.22),
 * with r_H the body's distance from the Sun and Delta from the observer
 * at the light-time corrected emission time (the hop of kete_fov_check
 * from the state x_epoch[b][j] of the frame's batch b), and alpha the
 * phase angle at the body between the Sun and the observer.
 *   x_epoch, t_ref, batch_off, frame_order, frames: as for kete_fov_check
 *               (the normals are not read)
 *   pf, po      device [n_pairs]: frame and object of each pair, as
 *               kete_fov_check returns them (any order)
 *   h_mag       device [n_obj]: absolute magnitude H
 *   g_slope     device [n_obj]: slope parameter G
 *   v_mag       device out [n_pairs]
 *   geom        device out [n_pairs][3] {r_H au, Delta au, alpha rad}, or NULL
 * A pair whose frame is in no batch, whose indices are out of range,
 * whose emission time leaves the ephemeris or whose hop ends on the Kepler
 * iteration cap (opts->kepler_iter) without converging gets NaN.
 * Asynchronous on `stream`; the caller owns every buffer.
 * Errors: KETE_EINVAL, KETE_EWORKSPACE, KETE_EDEVICE. */
int kete_pair_magnitudes(const kete_ephem_t *eph, const double *x_epoch, int64_t n_obj, int64_t n_batch,
                         const double *t_ref, const int32_t *batch_off, const int32_t *frame_order,
                         const kete_frames_t *frames, const int32_t *pf, const int32_t *po, int64_t n_pairs,
                         const double *h_mag, const double *g_slope, double *v_mag, double *geom,
                         const kete_opts_t *opts, void *workspace, size_t ws_bytes, void *stream);

/* kete_pair_magnitudes for callers that cannot allocate device memory:
 * code recorded into a HIP graph, tight serving loops, harnesses that
 * forbid hipMalloc.  Same arguments, results and errors as
 * kete_pair_magnitudes, without the workspace: the frame-to-batch map
 * (4 bytes per frame) lives in a static device array of the library, of
 * KETE_MAG_NOALLOC_MAX_FRAMES frames (8 MiB), one copy per GPU, held until
 * the process ends.  Its device address is looked up on the first call on
 * each device (the current device must be the one `stream` belongs to).
 * The call allocates nothing and calls no allocating routine; the map is
 * refilled by a kernel on every call, so the last call's contents do not
 * leak into the next.  With no room for kete_pair_magnitudes' per-frame
 * records, each pair computes its frame's quantities itself: slower, with
 * the same results bit for bit.  Calls that overlap in time on one GPU (on
 * different streams or threads) share the array and race: serialize them.
 * Errors: KETE_EWORKSPACE when n_frames exceeds
 * KETE_MAG_NOALLOC_MAX_FRAMES, otherwise as kete_pair_magnitudes. */
#define KETE_MAG_NOALLOC_MAX_FRAMES (1 << 21)
int kete_pair_magnitudes_noalloc(const kete_ephem_t *eph, const double *x_epoch, int64_t n_obj, int64_t n_batch,
                                 const double *t_ref, const int32_t *batch_off, const int32_t *frame_order,
                                 const kete_frames_t *frames, const int32_t *pf, const int32_t *po, int64_t n_pairs,
                                 const double *h_mag, const double *g_slope, double *v_mag, double *geom,
                                 const kete_opts_t *opts, void *stream);

/* Light-time corrected directions (the per-pair step of kete_fov_check,
 * exposed for checking): for every object j and query q, the direction
 * d = x_e - obs[q] of object j (state x_ref[j] at t_ref) at the emission
 * time t_obs[q] - tau.
 *   x_ref  device [n_obj][6]; t_obs device [n_q]; obs device [n_q][3]
 *   d      device out [n_q][n_obj][3]; tau device out [n_q][n_obj] or NULL
 * A hop that ends on the Kepler iteration cap without converging gives NaN. */
int kete_lighttime_directions(const kete_ephem_t *eph, const double *x_ref, double t_ref, int64_t n_obj,
                              const double *t_obs, const double *obs, int64_t n_q,
                              double *d, double *tau, const kete_opts_t *opts, void *stream);

/* Chebyshev positions and velocities (the ephemeris evaluator on its
 * own, for checking): out[q][b][6] for every body b at times t[q].
 *   t device [n_q]; out device [n_q][n_body][6].
 * Returns KETE_ERANGE when a time is outside the coverage (checked on
 * the host copy t_host, which must hold the same values). */
int kete_ephem_eval(const kete_ephem_t *eph, const double *t, const double *t_host, int64_t n_q,
                    double *out, void *stream);

#define KETE_ADJ_FWD 0
#define KETE_ADJ_BWD 1

/* Bytes of workspace needed by kete_propagate_adjoint (the same
 * workspace must be passed to the forward and the backward call). */
size_t kete_adjoint_workspace_size(int64_t n_obj, int32_t k_obs, double t0, double t_end, double ckpt_days,
                                   const kete_opts_t *opts);

/* Sky positions of observations and their gradient with respect to the
 * initial states.  Each object j starts from x0[j] at t0 and is integrated
 * with the force model of kete_propagate_nbody; its observations k at
 * times t_obs[j][k] (ascending, in [t0, t_end]) from observers at
 * obs_pos[j][k] get the state at t_obs from the integrator's collocation
 * polynomial, the light-time hop of Sect. 2 back to the emission time,
 * and RA/Dec (radians) in the equatorial J2000 frame (ecliptic rotated by
 * the obliquity 84381.448").
 *   An observation whose hop ends on the Kepler iteration cap
 *   (opts->kepler_iter) gets a NaN sky position and its object
 *   KETE_ST_KEPLER_NOCONV (so a zero gradient).
 *   mode KETE_ADJ_FWD: writes sky_out [N][K][2] and status [N], and stores
 *     in the workspace a checkpoint per ckpt_days (checkpoint c: the state
 *     at the first integration step starting at or after t0 + c ckpt_days,
 *     so the steps are not cut at checkpoints) and each observation's
 *     light time;
 *   mode KETE_ADJ_BWD: given dL_dsky [N][K][2] (device) for the same
 *     inputs, options and workspace, writes grad_x0 [N][6] = dL/dx0: the
 *     discrete adjoint of the forward computation, recomputing each
 *     checkpoint segment (on a second, library-owned stream, ordered by
 *     events; the call's stream sees the whole result).  Objects with a
 *     non-zero status get a zero gradient.
 * All arrays are device memory; t0, t_end and ckpt_days are host values.
 * Errors: KETE_EINVAL, KETE_ERANGE, KETE_EWORKSPACE, KETE_EDEVICE. */
int kete_propagate_adjoint(const kete_ephem_t *eph, int32_t mode, const double *x0, double t0, double t_end,
                           int64_t n_obj, int32_t k_obs, const double *t_obs, const double *obs_pos,
                           const double *dL_dsky, double ckpt_days, double *sky_out, double *grad_x0,
                           int32_t *status, const kete_opts_t *opts, void *workspace, size_t ws_bytes,
                           void *stream);

/* Bytes of workspace for a batched run (plan, run and pairs share it). */
size_t kete_batch_workspace_size(const kete_ephem_t *eph, const kete_batch_t *batch, int64_t pairs_cap,
                                 const kete_opts_t *opts);

/* Batched uneven jobs (one persistent launch for the propagation of every
 * job, then the field-of-view stages of kete_fov_check over all batches).
 * kete_batch_plan validates the batch, builds the tile queue (tiles of 64
 * bodies, longest jobs first) and the batch tables, and uploads them into
 * the workspace; it synchronizes `stream`.  The workspace layout depends
 * on the batch, pairs_cap and opts, so every call of one run passes the
 * same three.  kete_batch_run enqueues the
 * whole computation without any host synchronization or memset, so it can
 * be captured in a HIP graph; x_out receives every job's epoch states and
 * status every body's status.  kete_batch_pairs then reads the pair count
 * (one synchronization) and writes the pairs sorted by (frame, sub-frame,
 * body), bodies numbered by their row in x0; KETE_ECAPACITY as in
 * kete_fov_check. */
int kete_batch_plan(const kete_ephem_t *eph, const kete_batch_t *batch, int64_t pairs_cap, const kete_opts_t *opts,
                    void *workspace, size_t ws_bytes, void *stream);
int kete_batch_run(const kete_ephem_t *eph, const kete_batch_t *batch, int64_t pairs_cap, const kete_opts_t *opts,
                   double *x_out, int32_t *status, void *workspace, size_t ws_bytes, void *stream);
int kete_batch_pairs(const kete_batch_t *batch, int64_t pairs_cap, const kete_opts_t *opts, int32_t *pf, int32_t *ps,
                     int32_t *po, int64_t *n_pairs, void *workspace, size_t ws_bytes, void *stream);

/* The same kete_batch_run captured once in a HIP graph and replayed.
 * kete_batch_graph_create records the run (after kete_batch_plan) and
 * returns an opaque handle; kete_batch_graph_launch replays it on
 * `stream`; kete_batch_graph_destroy releases it.  The graph keeps the
 * pointers it was recorded with: inputs, outputs and workspace must stay
 * allocated, and replays see their current contents. */
int kete_batch_graph_create(const kete_ephem_t *eph, const kete_batch_t *batch, int64_t pairs_cap,
                            const kete_opts_t *opts, double *x_out, int32_t *status, void *workspace, size_t ws_bytes,
                            void *stream, void **graph);
int kete_batch_graph_launch(void *graph, void *stream);
int kete_batch_graph_destroy(void *graph);

/* Autotuner for batched runs: coordinate descent, starting from `base`
 * (NULL = defaults), over n_buckets {1,4,8,16}, persist_waves {2,4,8,12},
 * window_segs {1,2,4}, fov_block {64,128,256} and cell_chord
 * {0.05,0.10,0.16}, in that order; each candidate is planned, run once to
 * warm up and timed with HIP events over `reps` (1..100) runs of
 * kete_batch_run on `stream`.  Candidates whose workspace exceeds
 * ws_bytes are skipped.  progress (may be NULL) is called with user after
 * every timed candidate.  Every candidate computes the same states and
 * pairs (they change launch shapes and groupings only).  On return *best
 * holds the fastest options, *best_ms (if not NULL) its time per run, and
 * the workspace is planned for *best.  Synchronizes `stream`; x_out and
 * status are overwritten. */
typedef void (*kete_tune_progress_fn)(const kete_opts_t *tried, double ms, void *user);
int kete_batch_autotune(const kete_ephem_t *eph, const kete_batch_t *batch, int64_t pairs_cap,
                        const kete_opts_t *base, int32_t reps, double *x_out, int32_t *status, void *workspace,
                        size_t ws_bytes, void *stream, kete_tune_progress_fn progress, void *user,
                        kete_opts_t *best, double *best_ms);

/* Live kernel timing for measurement.  While enabled, the library's
 * launches made by the calling thread are bracketed by HIP events on the
 * stream they are launched on, by kind k: 0 the integrator launch, 1 every
 * kernel of a field-of-view check (two brackets per call: preparation
 * through the exact test, and the pair sort), 2 the adjoint, 3 a batched
 * run's propagation, 4 the field-of-view join (candidate kernels) alone.
 * kete_timing_read_all waits for the events and returns the summed
 * milliseconds ms[k] and bracket counts count[k] (k < 8), then forgets
 * them; kete_timing_read returns kinds 0..3 only. */
void kete_timing_enable(int on);
int kete_timing_read(double ms[4], int64_t count[4]);
int kete_timing_read_all(double ms[8], int64_t count[8]);

#ifdef __cplusplus
}
#endif
#endif /* KETE_MI_H */
