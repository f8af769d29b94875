// C ABI of the gfx950 known-object prediction path: argument checks,
// workspace layout, launch planning.  Every numerical step runs in the
// HIP kernels of this library.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "kete_adjoint.hpp"
#include "kete_batch.hpp"
#include "kete_fov.hpp"
#include "kete_internal.hpp"
#include "kete_mag.hpp"
#include "kete_mi.h"

namespace kete {
hipError_t launch_hpref_init(const double* x0, double* h_pref, uint32_t* keys, int n, double mu, double dt_lo,
                             double dt_hi, int n_class, hipStream_t s);
hipError_t launch_body_sort(const uint32_t* keys, int n, int n_class, int32_t* perm, int32_t* tmp, int32_t* counts,
                            hipStream_t s);
hipError_t launch_iota(int32_t* perm, int n, hipStream_t s);
size_t bucket_scratch_ints(int64_t n_obj, int n_buckets);
}  // namespace kete

using namespace kete;

namespace {

thread_local std::string g_err;
thread_local unsigned long long g_fov_stats[8] = {0, 0, 0, 0, 0, 0, 0, 0};

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIPCHK(expr)                                                                      \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess) return fail(KETE_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

constexpr double kC = 299792.458 * 86400.0 / 149597870.7;

// Pinned staging of a host table copied to the device on the caller's
// stream, so that the call returns without waiting for the copy.  One
// buffer per thread: before it is refilled, the copy out of it made by
// the previous call is waited for (normally long finished).
struct HostStage {
    void* buf = nullptr;
    size_t cap = 0;
    hipEvent_t done = nullptr;
    bool pending = false;
};
thread_local HostStage g_stage;

int stage_to_device(void* dst, const void* src, size_t bytes, hipStream_t s) {
    HostStage& h = g_stage;
    if (h.pending) {
        HIPCHK(hipEventSynchronize(h.done));
        h.pending = false;
    }
    if (bytes > h.cap) {
        if (h.buf) HIPCHK(hipHostFree(h.buf));
        h.buf = nullptr;
        h.cap = 0;
        const size_t want = std::max(bytes, (size_t)1 << 20);
        HIPCHK(hipHostMalloc(&h.buf, want, hipHostMallocDefault));
        h.cap = want;
    }
    if (!h.done) HIPCHK(hipEventCreateWithFlags(&h.done, hipEventDisableTiming));
    std::memcpy(h.buf, src, bytes);
    HIPCHK(hipMemcpyAsync(dst, h.buf, bytes, hipMemcpyHostToDevice, s));
    HIPCHK(hipEventRecord(h.done, s));
    h.pending = true;
    return KETE_OK;
}

// ---------------------------------------------------------------- Radau
typedef long double ld;

ld legendre(int n, ld x, ld* dp) {
    ld p0 = 1, p1 = x, d0 = 0, d1 = 1;
    if (n == 0) { if (dp) *dp = 0; return 1; }
    for (int k = 1; k < n; ++k) {
        ld p2 = ((2 * k + 1) * x * p1 - k * p0) / (k + 1);
        ld d2 = d0 + (2 * k + 1) * p1;            // P'_{k+1} = P'_{k-1} + (2k+1) P_k
        p0 = p1; p1 = p2; d0 = d1; d1 = d2;
    }
    if (dp) *dp = d1;
    return p1;
}

RadauConst build_radau() {
    RadauConst rc;
    std::memset(&rc, 0, sizeof(rc));
    // interior nodes: roots of P7 + P8 other than -1, found by scan + Newton
    std::vector<ld> xr;
    const int NS = 4096;
    auto f = [](ld x, ld* d) { ld d7, d8; ld v = legendre(7, x, &d7) + legendre(8, x, &d8); *d = d7 + d8; return v; };
    ld xa = -1.0L + 1e-6L, dd;
    ld fa = f(xa, &dd);
    for (int i = 1; i <= NS; ++i) {
        ld xb = -1.0L + 1e-6L + (2.0L - 1e-6L) * i / NS;
        ld fb = f(xb, &dd);
        if ((fa < 0) != (fb < 0)) {
            ld lo = xa, hi = xb, x = 0.5L * (xa + xb);
            for (int it = 0; it < 100; ++it) {
                ld d;
                ld v = f(x, &d);
                if ((v < 0) == (fa < 0)) lo = x; else hi = x;
                ld xn = x - v / d;
                if (!(xn > lo && xn < hi)) xn = 0.5L * (lo + hi);
                if (std::fabs(xn - x) < 1e-19L) { x = xn; break; }
                x = xn;
            }
            xr.push_back(x);
        }
        xa = xb; fa = fb;
    }
    ld S[9];
    S[0] = 0;
    for (int i = 0; i < 7; ++i) S[i + 1] = 0.5L * (xr[i] + 1.0L);
    S[8] = 1;
    // 8-point Gauss-Legendre rule (exact to degree 15) on [-1, 1]
    ld gx[8], gw[8];
    for (int i = 0; i < 8; ++i) {
        ld x = std::cos(3.14159265358979323846264338327950L * (i + 0.75L) / 8.5L);
        for (int it = 0; it < 100; ++it) {
            ld d;
            ld v = legendre(8, x, &d);
            ld dx = v / d;
            x -= dx;
            if (std::fabs(dx) < 1e-20L) break;
        }
        ld d;
        legendre(8, x, &d);
        gx[i] = x;
        gw[i] = 2.0L / ((1 - x * x) * d * d);
    }
    auto ell = [&](int m, ld s) {             // Lagrange basis on S[0..7]
        ld v = 1;
        for (int k = 0; k < 8; ++k) if (k != m) v *= (s - S[k]) / (S[m] - S[k]);
        return v;
    };
    for (int n = 0; n < 9; ++n) {
        const ld s = S[n];
        rc.s[n] = (double)s;
        rc.half_s2[n] = (double)(0.5L * s * s);
        for (int m = 1; m < 8; ++m) {
            ld a = 0, b = 0;
            for (int q = 0; q < 8; ++q) {
                ld sig = 0.5L * s * (gx[q] + 1);
                ld w = 0.5L * s * gw[q];
                ld l = ell(m, sig);
                a += w * (s - sig) * l;
                b += w * l;
            }
            rc.A[n][m - 1] = (double)a;
            rc.B[n][m - 1] = (double)b;
        }
    }
    for (int m = 1; m < 8; ++m) {
        ld den = 1;
        for (int k = 0; k < 8; ++k) if (k != m) den *= S[m] - S[k];
        rc.Lden[m - 1] = (double)(1 / den);
        rc.L1[m - 1] = (double)ell(m, 1);
    }
    for (int m = 1; m < 8; ++m) {
        ld p = 1;
        for (int k = 0; k < 8; ++k) if (k != m) p *= (S[m] - S[k]);
        rc.E6[m - 1] = (double)(1.0L / p);
        // monomial coefficients of the Lagrange basis polynomial ell_m
        ld poly[8] = {1, 0, 0, 0, 0, 0, 0, 0};
        int deg = 0;
        for (int k = 0; k < 8; ++k) {
            if (k == m) continue;
            ld nxt[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            for (int q = 0; q <= deg; ++q) {
                nxt[q + 1] += poly[q];
                nxt[q] -= S[k] * poly[q];
            }
            ++deg;
            for (int q = 0; q < 8; ++q) poly[q] = nxt[q];
        }
        for (int q = 0; q < 8; ++q) {
            const ld pk = poly[q] / p;
            rc.Bp[m - 1][q] = (double)(pk / (q + 1));
            rc.Ap[m - 1][q] = (double)(pk / ((q + 1) * (q + 2)));
        }
    }
    return rc;
}

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

struct Carver {
    char* base;
    size_t off = 0;
    template <class T>
    T* take(size_t count) {
        T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
        off += align_up(count * sizeof(T));
        return p;
    }
};

int ephem_args(const kete_ephem_t* eph, double c_light, EphemArgs& E) {
    if (!eph || !eph->coef || !eph->gm || !eph->flags) return fail(KETE_EINVAL, "ephemeris pointers must be non-null");
    if (eph->n_body < 1 || eph->n_body > KETE_MAX_BODIES) return fail(KETE_EINVAL, "n_body %d outside 1..%d", eph->n_body, KETE_MAX_BODIES);
    if (eph->n_seg < 1) return fail(KETE_EINVAL, "n_seg must be >= 1");
    if (eph->degree < 0 || eph->degree > KETE_MAX_DEGREE) return fail(KETE_EINVAL, "degree %d outside 0..%d", eph->degree, KETE_MAX_DEGREE);
    if (!(eph->seg_days > 0) || !std::isfinite(eph->t_start)) return fail(KETE_EINVAL, "bad segment timing");
    std::memset(&E, 0, sizeof(E));
    E.coef = eph->coef;
    E.n_body = eph->n_body;
    E.n_seg = eph->n_seg;
    E.deg1 = eph->degree + 1;
    E.t_start = eph->t_start;
    E.seg_days = eph->seg_days;
    E.inv_seg = 1.0 / eph->seg_days;
    const double c2 = c_light * c_light;
    for (int b = 0; b < eph->n_body; ++b) {
        if (!(eph->gm[b] >= 0) || !std::isfinite(eph->gm[b])) return fail(KETE_EINVAL, "gm[%d] invalid", b);
        E.gm[b] = eph->gm[b];
        E.kgr[b] = (eph->flags[b] & 1u) ? eph->gm[b] / c2 : 0.0;
        if (E.kgr[b] != 0.0) E.has_gr = 1;
    }
    if (!(eph->gm[0] > 0)) return fail(KETE_EINVAL, "gm[0] (Sun) must be positive");
    int slot = 0;
    for (int pass = 0; pass < 2; ++pass)
        for (int b = 0; b < eph->n_body; ++b)
            if ((E.kgr[b] != 0.0) == (pass == 0)) {
                E.slot_of |= (unsigned long long)slot << (4 * b);
                E.body_at |= (unsigned long long)b << (4 * slot);
                ++slot;
                if (pass == 0) ++E.n_gr;
            }
    if (eph->j2) {
        for (int b = 0; b < eph->n_body; ++b) {
            const double* q = eph->j2 + 5 * b;
            if (q[0] == 0.0) continue;
            const double pn = std::sqrt(q[2] * q[2] + q[3] * q[3] + q[4] * q[4]);
            if (!std::isfinite(q[0]) || !(q[1] > 0) || !std::isfinite(q[1]) || !(std::fabs(pn - 1.0) < 1e-6))
                return fail(KETE_EINVAL, "j2[%d]: need finite J2, radius > 0 and a unit pole", b);
            if (E.n_j2 >= KETE_MAX_J2) return fail(KETE_EINVAL, "more than %d bodies with J2", KETE_MAX_J2);
            const int i = E.n_j2++;
            E.j2_body[i] = b;
            E.j2_slot[i] = body_slot(E, b);
            E.j2k[i] = 1.5 * q[0] * eph->gm[b] * q[1] * q[1];
            for (int c = 0; c < 3; ++c) E.j2p[i][c] = q[2 + c] / pn;
        }
    }
    return KETE_OK;
}

double t_end_of(const kete_ephem_t* e) { return e->t_start + e->n_seg * e->seg_days; }

int seg_of(const kete_ephem_t* e, double t) {
    return seg_clamped(t, e->t_start, 1.0 / e->seg_days, e->n_seg);
}

// Windows between t0 and each epoch: every epoch ends a window, and a
// window never spans more than `wsegs` segment lengths (next_window).
std::vector<Window> plan_windows(const kete_ephem_t* e, double t0, const double* t_out, int64_t n_out, int wsegs,
                                 std::vector<int>& epoch_end_win) {
    std::vector<Window> w;
    epoch_end_win.assign(n_out, -1);
    const double inv = 1.0 / e->seg_days;
    double t = t0;
    for (int64_t k = 0; k < n_out; ++k) {
        const double target = t_out[k];
        while (t != target) {
            Window W = next_window(t, target, e->t_start, e->seg_days, inv, e->n_seg, wsegs);
            W.out = (W.t_b == target) ? (int32_t)k : -1;
            w.push_back(W);
            t = W.t_b;
        }
        if (w.empty() || w.back().out != (int32_t)k) {
            // epoch equal to the current time: an empty window that only writes output
            Window W{t, t, seg_of(e, t), seg_of(e, t), (int32_t)k, 0};
            w.push_back(W);
        }
        epoch_end_win[k] = (int)w.size() - 1;
    }
    return w;
}

}  // namespace

namespace {
struct TimedRec { int kind; hipEvent_t a, b; };
thread_local bool g_timing = false;
thread_local std::vector<TimedRec> g_timed;
thread_local std::vector<hipEvent_t> g_event_pool;

hipEvent_t pool_event() {
    if (!g_event_pool.empty()) { hipEvent_t e = g_event_pool.back(); g_event_pool.pop_back(); return e; }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}
}  // namespace

namespace kete {
TimedScope::TimedScope(int k, hipStream_t s) : kind(k), stream(s), stop(nullptr) {
    if (!g_timing) return;
    hipEvent_t a = pool_event(), b = pool_event();
    if (!a || !b) return;
    hipEventRecord(a, s);
    g_timed.push_back({k, a, b});
    stop = b;
}
TimedScope::~TimedScope() {
    if (stop) hipEventRecord((hipEvent_t)stop, stream);
}

const RadauConst& radau_const() {
    static RadauConst rc = build_radau();
    return rc;
}
}  // namespace kete

extern "C" {

const char* kete_last_error(void) { return g_err.c_str(); }

const char* kete_version(void) { return "kete-mi355x 0.1.0 (gfx950)"; }

void kete_default_opts(kete_opts_t* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->eps = 1e-9;
    o->h_init = 1.0;
    o->h_min = 1e-8;
    o->h_max = 0.0;
    o->c_light = kC;
    o->batch_span = 3.0;
    o->cell_chord = 0.0;
    o->lt_tol = 1e-15;
    o->max_steps = 2000000;
    o->max_iter = 12;
    o->n_buckets = 16;
    o->block = 0;
    o->rebucket_epochs = 0;
    o->window_segs = 0;
    o->persist_waves = 8;
    o->lanes_per_body = 7;
    o->lt_iter = 10;
    o->fov_block = 128;
    o->adj_seg_steps = 32;
    o->kepler_iter = kKeplerIterDefault;
}

int kete_make_batches(const double* t, int64_t n_frames, double span, int32_t* frame_order, int32_t* batch_off,
                      double* t_ref, int64_t* n_batch) {
    if (n_frames < 0 || n_frames > INT32_MAX) return fail(KETE_EINVAL, "n_frames out of range");
    if (!n_batch || !batch_off || (n_frames > 0 && (!t || !frame_order || !t_ref)))
        return fail(KETE_EINVAL, "null pointer");
    if (!(span >= 0) || !std::isfinite(span)) return fail(KETE_EINVAL, "span must be finite and >= 0");
    for (int64_t i = 0; i < n_frames; ++i)
        if (!std::isfinite(t[i])) return fail(KETE_EINVAL, "t[%lld] is not finite", (long long)i);
    std::vector<int32_t> idx(n_frames);
    std::iota(idx.begin(), idx.end(), 0);
    if (!std::is_sorted(t, t + n_frames)) {
        // order by (t, index): a stable LSD radix sort, 8 bits per pass, of
        // the times' bit patterns mapped to unsigned integers in the order
        // of the values (sign bit flipped for t >= 0, all bits for t < 0;
        // -0 and +0 map to neighbours, which keeps them in index order as
        // equal times are)
        std::vector<uint64_t> key(n_frames), key2(n_frames);
        std::vector<int32_t> idx2(n_frames);
        for (int64_t i = 0; i < n_frames; ++i) {
            uint64_t u;
            const double v = t[i] == 0.0 ? 0.0 : t[i];
            std::memcpy(&u, &v, sizeof(u));
            key[i] = (u >> 63) ? ~u : (u | (1ull << 63));
        }
        std::vector<int64_t> cnt(256);
        for (int pass = 0; pass < 8; ++pass) {
            const int sh = 8 * pass;
            std::fill(cnt.begin(), cnt.end(), 0);
            for (int64_t i = 0; i < n_frames; ++i) ++cnt[(key[i] >> sh) & 0xff];
            if (cnt[key[0] >> sh & 0xff] == n_frames) continue;     // one digit value: nothing moves
            int64_t run = 0;
            for (auto& c : cnt) { const int64_t k = c; c = run; run += k; }
            for (int64_t i = 0; i < n_frames; ++i) {
                const int64_t pos = cnt[(key[i] >> sh) & 0xff]++;
                key2[pos] = key[i];
                idx2[pos] = idx[i];
            }
            key.swap(key2);
            idx.swap(idx2);
        }
    }
    int64_t nb = 0;
    batch_off[0] = 0;
    int64_t i = 0;
    while (i < n_frames) {
        const double first = t[idx[i]];
        int64_t j = i;
        while (j + 1 < n_frames && t[idx[j + 1]] - first <= span) ++j;
        t_ref[nb] = 0.5 * (first + t[idx[j]]);
        batch_off[++nb] = (int32_t)(j + 1);
        i = j + 1;
    }
    std::copy(idx.begin(), idx.end(), frame_order);
    *n_batch = nb;
    return KETE_OK;
}

// window_segs, with 0 (auto) taken as dflt.
static int segs_or(const kete_opts_t* o, int dflt) { return o->window_segs > 0 ? o->window_segs : dflt; }

// Launch shape of the integrator where block or window_segs is 0 (auto).
// With epochs read off the step polynomials, steps run until a window ends,
// so windows are long: the longest (up to 6 segments) with which three
// blocks of 256 threads share a compute unit's 160 KB of LDS, else smaller
// blocks.  With landing on every epoch: 128 threads, 2 segments.
static void auto_integrator_shape(const kete_ephem_t* eph, bool dense, int& block, int& wsegs) {
    constexpr size_t kBlockLds = 53248;
    if (!dense) {
        if (block == 0) block = 128;
        if (wsegs <= 0) wsegs = 2;
        return;
    }
    for (int b : {256, 128, 64}) {
        if (block != 0 && b != block) continue;
        if (wsegs > 0) { block = b; return; }
        for (int w = 6; w >= 1; --w)
            if (nbody_g8_lds_bytes(eph->n_body, eph->degree + 1, w + 1, b) <= kBlockLds) {
                block = b;
                wsegs = w;
                return;
            }
    }
    if (block == 0) block = 64;
    if (wsegs <= 0) wsegs = 1;
}

// The output epochs and the dense-output rows travel in front of the window
// plan (one staged copy).
// Step-size buckets of the batched jobs' sort: kBucketSub per octave over
// opts->n_buckets octaves (1 octave: no sort).
static int bucket_count(const kete_opts_t* o) {
    const int oct = std::min(std::max(1, o->n_buckets), 32);
    return oct > 1 ? oct * kBucketSub : 1;
}

// Step classes of the body sort (the critical class and kClassSub per
// octave over opts->n_buckets octaves; 1: no sort).
static int sort_classes(const kete_opts_t* o) {
    const int oct = std::min(std::max(1, o->n_buckets), 32);
    return oct > 1 ? 1 + kClassSub * oct : 1;
}

// Scratch of the body sort: counting-sort counts, then the keys and the
// first pass's order (ints).
static size_t sort_scratch_ints(int64_t n_obj) {
    return bucket_scratch_ints(n_obj, kMaxBuckets) + 2 * (size_t)n_obj + 64;
}
struct SortScratch {
    int32_t* counts;
    uint32_t* keys;
    int32_t* tmp;
};
static SortScratch sort_scratch(int32_t* base, int64_t n_obj) {
    SortScratch S;
    S.counts = base;
    S.keys = reinterpret_cast<uint32_t*>(base + bucket_scratch_ints(n_obj, kMaxBuckets));
    S.tmp = reinterpret_cast<int32_t*>(S.keys + n_obj);
    return S;
}

static size_t epoch_table_bytes(int64_t n_out) {
    return ((((size_t)n_out + kDenseCoefDoubles) * sizeof(double)) + 31) & ~(size_t)31;
}

size_t kete_propagate_workspace_size(int64_t n_obj, int64_t n_out, const kete_opts_t* opts) {
    kete_opts_t d;
    if (!opts) { kete_default_opts(&d); opts = &d; }
    const int wsegs = std::max(1, opts->window_segs);
    // windows: epochs plus at most one extra per wsegs segments of span;
    // the span is unknown here, so reserve generously and check at call time
    const int64_t max_win = 4 * (n_out + 1) + 65536;
    (void)wsegs;
    Carver c{nullptr};
    c.take<double>((size_t)n_obj * 6);
    c.take<double>((size_t)n_obj);
    c.take<int32_t>((size_t)n_obj);
    c.take<char>(epoch_table_bytes(n_out) + (size_t)max_win * sizeof(Window));
    c.take<int32_t>(sort_scratch_ints(n_obj));
    return c.off;
}

int kete_propagate_nbody(const kete_ephem_t* eph, const double* x0, double t0, int64_t n_obj, const double* t_out,
                         int64_t n_out, double* x_out, int32_t* status, int64_t* stats, const kete_opts_t* opts,
                         void* workspace, size_t ws_bytes, void* stream) {
    kete_opts_t d;
    if (!opts) { kete_default_opts(&d); opts = &d; }
    g_err.clear();
    EphemArgs E;
    int rc = ephem_args(eph, opts->c_light > 0 ? opts->c_light : kC, E);
    if (rc) return rc;
    if (n_obj < 0 || n_obj > KETE_MAX_OBJ) return fail(KETE_EINVAL, "n_obj %lld outside 0..%d", (long long)n_obj, KETE_MAX_OBJ);
    if (n_out < 0) return fail(KETE_EINVAL, "n_out < 0");
    if (n_obj == 0 || n_out == 0) return KETE_OK;
    if (!x0 || !t_out || !x_out || !status) return fail(KETE_EINVAL, "null pointer");
    if (!std::isfinite(t0)) return fail(KETE_EINVAL, "t0 not finite");
    const double tlo = eph->t_start, thi = t_end_of(eph);
    if (!(t0 >= tlo && t0 <= thi)) return fail(KETE_ERANGE, "t0 %.9g outside ephemeris [%.9g, %.9g]", t0, tlo, thi);
    // direction from the first epoch after the start (the first may equal t0)
    const bool fwd = (n_out > 1 && t_out[0] == t0) ? t_out[1] > t0 : t_out[0] > t0;
    double prev = t0;
    for (int64_t k = 0; k < n_out; ++k) {
        if (!std::isfinite(t_out[k])) return fail(KETE_EINVAL, "t_out[%lld] not finite", (long long)k);
        if (!(t_out[k] >= tlo && t_out[k] <= thi))
            return fail(KETE_ERANGE, "t_out[%lld] = %.9g outside ephemeris [%.9g, %.9g]", (long long)k, t_out[k], tlo, thi);
        if (k > 0 && (fwd ? !(t_out[k] > prev) : !(t_out[k] < prev)))
            return fail(KETE_EINVAL, "t_out must be strictly monotone and on one side of t0");
        prev = t_out[k];
    }
    if (opts->block != 0 && opts->block != 64 && opts->block != 128 && opts->block != 256)
        return fail(KETE_EINVAL, "block must be 0 (auto), 64, 128 or 256");
    if (opts->lanes_per_body != 1 && opts->lanes_per_body != 7 && opts->lanes_per_body != 8)
        return fail(KETE_EINVAL, "lanes_per_body must be 1, 7 or 8");
    if (!(opts->eps > 0) || !(opts->h_init > 0) || !(opts->h_min > 0) || opts->max_iter < 1 || opts->max_steps < 1)
        return fail(KETE_EINVAL, "eps, h_init, h_min, max_iter and max_steps must be positive");
    const int ncls = sort_classes(opts);
    const bool dense = !opts->land_epochs && opts->lanes_per_body != 1;
    int block = opts->block, wsegs = opts->window_segs;
    auto_integrator_shape(eph, dense, block, wsegs);

    // Launches cover runs of rebucket_epochs epochs.  With landing on every
    // epoch each epoch ends a window; otherwise only a launch's last epoch
    // does and the kernel reads the others off the step polynomials.
    const int64_t R = opts->rebucket_epochs > 0 ? opts->rebucket_epochs : n_out;
    std::vector<int> epoch_win;
    std::vector<Window> win;
    if (!dense) {
        win = plan_windows(eph, t0, t_out, n_out, wsegs, epoch_win);
    } else {
        epoch_win.assign(n_out, -1);
        const double inv = 1.0 / eph->seg_days;
        double t = t0;
        for (int64_t e0 = 0; e0 < n_out; e0 += R) {
            const int64_t e1 = std::min(n_out, e0 + R) - 1;
            const double target = t_out[e1];
            if (t == target) {
                Window W{t, t, seg_of(eph, t), seg_of(eph, t), (int32_t)e1, 0};
                win.push_back(W);
            }
            while (t != target) {
                Window W = next_window(t, target, eph->t_start, eph->seg_days, inv, eph->n_seg, wsegs);
                W.out = (W.t_b == target) ? (int32_t)e1 : -1;
                win.push_back(W);
                t = W.t_b;
            }
            epoch_win[e1] = (int)win.size() - 1;
        }
    }
    const int64_t max_win = 4 * (n_out + 1) + 65536;
    if ((int64_t)win.size() > max_win) return fail(KETE_EINVAL, "too many integration windows (%zu)", win.size());

    if (!workspace) return fail(KETE_EWORKSPACE, "workspace is null");
    const size_t need = kete_propagate_workspace_size(n_obj, n_out, opts);
    if (ws_bytes < need) return fail(KETE_EWORKSPACE, "workspace %zu bytes < %zu required", ws_bytes, need);
    Carver c{(char*)workspace};
    double* state = c.take<double>((size_t)n_obj * 6);
    double* h_pref = c.take<double>((size_t)n_obj);
    int32_t* perm = c.take<int32_t>((size_t)n_obj);
    char* plan = c.take<char>(epoch_table_bytes(n_out) + (size_t)max_win * sizeof(Window));
    double* dcoef = (double*)plan;
    double* dt_out = dcoef + kDenseCoefDoubles;
    Window* dwin = (Window*)(plan + epoch_table_bytes(n_out));
    const SortScratch sorts = sort_scratch(c.take<int32_t>(sort_scratch_ints(n_obj)), n_obj);

    hipStream_t s = (hipStream_t)stream;
    {
        std::vector<char> host(epoch_table_bytes(n_out) + win.size() * sizeof(Window));
        const RadauConst& rcst = radau_const();
        std::memcpy(host.data(), &rcst.Ap[0][0], 56 * sizeof(double));
        std::memcpy(host.data() + 56 * sizeof(double), &rcst.Bp[0][0], 56 * sizeof(double));
        std::memcpy(host.data() + kDenseCoefDoubles * sizeof(double), t_out, (size_t)n_out * sizeof(double));
        std::memcpy(host.data() + epoch_table_bytes(n_out), win.data(), win.size() * sizeof(Window));
        if ((rc = stage_to_device(plan, host.data(), host.size(), s))) return rc;
    }
    HIPCHK(hipMemcpyAsync(state, x0, (size_t)n_obj * 6 * sizeof(double), hipMemcpyDeviceToDevice, s));
    HIPCHK(fill_zero(status, (size_t)n_obj * sizeof(int32_t), s));

    NbodyParams P;
    std::memset(&P, 0, sizeof(P));
    P.eph = E;
    P.rc = radau_const();
    P.state = state;
    P.h_pref = h_pref;
    P.status = status;
    P.x_out = x_out;
    P.t_out = dt_out;
    P.dense_coef = dcoef;
    P.stats = (unsigned long long*)stats;
    P.n_obj = (int32_t)n_obj;
    P.max_iter = opts->max_iter;
    P.max_steps = opts->max_steps;
    P.zero_start = opts->zero_start != 0;
    P.max_win_segs = wsegs + 1;
    P.eps = opts->eps;
    P.h_min = opts->h_min;
    P.h_max = opts->h_max;
    P.h_init = opts->h_init;
    P.safety = 0.25;

    int first = 0;
    for (int64_t e0 = 0; e0 < n_out; e0 += R) {
        const int64_t e1 = std::min(n_out, e0 + R) - 1;
        const int last = epoch_win[e1];
        P.e_first = dense ? (int32_t)e0 : (int32_t)e1;
        P.e_land = (int32_t)e1;
        // predicted steps and the body order over this launch's span, from
        // the bodies' states at its start
        const double ta = e0 == 0 ? t0 : t_out[e0 - 1];
        double dt_lo = 0.0, dt_hi = 0.0;
        for (int64_t k = e0; k <= e1; ++k) {
            dt_lo = std::min(dt_lo, t_out[k] - ta);
            dt_hi = std::max(dt_hi, t_out[k] - ta);
        }
        HIPCHK(launch_hpref_init(state, h_pref, ncls > 1 ? sorts.keys : nullptr, (int)n_obj, E.gm[0], dt_lo, dt_hi,
                                 ncls, s));
        if (ncls > 1) {
            HIPCHK(launch_body_sort(sorts.keys, (int)n_obj, ncls, perm, sorts.tmp, sorts.counts, s));
            P.perm = perm;
        } else {
            P.perm = nullptr;
        }
        P.win = dwin + first;
        P.n_win = last - first + 1;
        P.first_launch = (e0 == 0);
        {
            TimedScope ts(kTimeNbody, s);
            HIPCHK(launch_nbody(P, block, opts->lanes_per_body, s));
        }
        first = last + 1;
    }
    return KETE_OK;
}

// Exact-test candidates kept between the join and the exact test (only the
// pairs the linear-motion bound leaves undecided).
static int64_t cand_capacity(int64_t n_frames, int64_t pairs_cap) {
    return std::max<int64_t>(1 << 16, std::max<int64_t>(16 * n_frames, pairs_cap / 2));
}

// Device counters of the FoV stages: [0] pairs, [1..4] statistics,
// [5] candidates, [6] wide objects, [8] failed hops, [9] pairs kept after
// dropping failed objects; from [16] the work-queue cursors of the per-cell
// join, then those of the wide join.
constexpr int kFovCursorBase = 16;
constexpr int kFovWideCursorBase = kFovCursorBase + kJoinCursorWords / 2;
constexpr int kFovCounters = kFovWideCursorBase + kJoinCursorWords / 2;

// Drops the pairs of objects whose hop failed (n_fail > 0): survivors of
// keys[0..np) go to `out`, and their count is read back (one more
// synchronization, taken only when a hop failed).
static int drop_failed_pairs(const unsigned long long* keys, int64_t np, const int32_t* fail_flags,
                             unsigned long long* out, unsigned long long* counters, int64_t* kept, hipStream_t s) {
    HIPCHK(fill_zero(counters + 9, sizeof(unsigned long long), s));
    HIPCHK(fov_drop_failed(keys, np, fail_flags, out, counters + 9, s));
    unsigned long long k = 0;
    HIPCHK(hipMemcpyAsync(&k, counters + 9, sizeof(k), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    *kept = (int64_t)k;
    return KETE_OK;
}

// pairs_cap to retry with after a capacity failure: room for the pairs
// found and, at cand_capacity's pairs_cap / 2, for every counted candidate.
static int64_t retry_pairs_cap(int64_t pairs, int64_t cands, int64_t pairs_cap) {
    return std::max<int64_t>(std::max<int64_t>(pairs, 2 * cands), pairs_cap + 1);
}

static int grid_dims(const kete_opts_t* o, int64_t n_batch, int& G, double& L) {
    L = o->cell_chord > 0 ? o->cell_chord : 0.10;
    G = (int)std::ceil(2.0 / L - 1e-9);
    if (G < 1) G = 1;
    if (G > 128) return fail(KETE_EINVAL, "cell_chord too small (grid > 128 cells per axis)");
    if ((double)n_batch * G * G * G > 2.0e9) return fail(KETE_EINVAL, "sky grid too large for %lld batches", (long long)n_batch);
    return KETE_OK;
}

size_t kete_fov_workspace_size(int64_t n_obj, int64_t n_frames, int64_t n_batch, int32_t n_sub, int64_t pairs_cap,
                               const kete_opts_t* opts) {
    kete_opts_t d;
    if (!opts) { kete_default_opts(&d); opts = &d; }
    int G; double L;
    if (grid_dims(opts, n_batch, G, L)) return 0;
    const int64_t nkeys = n_batch * ((int64_t)G * G * G + 1);
    Carver c{nullptr};
    c.take<double>((size_t)n_frames * 8);
    c.take<double>((size_t)n_batch * kBatchStride);
    c.take<int32_t>((size_t)n_frames);
    c.take<int32_t>((size_t)nkeys + 1);
    c.take<int32_t>((size_t)nkeys + 1);
    c.take<int32_t>((size_t)n_frames);
    c.take<double>((size_t)n_frames * 8);           // frame caps in cell order
    c.take<unsigned long long>((size_t)std::max<int64_t>(pairs_cap, 1));
    c.take<unsigned long long>(kFovCounters);
    c.take<int32_t>((size_t)n_frames + 1);
    c.take<int32_t>((size_t)n_frames + 1);
    c.take<unsigned long long>((size_t)std::max<int64_t>(pairs_cap, 1));
    c.take<char>(std::max(scan_scratch_bytes(nkeys), scan_scratch_bytes(n_frames)));
    c.take<unsigned long long>((size_t)cand_capacity(n_frames, pairs_cap));
    c.take<int32_t>((size_t)n_frames);
    c.take<int32_t>((size_t)(n_batch * n_obj));     // object cell keys
    c.take<int32_t>((size_t)(n_batch * n_obj));     // object ranks inside their cell
    c.take<int32_t>((size_t)(n_batch * n_obj));     // objects sorted by cell
    c.take<int32_t>((size_t)(n_batch * n_obj));     // object sub-cell keys
    c.take<int32_t>((size_t)nkeys + 1);             // object cell starts and counts
    c.take<int32_t>((size_t)nkeys + 1);
    c.take<unsigned long long>((size_t)(n_batch * n_obj));   // wide objects
    c.take<char>(scan_scratch_bytes(nkeys));
    c.take<int32_t>((size_t)nkeys + 1);             // join work items per key and their starts
    c.take<int32_t>((size_t)nkeys + 1);
    c.take<unsigned long long>((size_t)fov_item_capacity(nkeys, n_batch * n_obj));
    c.take<int64_t>((size_t)n_batch + 1);          // batch -> object layout
    c.take<int32_t>((size_t)n_batch);
    c.take<int64_t>((size_t)n_batch);
    c.take<int32_t>((size_t)n_batch);              // grid sizes and key offsets
    c.take<int64_t>((size_t)n_batch + 1);
    c.take<int32_t>((size_t)std::max<int64_t>(n_obj, 1));   // objects whose hop failed
    if (n_sub > 1) c.take<double>((size_t)n_frames * kLocStride);   // sub-frame locators
    c.take<double>((size_t)fov_cell_frame_doubles(n_frames, n_sub));  // frame data in cell order
    c.take<int32_t>((size_t)(n_batch * n_obj));     // parts of the wide objects and their scan
    c.take<int32_t>((size_t)(n_batch * n_obj) + 1);
    c.take<char>(scan_scratch_bytes(n_batch * n_obj));
    return c.off;
}

int kete_fov_check(const kete_ephem_t* eph, const double* x_epoch, int32_t* status, int64_t n_obj,
                   int64_t n_batch, const double* t_ref, const int32_t* batch_off, const int32_t* frame_order,
                   const kete_frames_t* frames, const kete_opts_t* opts, int32_t* pf, int32_t* ps, int32_t* po,
                   int64_t pairs_cap, int64_t* n_pairs, void* workspace, size_t ws_bytes, void* stream) {
    kete_opts_t d;
    if (!opts) { kete_default_opts(&d); opts = &d; }
    g_err.clear();
    EphemArgs E;
    const double cl = opts->c_light > 0 ? opts->c_light : kC;
    int rc = ephem_args(eph, cl, E);
    if (rc) return rc;
    if (!n_pairs) return fail(KETE_EINVAL, "n_pairs is null");
    *n_pairs = 0;
    if (!frames) return fail(KETE_EINVAL, "frames is null");
    if (n_obj < 0 || n_obj > KETE_MAX_OBJ) return fail(KETE_EINVAL, "n_obj %lld outside 0..%d", (long long)n_obj, KETE_MAX_OBJ);
    if (n_batch < 0 || frames->n_frames < 0 || frames->n_frames > INT32_MAX) return fail(KETE_EINVAL, "bad sizes");
    if ((double)n_batch * (double)n_obj >= 2.0e9) return fail(KETE_EINVAL, "n_batch x n_obj must stay below 2^31");
    if (frames->n_sub < 1 || frames->n_sub > KETE_MAX_SUB) return fail(KETE_EINVAL, "n_sub %d outside 1..%d", frames->n_sub, KETE_MAX_SUB);
    if (pairs_cap < 0) return fail(KETE_EINVAL, "pairs_cap < 0");
    if (n_obj == 0 || n_batch == 0 || frames->n_frames == 0) { std::memset(g_fov_stats, 0, sizeof(g_fov_stats)); return KETE_OK; }
    if (!x_epoch || !t_ref || !batch_off || !frame_order || !frames->t || !frames->obs || !frames->normals)
        return fail(KETE_EINVAL, "null pointer");
    if (pairs_cap > 0 && (!pf || !ps || !po)) return fail(KETE_EINVAL, "null output pointer");
    if (opts->fov_block != 64 && opts->fov_block != 128 && opts->fov_block != 256)
        return fail(KETE_EINVAL, "fov_block must be 64, 128 or 256");
    int G; double L;
    if ((rc = grid_dims(opts, n_batch, G, L))) return rc;
    const int64_t nkeys = n_batch * ((int64_t)G * G * G + 1);
    const int64_t F = frames->n_frames;
    if (!workspace) return fail(KETE_EWORKSPACE, "workspace is null");
    const size_t need = kete_fov_workspace_size(n_obj, F, n_batch, frames->n_sub, pairs_cap, opts);
    if (ws_bytes < need) return fail(KETE_EWORKSPACE, "workspace %zu bytes < %zu required", ws_bytes, need);

    Carver c{(char*)workspace};
    FovParams P;
    std::memset(&P, 0, sizeof(P));
    P.fcap = c.take<double>((size_t)F * 8);
    P.btab = c.take<double>((size_t)n_batch * kBatchStride);
    int32_t* qkey = c.take<int32_t>((size_t)F);
    int32_t* cnt = c.take<int32_t>((size_t)nkeys + 1);
    P.cell_start = c.take<int32_t>((size_t)nkeys + 1);
    P.cell_frames = c.take<int32_t>((size_t)F);
    P.cell_caps = c.take<double>((size_t)F * 8);
    P.pairs = c.take<unsigned long long>((size_t)std::max<int64_t>(pairs_cap, 1));
    unsigned long long* counters = c.take<unsigned long long>(kFovCounters);
    int32_t* fcnt = c.take<int32_t>((size_t)F + 1);
    int32_t* fstart = c.take<int32_t>((size_t)F + 1);
    unsigned long long* sorted = c.take<unsigned long long>((size_t)std::max<int64_t>(pairs_cap, 1));
    void* scan_scratch = c.take<char>(std::max(scan_scratch_bytes(nkeys), scan_scratch_bytes(F)));
    P.cand_cap = cand_capacity(F, pairs_cap);
    P.cand = c.take<unsigned long long>((size_t)P.cand_cap);
    P.frame_batch = c.take<int32_t>((size_t)F);
    int32_t* okey = c.take<int32_t>((size_t)(n_batch * n_obj));
    int32_t* orank = c.take<int32_t>((size_t)(n_batch * n_obj));
    int32_t* osorted = c.take<int32_t>((size_t)(n_batch * n_obj));
    int32_t* osub = c.take<int32_t>((size_t)(n_batch * n_obj));
    int32_t* ostart = c.take<int32_t>((size_t)nkeys + 1);
    int32_t* ocnt = c.take<int32_t>((size_t)nkeys + 1);
    P.wide = c.take<unsigned long long>((size_t)(n_batch * n_obj));
    void* oscan = c.take<char>(scan_scratch_bytes(nkeys));
    int32_t* icnt = c.take<int32_t>((size_t)nkeys + 1);
    int32_t* istart = c.take<int32_t>((size_t)nkeys + 1);
    unsigned long long* items = c.take<unsigned long long>((size_t)fov_item_capacity(nkeys, n_batch * n_obj));
    int64_t* b_poff = c.take<int64_t>((size_t)n_batch + 1);
    int32_t* b_obj0 = c.take<int32_t>((size_t)n_batch);
    int64_t* b_xoff = c.take<int64_t>((size_t)n_batch);
    int32_t* b_G = c.take<int32_t>((size_t)n_batch);
    int64_t* b_koff = c.take<int64_t>((size_t)n_batch + 1);
    P.fail = c.take<int32_t>((size_t)std::max<int64_t>(n_obj, 1));
    P.loc = frames->n_sub > 1 ? c.take<double>((size_t)F * kLocStride) : nullptr;
    P.cell_obs = c.take<double>((size_t)fov_cell_frame_doubles(F, frames->n_sub));
    P.cell_normals = reinterpret_cast<float*>(P.cell_obs + 4 * F);
    P.exact_rec = P.cell_obs + 4 * F + 6 * (int64_t)frames->n_sub * F;
    P.wide_parts = c.take<int32_t>((size_t)(n_batch * n_obj));
    P.wide_off = c.take<int32_t>((size_t)(n_batch * n_obj) + 1);
    void* wscan = c.take<char>(scan_scratch_bytes(n_batch * n_obj));
    P.wide_next = (unsigned int*)(counters + kFovWideCursorBase);
    P.status_out = status;
    P.n_fail = counters + 8;
    P.b_poff = b_poff;
    P.b_obj0 = b_obj0;
    P.b_xoff = b_xoff;
    P.b_G = b_G;
    P.b_koff = b_koff;
    P.n_keys = nkeys;
    P.n_pairs_total = n_batch * n_obj;
    P.max_batch_obj = n_obj;

    P.eph = E;
    P.x_epoch = x_epoch;
    P.status = status;
    P.n_obj = (int32_t)n_obj;
    P.n_batch = (int32_t)n_batch;
    P.n_frames = F;
    P.t_ref = t_ref;
    P.batch_off = batch_off;
    P.frame_order = frame_order;
    P.ft = frames->t;
    P.fobs = frames->obs;
    P.normals = frames->normals;
    P.n_sub = frames->n_sub;
    P.n_pairs = counters;
    P.stats = counters + 1;
    P.n_cand = counters + 5;
    P.cap = pairs_cap;
    P.mu = E.gm[0];
    P.smu = std::sqrt(E.gm[0]);
    P.c_light = cl;
    P.lt_tol = opts->lt_tol > 0 ? opts->lt_tol : 1e-15;
    P.lt_iter = opts->lt_iter > 0 ? opts->lt_iter : 10;
    if (opts->kepler_iter < 0) return fail(KETE_EINVAL, "kepler_iter must be >= 0");
    P.kepler_iter = opts->kepler_iter > 0 ? opts->kepler_iter : kKeplerIterDefault;
    P.max_cells = 1024;
    P.sin_overflow = 0.5;

    hipStream_t s = (hipStream_t)stream;
    {
        TimedScope ts(kTimeFov, s);
        HIPCHK(fill_zero(counters, kFovCounters * sizeof(unsigned long long), s));
        HIPCHK(fill_zero(P.fail, (size_t)n_obj * sizeof(int32_t), s));
        HIPCHK(fov_single_job_layout(b_poff, b_obj0, b_xoff, b_G, b_koff, n_batch, n_obj, G, s));
        HIPCHK(fov_prepare(P, qkey, cnt, cnt, scan_scratch, s));
        P.n_wide = counters + 6;
        HIPCHK(fov_sort_objects(P, okey, orank, ocnt, ostart, osorted, osub, oscan, s));
        P.obj_sorted = osorted;
        P.obj_start = ostart;
        P.obj_count = ocnt;
        {
            TimedScope tj(kTimeFovJoin, s);
            HIPCHK(fov_candidates(P, icnt, istart, items, (unsigned int*)(counters + kFovCursorBase), oscan, wscan, s));
        }
        HIPCHK(fov_exact(P, s));
    }
    unsigned long long host_counters[kFovCursorBase];
    HIPCHK(hipMemcpyAsync(host_counters, counters, sizeof(host_counters), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (int i = 0; i < 4; ++i) g_fov_stats[i] = host_counters[1 + i];
    g_fov_stats[4] = host_counters[5];
    g_fov_stats[5] = host_counters[6];
    g_fov_stats[6] = host_counters[8];
    int64_t np = (int64_t)host_counters[0];
    *n_pairs = np;
    if ((int64_t)host_counters[5] > P.cand_cap || np > pairs_cap) {
        *n_pairs = retry_pairs_cap(np, (int64_t)host_counters[5], pairs_cap);
        return fail(KETE_ECAPACITY, "%lld pairs / %llu exact-test candidates exceed pairs_cap %lld / %lld",
                    (long long)np, host_counters[5], (long long)pairs_cap, (long long)P.cand_cap);
    }
    TimedScope ts(kTimeFov, s);
    if (host_counters[8] > 0) {
        if ((rc = drop_failed_pairs(P.pairs, np, P.fail, sorted, counters, &np, s))) return rc;
        *n_pairs = np;
        HIPCHK(fov_sort(sorted, np, F, n_obj, frames->n_sub, fcnt, fstart, P.pairs, scan_scratch, pf, ps, po, s));
        return KETE_OK;
    }
    HIPCHK(fov_sort(P.pairs, np, F, n_obj, frames->n_sub, fcnt, fstart, sorted, scan_scratch, pf, ps, po, s));
    return KETE_OK;
}

// Checkpoint segments of the adjoint: C = ceil((t_end - t0) / ckpt_days).
// The kernels plan their own windows (aligned_window) and take checkpoint c
// at the first step start at or after t0 + c ckpt_days.
static int adjoint_plan(const kete_ephem_t* eph, double t0, double t_end, double ckpt_days, int64_t& C) {
    if (!std::isfinite(t0) || !std::isfinite(t_end) || !(t_end > t0))
        return fail(KETE_EINVAL, "need finite t0 < t_end");
    if (!(ckpt_days > 0) || !std::isfinite(ckpt_days)) return fail(KETE_EINVAL, "ckpt_days must be positive");
    const double tlo = eph->t_start, thi = t_end_of(eph);
    if (!(t0 >= tlo && t_end <= thi)) return fail(KETE_ERANGE, "[t0, t_end] outside the ephemeris");
    C = (int64_t)std::ceil((t_end - t0) / ckpt_days - 1e-12);
    if (C < 1 || C > 1000000) return fail(KETE_EINVAL, "bad checkpoint count");
    return KETE_OK;
}

static int adj_steps(const kete_opts_t* o) { return o->adj_seg_steps > 0 ? std::min(o->adj_seg_steps, 4096) : 32; }


size_t kete_adjoint_workspace_size(int64_t n_obj, int32_t k_obs, double t0, double t_end, double ckpt_days,
                                   const kete_opts_t* opts) {
    kete_opts_t d;
    if (!opts) { kete_default_opts(&d); opts = &d; }
    if (!(t_end > t0) || !(ckpt_days > 0) || n_obj < 0 || k_obs < 0) return 0;
    const int64_t C = (int64_t)std::ceil((t_end - t0) / ckpt_days - 1e-12);
    Carver c{nullptr};
    c.take<int32_t>((size_t)n_obj);                                   // perm
    c.take<double>((size_t)n_obj);                                    // h_pref
    c.take<double>((size_t)(C + 1) * n_obj * kCkptDoubles);
    c.take<double>((size_t)2 * adj_steps(opts) * kStepRecDoubles * n_obj);   // two step stores
    c.take<double>((size_t)n_obj * std::max(0, k_obs) * 6);    // observation states
    c.take<double>((size_t)n_obj * std::max(0, k_obs) * 6);    // observation cotangents
    c.take<double>((size_t)n_obj * std::max(0, k_obs) * 2);    // light times and anomalies
    c.take<int32_t>(sort_scratch_ints(n_obj));
    c.take<double>((size_t)n_obj * kAdjStateDoubles);                 // carried backward state
    c.take<int32_t>((size_t)2 * ((n_obj + kAdjLanes - 1) / kAdjLanes));     // steps per wavefront, per store
    c.take<double>((size_t)kAdjTabDoubles);                           // reverse-sweep constants
    c.take<double>((size_t)kDenseCoefDoubles);                        // dense-output rows
    return c.off;
}

int kete_propagate_adjoint(const kete_ephem_t* eph, int32_t mode, const double* x0, double t0, double t_end,
                           int64_t n_obj, int32_t k_obs, const double* t_obs, const double* obs_pos,
                           const double* dL_dsky, double ckpt_days, double* sky_out, double* grad_x0,
                           int32_t* status, const kete_opts_t* opts, void* workspace, size_t ws_bytes,
                           void* stream) {
    kete_opts_t dflt;
    if (!opts) { kete_default_opts(&dflt); opts = &dflt; }
    g_err.clear();
    EphemArgs E;
    const double cl = opts->c_light > 0 ? opts->c_light : kC;
    int rc = ephem_args(eph, cl, E);
    if (rc) return rc;
    if (mode != KETE_ADJ_FWD && mode != KETE_ADJ_BWD) return fail(KETE_EINVAL, "mode must be KETE_ADJ_FWD or KETE_ADJ_BWD");
    if (n_obj < 0 || n_obj > KETE_MAX_OBJ || k_obs < 0) return fail(KETE_EINVAL, "bad sizes");
    int64_t C = 0;
    if ((rc = adjoint_plan(eph, t0, t_end, ckpt_days, C))) return rc;
    if (n_obj == 0) return KETE_OK;
    if (!x0 || !status || (k_obs > 0 && (!t_obs || !obs_pos))) return fail(KETE_EINVAL, "null pointer");
    if (mode == KETE_ADJ_FWD && k_obs > 0 && !sky_out) return fail(KETE_EINVAL, "sky_out is null");
    if (mode == KETE_ADJ_BWD && (!grad_x0 || (k_obs > 0 && !dL_dsky))) return fail(KETE_EINVAL, "null gradient pointer");
    if (!(opts->eps > 0) || !(opts->h_init > 0) || !(opts->h_min > 0) || opts->max_iter < 1 || opts->max_steps < 1)
        return fail(KETE_EINVAL, "eps, h_init, h_min, max_iter and max_steps must be positive");
    const int ncls = sort_classes(opts);
    if (!workspace) return fail(KETE_EWORKSPACE, "workspace is null");
    const size_t need = kete_adjoint_workspace_size(n_obj, k_obs, t0, t_end, ckpt_days, opts);
    if (ws_bytes < need) return fail(KETE_EWORKSPACE, "workspace %zu bytes < %zu required", ws_bytes, need);
    Carver c{(char*)workspace};
    int32_t* perm = c.take<int32_t>((size_t)n_obj);
    double* h_pref = c.take<double>((size_t)n_obj);
    double* ckpt = c.take<double>((size_t)(C + 1) * n_obj * kCkptDoubles);
    double* scratch = c.take<double>((size_t)2 * adj_steps(opts) * kStepRecDoubles * n_obj);
    double* obs_state = c.take<double>((size_t)n_obj * k_obs * 6);
    double* obs_grad = c.take<double>((size_t)n_obj * k_obs * 6);
    double* obs_hop = c.take<double>((size_t)n_obj * k_obs * 2);
    const SortScratch sorts = sort_scratch(c.take<int32_t>(sort_scratch_ints(n_obj)), n_obj);
    double* adj_state = c.take<double>((size_t)n_obj * kAdjStateDoubles);
    int32_t* seg_ns = c.take<int32_t>((size_t)2 * ((n_obj + kAdjLanes - 1) / kAdjLanes));
    double* adj_tab = c.take<double>((size_t)kAdjTabDoubles);
    double* dense_coef = c.take<double>((size_t)kDenseCoefDoubles);

    hipStream_t s = (hipStream_t)stream;

    AdjParams P;
    std::memset(&P, 0, sizeof(P));
    P.eph = E;
    P.rc = radau_const();
    P.x0 = x0;
    P.perm = perm;
    P.t0 = t0;
    P.n_obj = (int32_t)n_obj;
    P.k_obs = k_obs;
    P.t_obs = t_obs;
    P.obs_pos = obs_pos;
    P.dL_dsky = dL_dsky;
    P.sky_out = sky_out;
    P.grad = grad_x0;
    P.status = status;
    P.h_pref = h_pref;
    P.ckpt = ckpt;
    P.t_end = t_end;
    P.ckpt_days = ckpt_days;
    P.n_ckpt = (int32_t)C;
    P.obs_state = obs_state;
    P.obs_grad = obs_grad;
    P.obs_hop = obs_hop;
    P.steps = scratch;
    P.jac = scratch + (size_t)adj_steps(opts) * kStepDoubles * n_obj;
    P.s_max = adj_steps(opts);
    P.adj_state = adj_state;
    P.seg_ns = seg_ns;
    P.adj_tab = adj_tab;
    P.dense_coef = dense_coef;
    P.max_win_segs = segs_or(opts, 3) + 1;      // the adjoint's own windows: 3 segments (auto)
    P.max_iter = opts->max_iter;
    P.max_steps = opts->max_steps;
    P.zero_start = opts->zero_start != 0;
    P.eps = opts->eps;
    P.h_min = opts->h_min;
    P.h_max = opts->h_max;
    P.h_init = opts->h_init;
    P.safety = 0.25;
    P.smu = std::sqrt(E.gm[0]);
    P.c_light = cl;
    P.lt_tol = opts->lt_tol > 0 ? opts->lt_tol : 1e-15;
    P.lt_iter = opts->lt_iter > 0 ? opts->lt_iter : 10;
    if (opts->kepler_iter < 0) return fail(KETE_EINVAL, "kepler_iter must be >= 0");
    P.kepler_iter = opts->kepler_iter > 0 ? opts->kepler_iter : kKeplerIterDefault;
    const double obliq = 84381.448 / 3600.0 * 3.14159265358979323846 / 180.0;
    P.cos_eps = std::cos(obliq);
    P.sin_eps = std::sin(obliq);

    if (mode == KETE_ADJ_FWD) {
        HIPCHK(fill_zero(status, (size_t)n_obj * sizeof(int32_t), s));
        HIPCHK(launch_hpref_init(x0, h_pref, ncls > 1 ? sorts.keys : nullptr, (int)n_obj, E.gm[0], 0.0, t_end - t0,
                                 ncls, s));
        if (ncls > 1) {
            HIPCHK(launch_body_sort(sorts.keys, (int)n_obj, ncls, perm, sorts.tmp, sorts.counts, s));
        } else {
            HIPCHK(launch_iota(perm, (int)n_obj, s));
        }
    }
    {
        TimedScope ts(kTimeAdjoint, s);
        HIPCHK(launch_adjoint(P, mode, s));
    }
    return KETE_OK;
}

// ---------------------------------------------------------------- batched jobs
namespace {

// Sizes and host-side tables of a batched run (recomputed identically by
// every batch call from the host copies).
struct BatchDims {
    int64_t F = 0, B = 0, NP = 0, nkeys = 0, cand_cap = 0, pairs_cap = 0, max_batch_obj = 0;
    int32_t n_tiles = 0, n_sub = 1;
    std::vector<int2> tiles;
    std::vector<int64_t> b_poff, b_xoff, b_koff;
    std::vector<int32_t> b_obj0, b_G;
};

constexpr int kSmallBatchFrames = 256;   // below this a batch's frames share one grid cell

int batch_dims(const kete_ephem_t* eph, const kete_batch_t* bt, int64_t pairs_cap, const kete_opts_t* o,
               bool tables, BatchDims& d) {
    if (!bt || !bt->jobs_host || bt->n_jobs < 0 || bt->n_batch < 0 || bt->n_bodies < 0)
        return fail(KETE_EINVAL, "bad batch description");
    if (bt->n_bodies > KETE_MAX_OBJ) return fail(KETE_EINVAL, "too many bodies");
    if (pairs_cap < 0) return fail(KETE_EINVAL, "pairs_cap < 0");
    d.F = bt->frames.n_frames;
    d.B = bt->n_batch;
    d.n_sub = bt->frames.n_sub;
    d.pairs_cap = pairs_cap;
    if (d.n_sub < 1 || d.n_sub > KETE_MAX_SUB) return fail(KETE_EINVAL, "n_sub outside 1..%d", KETE_MAX_SUB);
    if (d.B > 0 && (!bt->batch_job_host || !bt->batch_epoch_host || !bt->batch_off_host))
        return fail(KETE_EINVAL, "null batch host tables");
    const double L = o->cell_chord > 0 ? o->cell_chord : 0.10;
    const int Gbig = (int)std::ceil(2.0 / L - 1e-9);
    if (Gbig > 128) return fail(KETE_EINVAL, "cell_chord too small");
    // jobs
    const kete_job_t* J = bt->jobs_host;
    double tlo = eph ? eph->t_start : -1e300, thi = eph ? t_end_of(eph) : 1e300;
    for (int j = 0; j < bt->n_jobs; ++j) {
        if (J[j].n_obj < 0 || J[j].n_epoch < 0 || J[j].obj_off < 0 || J[j].obj_off + J[j].n_obj > bt->n_bodies ||
            J[j].epoch_off < 0 || J[j].epoch_off + J[j].n_epoch > bt->n_epochs || J[j].xout_off < 0)
            return fail(KETE_EINVAL, "job %d out of range", j);
        if (!(J[j].t0 >= tlo && J[j].t0 <= thi)) return fail(KETE_ERANGE, "job %d t0 outside the ephemeris", j);
    }
    // tiles of KETE_BATCH_TILE bodies
    constexpr int T = KETE_BATCH_TILE;
    int64_t n_tiles = 0;
    for (int j = 0; j < bt->n_jobs; ++j) n_tiles += (J[j].n_obj + T - 1) / T;
    if (n_tiles > INT32_MAX) return fail(KETE_EINVAL, "too many tiles");
    d.n_tiles = (int32_t)n_tiles;
    if (tables) {
        d.tiles.reserve(d.n_tiles);
        for (int j = 0; j < bt->n_jobs; ++j)
            for (int t = 0; t < (J[j].n_obj + T - 1) / T; ++t) d.tiles.push_back(make_int2(j, t));
    }
    // batches
    if (tables) {
        d.b_poff.assign(d.B + 1, 0);
        d.b_koff.assign(d.B + 1, 0);
        d.b_xoff.assign(d.B, 0);
        d.b_obj0.assign(d.B, 0);
        d.b_G.assign(d.B, 1);
    }
    int64_t np = 0, nk = 0;
    for (int64_t b = 0; b < d.B; ++b) {
        const int j = bt->batch_job_host[b];
        if (j < 0 || j >= bt->n_jobs) return fail(KETE_EINVAL, "batch %lld has no job", (long long)b);
        const int e = bt->batch_epoch_host[b];
        if (e < 0 || e >= J[j].n_epoch) return fail(KETE_EINVAL, "batch %lld epoch out of range", (long long)b);
        const int nf = bt->batch_off_host[b + 1] - bt->batch_off_host[b];
        const int G = nf < kSmallBatchFrames ? 1 : Gbig;
        if (tables) {
            d.b_poff[b] = np;
            d.b_koff[b] = nk;
            d.b_xoff[b] = J[j].xout_off + 6 * (int64_t)e * J[j].n_obj;
            d.b_obj0[b] = (int32_t)J[j].obj_off;
            d.b_G[b] = G;
        }
        np += J[j].n_obj;
        nk += (int64_t)G * G * G + 1;
        d.max_batch_obj = std::max<int64_t>(d.max_batch_obj, J[j].n_obj);
    }
    if (tables) { d.b_poff[d.B] = np; d.b_koff[d.B] = nk; }
    if (np >= 2000000000LL || nk >= 2000000000LL) return fail(KETE_EINVAL, "batch too large for 32-bit indices");
    d.NP = np;
    d.nkeys = nk;
    d.cand_cap = cand_capacity(d.F, pairs_cap);
    // Longest first: a tile's cost is about the integrated path length of
    // its job (days from t0 through every epoch in order) plus a couple of
    // steps per landing; without host epochs the landing count alone.
    if (tables && !d.tiles.empty()) {
        std::vector<double> c(bt->n_jobs);
        for (int j = 0; j < bt->n_jobs; ++j) {
            double len = 0.0, t = J[j].t0;
            if (bt->epochs_host)
                for (int e = 0; e < J[j].n_epoch; ++e) {
                    const double te = bt->epochs_host[J[j].epoch_off + e];
                    len += std::fabs(te - t);
                    t = te;
                }
            c[j] = len + 8.0 * J[j].n_epoch;
        }
        std::stable_sort(d.tiles.begin(), d.tiles.end(),
                         [&](const int2& a, const int2& b) { return c[a.x] > c[b.x]; });
    }
    return KETE_OK;
}

struct BatchWs {
    int2* tiles;
    unsigned int* tile_counter;
    double* dense_coef;
    int32_t* perm;
    FovParams P;
    int32_t *qkey, *cnt, *fcnt, *fstart, *okey, *orank, *osorted, *osub, *ostart, *ocnt, *icnt, *istart;
    unsigned long long* items;
    unsigned long long *counters, *sorted;
    void *scan_scratch, *oscan, *wscan;
    int64_t *b_poff, *b_xoff, *b_koff;
    int32_t *b_obj0, *b_G;
};

size_t batch_carve(const BatchDims& d, const kete_batch_t* bt, char* base, BatchWs& w) {
    Carver c{base};
    w.tiles = c.take<int2>((size_t)std::max(d.n_tiles, 1));
    w.tile_counter = c.take<unsigned int>(64);
    w.dense_coef = c.take<double>(kDenseCoefDoubles);
    w.perm = c.take<int32_t>((size_t)std::max<int64_t>(bt->n_bodies, 1));
    FovParams& P = w.P;
    std::memset(&P, 0, sizeof(P));
    P.fcap = c.take<double>((size_t)d.F * 8);
    P.btab = c.take<double>((size_t)d.B * kBatchStride);
    w.qkey = c.take<int32_t>((size_t)d.F);
    w.cnt = c.take<int32_t>((size_t)d.nkeys + 1);
    P.cell_start = c.take<int32_t>((size_t)d.nkeys + 1);
    P.cell_frames = c.take<int32_t>((size_t)d.F);
    P.cell_caps = c.take<double>((size_t)d.F * 8);
    P.pairs = c.take<unsigned long long>((size_t)std::max<int64_t>(d.pairs_cap, 1));
    w.counters = c.take<unsigned long long>(kFovCounters);
    w.fcnt = c.take<int32_t>((size_t)d.F + 1);
    w.fstart = c.take<int32_t>((size_t)d.F + 1);
    w.sorted = c.take<unsigned long long>((size_t)std::max<int64_t>(d.pairs_cap, 1));
    w.scan_scratch = c.take<char>(std::max(scan_scratch_bytes(d.nkeys), scan_scratch_bytes(d.F)));
    P.cand = c.take<unsigned long long>((size_t)d.cand_cap);
    P.frame_batch = c.take<int32_t>((size_t)d.F);
    w.okey = c.take<int32_t>((size_t)d.NP);
    w.orank = c.take<int32_t>((size_t)d.NP);
    w.osorted = c.take<int32_t>((size_t)d.NP);
    w.osub = c.take<int32_t>((size_t)d.NP);
    w.ostart = c.take<int32_t>((size_t)d.nkeys + 1);
    w.ocnt = c.take<int32_t>((size_t)d.nkeys + 1);
    P.wide = c.take<unsigned long long>((size_t)std::max<int64_t>(d.NP, 1));
    w.oscan = c.take<char>(scan_scratch_bytes(d.nkeys));
    w.icnt = c.take<int32_t>((size_t)d.nkeys + 1);
    w.istart = c.take<int32_t>((size_t)d.nkeys + 1);
    w.items = c.take<unsigned long long>((size_t)fov_item_capacity(d.nkeys, d.NP));
    w.b_poff = c.take<int64_t>((size_t)d.B + 1);
    w.b_obj0 = c.take<int32_t>((size_t)d.B + 1);
    w.b_xoff = c.take<int64_t>((size_t)d.B + 1);
    w.b_G = c.take<int32_t>((size_t)d.B + 1);
    w.b_koff = c.take<int64_t>((size_t)d.B + 1);
    P.fail = c.take<int32_t>((size_t)std::max<int64_t>(bt->n_bodies, 1));
    P.loc = bt->frames.n_sub > 1 ? c.take<double>((size_t)d.F * kLocStride) : nullptr;
    P.cell_obs = c.take<double>((size_t)fov_cell_frame_doubles(d.F, bt->frames.n_sub));
    P.cell_normals = P.cell_obs ? reinterpret_cast<float*>(P.cell_obs + 4 * d.F) : nullptr;
    P.exact_rec = P.cell_obs ? P.cell_obs + 4 * d.F + 6 * (int64_t)bt->frames.n_sub * d.F : nullptr;
    P.wide_parts = c.take<int32_t>((size_t)std::max<int64_t>(d.NP, 1));
    P.wide_off = c.take<int32_t>((size_t)d.NP + 1);
    w.wscan = c.take<char>(scan_scratch_bytes(d.NP));
    P.wide_next = w.counters ? (unsigned int*)(w.counters + kFovWideCursorBase) : nullptr;
    return c.off;
}

}  // namespace

size_t kete_batch_workspace_size(const kete_ephem_t* eph, const kete_batch_t* batch, int64_t pairs_cap,
                                 const kete_opts_t* opts) {
    kete_opts_t dflt;
    if (!opts) { kete_default_opts(&dflt); opts = &dflt; }
    BatchDims d;
    if (batch_dims(eph, batch, pairs_cap, opts, false, d)) return 0;
    BatchWs w;
    return batch_carve(d, batch, nullptr, w);
}

int kete_batch_plan(const kete_ephem_t* eph, const kete_batch_t* batch, int64_t pairs_cap, const kete_opts_t* opts,
                    void* workspace, size_t ws_bytes, void* stream) {
    kete_opts_t dflt;
    if (!opts) { kete_default_opts(&dflt); opts = &dflt; }
    g_err.clear();
    EphemArgs E;
    int rc = ephem_args(eph, opts->c_light > 0 ? opts->c_light : kC, E);
    if (rc) return rc;
    BatchDims d;
    if ((rc = batch_dims(eph, batch, pairs_cap, opts, true, d))) return rc;
    if (!workspace) return fail(KETE_EWORKSPACE, "workspace is null");
    BatchWs w;
    const size_t need = batch_carve(d, batch, nullptr, w);
    if (ws_bytes < need) return fail(KETE_EWORKSPACE, "workspace %zu bytes < %zu required", ws_bytes, need);
    batch_carve(d, batch, (char*)workspace, w);
    hipStream_t s = (hipStream_t)stream;
    if (d.n_tiles) HIPCHK(hipMemcpyAsync(w.tiles, d.tiles.data(), d.tiles.size() * sizeof(int2), hipMemcpyHostToDevice, s));
    if (d.B) {
        HIPCHK(hipMemcpyAsync(w.b_poff, d.b_poff.data(), d.b_poff.size() * sizeof(int64_t), hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(w.b_koff, d.b_koff.data(), d.b_koff.size() * sizeof(int64_t), hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(w.b_xoff, d.b_xoff.data(), d.b_xoff.size() * sizeof(int64_t), hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(w.b_obj0, d.b_obj0.data(), d.b_obj0.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(w.b_G, d.b_G.data(), d.b_G.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
    }
    HIPCHK(hipStreamSynchronize(s));
    return KETE_OK;
}

int kete_batch_run(const kete_ephem_t* eph, const kete_batch_t* batch, int64_t pairs_cap, const kete_opts_t* opts,
                   double* x_out, int32_t* status, void* workspace, size_t ws_bytes, void* stream) {
    kete_opts_t dflt;
    if (!opts) { kete_default_opts(&dflt); opts = &dflt; }
    g_err.clear();
    EphemArgs E;
    const double cl = opts->c_light > 0 ? opts->c_light : kC;
    int rc = ephem_args(eph, cl, E);
    if (rc) return rc;
    if (!workspace || (!x_out && batch->n_bodies) || (!status && batch->n_bodies)) return fail(KETE_EINVAL, "null pointer");
    if (!batch->jobs || (batch->n_bodies && !batch->x0) || (batch->n_epochs && !batch->epochs)) return fail(KETE_EINVAL, "null batch pointer");
    hipStream_t s = (hipStream_t)stream;
    const int64_t cap = pairs_cap;
    BatchDims dc;
    if ((rc = batch_dims(eph, batch, cap, opts, false, dc))) return rc;
    BatchWs w;
    if (ws_bytes < batch_carve(dc, batch, nullptr, w)) return fail(KETE_EWORKSPACE, "workspace too small");
    batch_carve(dc, batch, (char*)workspace, w);
    BatchParams B;
    std::memset(&B, 0, sizeof(B));
    B.eph = E;
    B.rc = radau_const();
    B.jobs = batch->jobs;
    B.n_jobs = batch->n_jobs;
    B.n_tiles = dc.n_tiles;
    B.tiles = w.tiles;
    B.tile_counter = w.tile_counter;
    B.x0 = batch->x0;
    B.epochs = batch->epochs;
    B.x_out = x_out;
    B.status = status;
    B.perm = w.perm;
    B.n_buckets = bucket_count(opts);
    B.max_win_segs = segs_or(opts, 2) + 1;
    B.max_iter = opts->max_iter;
    B.max_steps = opts->max_steps;
    B.zero_start = opts->zero_start != 0;
    B.land_epochs = opts->land_epochs != 0;
    B.dense_coef = w.dense_coef;
    B.eps = opts->eps;
    B.h_min = opts->h_min;
    B.h_max = opts->h_max;
    B.h_init = opts->h_init;
    B.safety = 0.25;
    {
        TimedScope ts(kTimeBatch, s);
        HIPCHK(launch_batch(B, opts->persist_waves > 0 ? std::min(opts->persist_waves, 32) : 8, s));
    }
    // field-of-view stages over every batch
    FovParams& P = w.P;
    P.eph = E;
    P.x_epoch = x_out;
    P.status = status;
    P.n_obj = (int32_t)batch->n_bodies;
    P.n_batch = (int32_t)dc.B;
    P.n_frames = dc.F;
    P.t_ref = batch->t_ref;
    P.batch_off = batch->batch_off;
    P.frame_order = batch->frame_order;
    P.ft = batch->frames.t;
    P.fobs = batch->frames.obs;
    P.normals = batch->frames.normals;
    P.n_sub = batch->frames.n_sub;
    P.n_pairs = w.counters;
    P.stats = w.counters + 1;
    P.n_cand = w.counters + 5;
    P.n_wide = w.counters + 6;
    P.n_fail = w.counters + 8;
    P.status_out = status;
    P.cap = cap;
    P.cand_cap = dc.cand_cap;
    P.b_poff = w.b_poff;
    P.b_obj0 = w.b_obj0;
    P.b_xoff = w.b_xoff;
    P.b_G = w.b_G;
    P.b_koff = w.b_koff;
    P.n_keys = dc.nkeys;
    P.n_pairs_total = dc.NP;
    P.max_batch_obj = dc.max_batch_obj;
    P.mu = E.gm[0];
    P.smu = std::sqrt(E.gm[0]);
    P.c_light = cl;
    P.lt_tol = opts->lt_tol > 0 ? opts->lt_tol : 1e-15;
    P.lt_iter = opts->lt_iter > 0 ? opts->lt_iter : 10;
    if (opts->kepler_iter < 0) return fail(KETE_EINVAL, "kepler_iter must be >= 0");
    P.kepler_iter = opts->kepler_iter > 0 ? opts->kepler_iter : kKeplerIterDefault;
    P.max_cells = 1024;
    P.sin_overflow = 0.5;
    TimedScope ts(kTimeFov, s);
    HIPCHK(fill_zero(w.counters, kFovCounters * sizeof(unsigned long long), s));
    HIPCHK(fill_zero(P.fail, (size_t)std::max<int64_t>(batch->n_bodies, 1) * sizeof(int32_t), s));
    if (dc.B > 0 && dc.F > 0 && dc.NP > 0) {
        HIPCHK(fov_prepare(P, w.qkey, w.cnt, w.cnt, w.scan_scratch, s));
        HIPCHK(fov_sort_objects(P, w.okey, w.orank, w.ocnt, w.ostart, w.osorted, w.osub, w.oscan, s));
        P.obj_sorted = w.osorted;
        P.obj_start = w.ostart;
        P.obj_count = w.ocnt;
        {
            TimedScope tj(kTimeFovJoin, s);
            HIPCHK(fov_candidates(P, w.icnt, w.istart, w.items, (unsigned int*)(w.counters + kFovCursorBase), w.oscan,
                                  w.wscan, s));
        }
        HIPCHK(fov_exact(P, s));
    }
    return KETE_OK;
}

int kete_batch_pairs(const kete_batch_t* batch, int64_t pairs_cap, const kete_opts_t* opts, int32_t* pf, int32_t* ps,
                     int32_t* po, int64_t* n_pairs, void* workspace, size_t ws_bytes, void* stream) {
    g_err.clear();
    kete_opts_t dflt;
    if (!opts) { kete_default_opts(&dflt); opts = &dflt; }
    if (!n_pairs || !workspace) return fail(KETE_EINVAL, "null pointer");
    *n_pairs = 0;
    BatchDims d;
    int rc = batch_dims(nullptr, batch, pairs_cap, opts, false, d);
    if (rc) return rc;
    BatchWs w;
    if (ws_bytes < batch_carve(d, batch, nullptr, w)) return fail(KETE_EWORKSPACE, "workspace too small");
    batch_carve(d, batch, (char*)workspace, w);
    hipStream_t s = (hipStream_t)stream;
    unsigned long long hc[kFovCursorBase];
    HIPCHK(hipMemcpyAsync(hc, w.counters, sizeof(hc), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (int i = 0; i < 4; ++i) g_fov_stats[i] = hc[1 + i];
    int64_t np = (int64_t)hc[0];
    *n_pairs = np;
    if ((int64_t)hc[5] > d.cand_cap || np > pairs_cap) {
        *n_pairs = retry_pairs_cap(np, (int64_t)hc[5], pairs_cap);
        return fail(KETE_ECAPACITY, "%lld pairs / %llu exact-test candidates exceed pairs_cap %lld / %lld",
                    (long long)np, hc[5], (long long)pairs_cap, (long long)d.cand_cap);
    }
    if (np > 0 && (!pf || !ps || !po)) return fail(KETE_EINVAL, "null output pointer");
    if (hc[8] > 0) {
        if ((rc = drop_failed_pairs(w.P.pairs, np, w.P.fail, w.sorted, w.counters, &np, s))) return rc;
        *n_pairs = np;
        HIPCHK(fov_sort(w.sorted, np, d.F, batch->n_bodies, batch->frames.n_sub, w.fcnt, w.fstart, w.P.pairs,
                        w.scan_scratch, pf, ps, po, s));
        return KETE_OK;
    }
    HIPCHK(fov_sort(w.P.pairs, np, d.F, batch->n_bodies, batch->frames.n_sub, w.fcnt, w.fstart, w.sorted,
                    w.scan_scratch, pf, ps, po, s));
    return KETE_OK;
}

struct BatchGraph {
    hipGraph_t graph;
    hipGraphExec_t exec;
};

int kete_batch_graph_create(const kete_ephem_t* eph, const kete_batch_t* batch, int64_t pairs_cap,
                            const kete_opts_t* opts, double* x_out, int32_t* status, void* workspace, size_t ws_bytes,
                            void* stream, void** graph) {
    g_err.clear();
    if (!graph) return fail(KETE_EINVAL, "graph is null");
    *graph = nullptr;
    hipStream_t cs = nullptr;
    HIPCHK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) { hipStreamDestroy(cs); return fail(KETE_EDEVICE, "begin capture: %s", hipGetErrorString(e)); }
    const bool was_timing = g_timing;
    g_timing = false;
    int rc = kete_batch_run(eph, batch, pairs_cap, opts, x_out, status, workspace, ws_bytes, cs);
    g_timing = was_timing;
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(cs, &g);
    hipStreamDestroy(cs);
    if (rc) { if (g) hipGraphDestroy(g); return rc; }
    if (e != hipSuccess || !g) return fail(KETE_EDEVICE, "end capture: %s", hipGetErrorString(e));
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    if (e != hipSuccess) { hipGraphDestroy(g); return fail(KETE_EDEVICE, "instantiate: %s", hipGetErrorString(e)); }
    BatchGraph* bg = new BatchGraph{g, ex};
    *graph = bg;
    (void)stream;
    return KETE_OK;
}

int kete_batch_graph_launch(void* graph, void* stream) {
    g_err.clear();
    if (!graph) return fail(KETE_EINVAL, "graph is null");
    BatchGraph* bg = (BatchGraph*)graph;
    hipStream_t s = (hipStream_t)stream;
    TimedScope ts(kTimeBatch, s);
    HIPCHK(hipGraphLaunch(bg->exec, s));
    return KETE_OK;
}

int kete_batch_graph_destroy(void* graph) {
    if (!graph) return KETE_OK;
    BatchGraph* bg = (BatchGraph*)graph;
    hipGraphExecDestroy(bg->exec);
    hipGraphDestroy(bg->graph);
    delete bg;
    return KETE_OK;
}

// Coordinate descent over the launch parameters of a batched run, each
// candidate timed with events over `reps` runs after one warm-up run.
int kete_batch_autotune(const kete_ephem_t* eph, const kete_batch_t* batch, int64_t pairs_cap,
                        const kete_opts_t* base, int32_t reps, double* x_out, int32_t* status, void* workspace,
                        size_t ws_bytes, void* stream, kete_tune_progress_fn progress, void* user,
                        kete_opts_t* best, double* best_ms) {
    g_err.clear();
    if (!best) return fail(KETE_EINVAL, "best is null");
    if (reps < 1 || reps > 100) return fail(KETE_EINVAL, "reps outside 1..100");
    kete_opts_t cur;
    if (base) cur = *base; else kete_default_opts(&cur);
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t ea = nullptr, eb = nullptr;
    HIPCHK(hipEventCreate(&ea));
    if (hipEventCreate(&eb) != hipSuccess) { hipEventDestroy(ea); return fail(KETE_EDEVICE, "event create"); }
    auto trial = [&](const kete_opts_t& o, double& ms) -> int {
        ms = HUGE_VAL;
        const size_t need = kete_batch_workspace_size(eph, batch, pairs_cap, &o);
        if (need == 0) return KETE_EINVAL;
        if (need > ws_bytes) return KETE_OK;          // candidate does not fit: skipped
        int rc = kete_batch_plan(eph, batch, pairs_cap, &o, workspace, ws_bytes, stream);
        if (!rc) rc = kete_batch_run(eph, batch, pairs_cap, &o, x_out, status, workspace, ws_bytes, stream);
        if (rc) return rc;
        if (hipEventRecord(ea, s) != hipSuccess) return fail(KETE_EDEVICE, "event record");
        for (int r = 0; r < reps && !rc; ++r)
            rc = kete_batch_run(eph, batch, pairs_cap, &o, x_out, status, workspace, ws_bytes, stream);
        if (rc) return rc;
        float t = 0.0f;
        if (hipEventRecord(eb, s) != hipSuccess || hipEventSynchronize(eb) != hipSuccess ||
            hipEventElapsedTime(&t, ea, eb) != hipSuccess)
            return fail(KETE_EDEVICE, "event timing");
        ms = (double)t / reps;
        if (progress) progress(&o, ms, user);
        return KETE_OK;
    };
    double cur_ms;
    int rc = trial(cur, cur_ms);
    if (!rc && !(cur_ms < HUGE_VAL)) rc = fail(KETE_EWORKSPACE, "workspace too small for the base options");
    struct Axis { int which; double v[5]; int n; };
    const Axis axes[] = {
        {0, {1, 4, 8, 16}, 4},             // n_buckets
        {1, {2, 4, 8, 12}, 4},             // persist_waves
        {2, {1, 2, 4}, 3},                 // window_segs
        {3, {64, 128, 256}, 3},            // fov_block
        {4, {0.05, 0.10, 0.16}, 3},        // cell_chord
    };
    auto with = [](kete_opts_t o, int which, double v) {
        switch (which) {
            case 0: o.n_buckets = (int32_t)v; break;
            case 1: o.persist_waves = (int32_t)v; break;
            case 2: o.window_segs = (int32_t)v; break;
            case 3: o.fov_block = (int32_t)v; break;
            default: o.cell_chord = v; break;
        }
        return o;
    };
    for (const Axis& a : axes) {
        if (rc) break;
        kete_opts_t axis_best = cur;
        double axis_ms = cur_ms;
        for (int i = 0; i < a.n && !rc; ++i) {
            const kete_opts_t o = with(cur, a.which, a.v[i]);
            if (std::memcmp(&o, &cur, sizeof(o)) == 0) continue;
            double ms;
            rc = trial(o, ms);
            if (!rc && ms < axis_ms) { axis_ms = ms; axis_best = o; }
        }
        cur = axis_best;
        cur_ms = axis_ms;
    }
    hipEventDestroy(ea);
    hipEventDestroy(eb);
    if (rc) return rc;
    // leave the workspace planned for the winner
    if ((rc = kete_batch_plan(eph, batch, pairs_cap, &cur, workspace, ws_bytes, stream))) return rc;
    *best = cur;
    if (best_ms) *best_ms = cur_ms;
    return KETE_OK;
}

// Live kernel timing: while enabled, every integrator / FoV launch made by
// this thread is bracketed by HIP events on its stream.
void kete_timing_enable(int on) {
    g_timing = on != 0;
}

// Waits for the recorded events, returns the summed milliseconds and the
// bracket count per kind (see kete_timing_read_all) and forgets them.
int kete_timing_read_all(double ms[8], int64_t count[8]) {
    for (int k = 0; k < kTimeKinds; ++k) { ms[k] = 0.0; count[k] = 0; }
    int rc = KETE_OK;
    for (auto& r : g_timed) {
        float t = 0.0f;
        if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&t, r.a, r.b) != hipSuccess) {
            rc = fail(KETE_EDEVICE, "event timing failed");
        } else {
            ms[r.kind] += t;
            count[r.kind] += 1;
        }
        g_event_pool.push_back(r.a);
        g_event_pool.push_back(r.b);
    }
    g_timed.clear();
    return rc;
}

int kete_timing_read(double ms[4], int64_t count[4]) {
    double m8[kTimeKinds];
    int64_t c8[kTimeKinds];
    const int rc = kete_timing_read_all(m8, c8);
    for (int k = 0; k < 4; ++k) { ms[k] = m8[k]; count[k] = c8[k]; }
    return rc;
}

void kete_fov_last_stats(int64_t out[4]) {
    for (int i = 0; i < 4; ++i) out[i] = (int64_t)g_fov_stats[i];
}

void kete_fov_last_counts(int64_t out[8]) {
    for (int i = 0; i < 8; ++i) out[i] = (int64_t)g_fov_stats[i];
}

int kete_lighttime_directions(const kete_ephem_t* eph, const double* x_ref, double t_ref, int64_t n_obj,
                              const double* t_obs, const double* obs, int64_t n_q, double* d, double* tau,
                              const kete_opts_t* opts, void* stream) {
    kete_opts_t dflt;
    if (!opts) { kete_default_opts(&dflt); opts = &dflt; }
    g_err.clear();
    EphemArgs E;
    const double cl = opts->c_light > 0 ? opts->c_light : kC;
    int rc = ephem_args(eph, cl, E);
    if (rc) return rc;
    if (n_obj < 0 || n_q < 0 || n_obj > KETE_MAX_OBJ) return fail(KETE_EINVAL, "bad sizes");
    if (n_obj == 0 || n_q == 0) return KETE_OK;
    if (!x_ref || !t_obs || !obs || !d) return fail(KETE_EINVAL, "null pointer");
    FovParams P;
    std::memset(&P, 0, sizeof(P));
    P.eph = E;
    P.n_obj = (int32_t)n_obj;
    P.mu = E.gm[0];
    P.smu = std::sqrt(E.gm[0]);
    P.c_light = cl;
    P.lt_tol = opts->lt_tol > 0 ? opts->lt_tol : 1e-15;
    P.lt_iter = opts->lt_iter > 0 ? opts->lt_iter : 10;
    if (opts->kepler_iter < 0) return fail(KETE_EINVAL, "kepler_iter must be >= 0");
    P.kepler_iter = opts->kepler_iter > 0 ? opts->kepler_iter : kKeplerIterDefault;
    HIPCHK(launch_directions(P, x_ref, t_ref, t_obs, obs, n_q, d, tau, (hipStream_t)stream));
    return KETE_OK;
}

size_t kete_magnitudes_workspace_size(int64_t n_frames) {
    if (n_frames < 0 || n_frames > INT32_MAX) return 0;
    return mag_workspace_bytes(n_frames);
}

}  // extern "C"

namespace {

// Shared body of the two magnitude entry points.  static_scratch: the
// frame-to-batch map lives in the library's static device array (its
// frame limit is checked, nothing is allocated) instead of the caller's
// workspace.
int pair_magnitudes_impl(const kete_ephem_t* eph, const double* x_epoch, int64_t n_obj, int64_t n_batch,
                         const double* t_ref, const int32_t* batch_off, const int32_t* frame_order,
                         const kete_frames_t* frames, const int32_t* pf, const int32_t* po, int64_t n_pairs,
                         const double* h_mag, const double* g_slope, double* v_mag, double* geom,
                         const kete_opts_t* opts, void* workspace, size_t ws_bytes, bool static_scratch,
                         void* stream) {
    kete_opts_t dflt;
    if (!opts) { kete_default_opts(&dflt); opts = &dflt; }
    g_err.clear();
    EphemArgs E;
    const double cl = opts->c_light > 0 ? opts->c_light : kC;
    int rc = ephem_args(eph, cl, E);
    if (rc) return rc;
    if (!frames) return fail(KETE_EINVAL, "frames is null");
    if (n_obj < 0 || n_obj > KETE_MAX_OBJ) return fail(KETE_EINVAL, "n_obj %lld outside 0..%d", (long long)n_obj, KETE_MAX_OBJ);
    if (n_batch < 0 || n_pairs < 0 || frames->n_frames < 0 || frames->n_frames > INT32_MAX)
        return fail(KETE_EINVAL, "bad sizes");
    if ((double)n_batch * (double)n_obj >= 2.0e9) return fail(KETE_EINVAL, "n_batch x n_obj must stay below 2^31");
    if (n_pairs == 0) return KETE_OK;
    if (!pf || !po || !h_mag || !g_slope || !v_mag) return fail(KETE_EINVAL, "null pointer");
    const int64_t F = frames->n_frames;
    if (n_obj > 0 && n_batch > 0 && F > 0 && (!x_epoch || !t_ref || !batch_off || !frame_order || !frames->t ||
                                              !frames->obs))
        return fail(KETE_EINVAL, "null pointer");
    if (static_scratch) {
        if (F > kMagScratchFrames)
            return fail(KETE_EWORKSPACE, "n_frames %lld exceeds the %lld frames of the static scratch",
                        (long long)F, (long long)kMagScratchFrames);
        HIPCHK(mag_static_scratch(&workspace));
    } else {
        if (!workspace) return fail(KETE_EWORKSPACE, "workspace is null");
        const size_t need = kete_magnitudes_workspace_size(F);
        if (ws_bytes < need) return fail(KETE_EWORKSPACE, "workspace %zu bytes < %zu required", ws_bytes, need);
    }
    MagParams P;
    std::memset(&P, 0, sizeof(P));
    P.eph = E;
    P.x_epoch = x_epoch;
    P.n_obj = (int32_t)n_obj;
    // with no bodies, batches or frames every pair is out of range: NaN
    P.n_batch = (n_obj > 0 && F > 0) ? (int32_t)n_batch : 0;
    P.n_frames = F;
    P.t_ref = t_ref;
    P.batch_off = batch_off;
    P.frame_order = frame_order;
    P.ft = frames->t;
    P.fobs = frames->obs;
    P.pf = pf;
    P.po = po;
    P.n_pairs = n_pairs;
    P.h_mag = h_mag;
    P.g_slope = g_slope;
    P.v_mag = v_mag;
    P.geom = geom;
    P.smu = std::sqrt(E.gm[0]);
    P.c_light = cl;
    P.lt_tol = opts->lt_tol > 0 ? opts->lt_tol : 1e-15;
    P.lt_iter = opts->lt_iter > 0 ? opts->lt_iter : 10;
    if (opts->kepler_iter < 0) return fail(KETE_EINVAL, "kepler_iter must be >= 0");
    P.kepler_iter = opts->kepler_iter > 0 ? opts->kepler_iter : kKeplerIterDefault;
    P.t_lo = eph->t_start;
    P.t_hi = t_end_of(eph);
    HIPCHK(launch_pair_mag(P, workspace, !static_scratch, (hipStream_t)stream));
    return KETE_OK;
}

}  // namespace

extern "C" {

int kete_pair_magnitudes(const kete_ephem_t* eph, const double* x_epoch, int64_t n_obj, int64_t n_batch,
                         const double* t_ref, const int32_t* batch_off, const int32_t* frame_order,
                         const kete_frames_t* frames, const int32_t* pf, const int32_t* po, int64_t n_pairs,
                         const double* h_mag, const double* g_slope, double* v_mag, double* geom,
                         const kete_opts_t* opts, void* workspace, size_t ws_bytes, void* stream) {
    return pair_magnitudes_impl(eph, x_epoch, n_obj, n_batch, t_ref, batch_off, frame_order, frames, pf, po, n_pairs,
                                h_mag, g_slope, v_mag, geom, opts, workspace, ws_bytes, false, stream);
}

int kete_pair_magnitudes_noalloc(const kete_ephem_t* eph, const double* x_epoch, int64_t n_obj, int64_t n_batch,
                                 const double* t_ref, const int32_t* batch_off, const int32_t* frame_order,
                                 const kete_frames_t* frames, const int32_t* pf, const int32_t* po, int64_t n_pairs,
                                 const double* h_mag, const double* g_slope, double* v_mag, double* geom,
                                 const kete_opts_t* opts, void* stream) {
    return pair_magnitudes_impl(eph, x_epoch, n_obj, n_batch, t_ref, batch_off, frame_order, frames, pf, po, n_pairs,
                                h_mag, g_slope, v_mag, geom, opts, nullptr, 0, true, stream);
}

int kete_ephem_eval(const kete_ephem_t* eph, const double* t, const double* t_host, int64_t n_q, double* out,
                    void* stream) {
    g_err.clear();
    EphemArgs E;
    int rc = ephem_args(eph, kC, E);
    if (rc) return rc;
    if (n_q < 0) return fail(KETE_EINVAL, "n_q < 0");
    if (n_q == 0) return KETE_OK;
    if (!t || !t_host || !out) return fail(KETE_EINVAL, "null pointer");
    for (int64_t i = 0; i < n_q; ++i)
        if (!(t_host[i] >= eph->t_start && t_host[i] <= t_end_of(eph)))
            return fail(KETE_ERANGE, "t[%lld] = %.9g outside ephemeris", (long long)i, t_host[i]);
    HIPCHK(launch_ephem_eval(E, t, n_q, out, (hipStream_t)stream));
    return KETE_OK;
}

}  // extern "C"
