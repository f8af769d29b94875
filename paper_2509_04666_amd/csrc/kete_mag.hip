// Apparent V magnitude of every (frame, object) pair in the H-G system
// (Sect. 3.3; Bowell et al. 1989), an epilogue of the field-of-view stage.
//
// One lane per pair.  The lane repeats the exact test's light-time hop
// from the pair's batch epoch (it is cheap next to finding the pairs and
// saves the field-of-view kernels a per-pair record), which gives the
// observer-to-body vector d, and the heliocentric emission position r
// from the Sun's cubic about the frame time.  With
// c = r . d and s = |r x d| the phase angle is atan2(s, c) and
// tan(alpha / 2) = s / (|r| |d| + c), so the phase functions need no
// trigonometric call.  Reads per pair: two indices, the batch and frame
// records and one body state (about 120 bytes); the work is the hop's
// handful of Kepler iterations and Chebyshev evaluations, so the kernel
// is bound by FP64 arithmetic, not by HBM.
#include <math.h>

#include <mutex>

#include "kete_mag.hpp"

namespace kete {
namespace {

constexpr double kNaN = __builtin_nan("");

// Constants of the two H-G phase functions Phi_i = exp(-A_i t^B_i),
// t = tan(alpha / 2).
constexpr double kA1 = 3.33, kB1 = 0.63, kA2 = 1.87, kB2 = 1.22;

__global__ void k_mag_fill(int32_t* __restrict__ fb, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        fb[i] = -1;
}

// Batch of every frame: position q of the batched frame order lies in
// batch b when batch_off[b] <= q < batch_off[b + 1].
__global__ void k_mag_frame_batch(const MagParams p, int32_t* __restrict__ fb) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= p.n_frames || q >= (int64_t)p.batch_off[p.n_batch]) return;
    int lo = 0, hi = p.n_batch - 1;           // last b with batch_off[b] <= q
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if ((int64_t)p.batch_off[mid] <= q) lo = mid; else hi = mid - 1;
    }
    const int32_t f = p.frame_order[q];
    if (f >= 0 && f < p.n_frames) fb[f] = lo;
}

// What a pair needs of its frame, computed once per frame when the caller's
// workspace has room (kMagRec doubles): frame time, batch epoch, observer,
// the Sun's position and velocity at the epoch, and its cubic about the
// frame time.  Frames outside every batch get a NaN epoch.
__device__ __forceinline__ void mag_frame_quantities(const MagParams& p, int b, int64_t f, double* R) {
    const EphemArgs& E = p.eph;
    const double tr = p.t_ref[b], tf = p.ft[f];
    // the Sun at the epoch from the same chunked evaluation as its cubic
    // about the frame time: a few rounds of coefficient loads, not one
    // dependent load per coefficient
    const SunCubic s_ref = sun_cubic(E.coef, 0, E.deg1, tr, E.t_start, E.seg_days, E.inv_seg, 0, E.n_seg - 1);
    const SunCubic s_f = sun_cubic(E.coef, 0, E.deg1, tf, E.t_start, E.seg_days, E.inv_seg, 0, E.n_seg - 1);
    R[0] = tf;
    R[1] = tr;
    for (int k = 0; k < 3; ++k) {
        R[2 + k] = p.fobs[3 * f + k];
        R[5 + k] = s_ref.s[k];
        R[8 + k] = s_ref.v[k];
        R[11 + k] = s_f.s[k];
        R[14 + k] = s_f.v[k];
        R[17 + k] = s_f.a[k];
        R[20 + k] = s_f.j[k];
    }
    R[23] = 0.0;
}

__global__ void k_mag_frame_rec(const MagParams p, const int32_t* __restrict__ fb, double* __restrict__ rec) {
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= p.n_frames) return;
    double* R = rec + (size_t)kMagRec * f;
    const int b = fb[f];
    if (b < 0) {
        for (int k = 0; k < kMagRec; ++k) R[k] = kNaN;
        return;
    }
    mag_frame_quantities(p, b, f, R);
}

// One lane per pair; the frame's quantities come from its record when
// there is one (rec), else the lane computes them (the same functions, so
// the results are the same bits).
__global__ __launch_bounds__(256) void k_pair_mag(const MagParams p, const int32_t* __restrict__ fb,
                                                 const double* __restrict__ rec) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= p.n_pairs) return;
    const int32_t f = p.pf[i], j = p.po[i];
    const int b = (f >= 0 && f < p.n_frames) ? fb[f] : -1;
    double v = kNaN, rh = kNaN, dl = kNaN, al = kNaN;
    if (b >= 0 && j >= 0 && j < p.n_obj) {
        const EphemArgs& E = p.eph;
        double R[kMagRec];
        if (rec) {
            const double2* q = reinterpret_cast<const double2*>(rec + (size_t)kMagRec * f);
#pragma unroll
            for (int k = 0; k < kMagRec / 2; ++k) {
                const double2 w = q[k];
                R[2 * k] = w.x;
                R[2 * k + 1] = w.y;
            }
        } else {
            mag_frame_quantities(p, b, f, R);
        }
        const double tf = R[0], tr = R[1];
        const double* st = p.x_epoch + 6 * ((int64_t)b * p.n_obj + j);
        const double r0[3] = {st[0] - R[5], st[1] - R[6], st[2] - R[7]};
        const double v0[3] = {st[3] - R[8], st[4] - R[9], st[5] - R[10]};
        SunCubic sun_e = sun_table(E.coef, 0, E.deg1, E.t_start, E.seg_days, E.inv_seg, 0, E.n_seg - 1);
        sun_e.t0 = tf;
        for (int k = 0; k < 3; ++k) {
            sun_e.s[k] = R[11 + k];
            sun_e.v[k] = R[14 + k];
            sun_e.a[k] = R[17 + k];
            sun_e.j[k] = R[20 + k];
        }
        const double o[3] = {R[2], R[3], R[4]};
        double d[3], tau, ve[3];
        // a hop that ends on the Kepler iteration cap gives NaN, as a pair
        // outside the ephemeris does
        const int kst = lighttime(sun_e, E.gm[0], p.smu, p.c_light, p.lt_tol, p.lt_iter, tr, r0, v0, tf, o, d,
                                  tau, ve, nullptr, p.kepler_iter);
        const double te = tf - tau;
        if (kst == 0 && te >= p.t_lo && te <= p.t_hi) {
            // heliocentric emission point r = (d + o) - S(te)
            double Se[3], Sde[3];
            sun_e.eval(te, Se, Sde);
            const double r[3] = {d[0] + o[0] - Se[0], d[1] + o[1] - Se[1], d[2] + o[2] - Se[2]};
            const double c = dot3(r, d);
            const double cx = r[1] * d[2] - r[2] * d[1];
            const double cy = r[2] * d[0] - r[0] * d[2];
            const double cz = r[0] * d[1] - r[1] * d[0];
            const double s = sqrt(cx * cx + cy * cy + cz * cz);
            rh = sqrt(dot3(r, r));
            dl = sqrt(dot3(d, d));
            // the phase angle itself only when the geometry is asked for
            if (p.geom) al = atan2(s, c);
            const double t = s / (rh * dl + c);
            // t^B as exp(B log t); t = 0 (zero phase) gives Phi = 1
            const double lt = log(t);
            const double phi1 = t > 0.0 ? exp(-kA1 * exp(kB1 * lt)) : 1.0;
            const double phi2 = t > 0.0 ? exp(-kA2 * exp(kB2 * lt)) : 1.0;
            const double G = p.g_slope[j];
            // 5 log10(r D) - 2.5 log10(Phi) with one logarithm
            const double rd = rh * dl;
            v = p.h_mag[j] + 2.5 * log10(rd * rd / ((1.0 - G) * phi1 + G * phi2));
        }
    }
    p.v_mag[i] = v;
    if (p.geom) {
        p.geom[3 * i] = rh;
        p.geom[3 * i + 1] = dl;
        p.geom[3 * i + 2] = al;
    }
}

}  // namespace

// Frame-to-batch map of the entry point that allocates nothing: a
// file-scope array in device memory (each GPU the library runs on holds
// its own copy until the process ends).  Host code never passes the
// array's name to a kernel: it is a host-side stand-in, not the device
// address, which comes from hipGetSymbolAddress once per device.
static __device__ __align__(256) int32_t scratch[kMagScratchFrames];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t mag_static_scratch(void** ptr) {
    *ptr = nullptr;
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    return hipSuccess;
}

static size_t mag_map_bytes(int64_t n_frames) {
    return ((size_t)std::max<int64_t>(n_frames, 1) * sizeof(int32_t) + 255) & ~(size_t)255;
}

size_t mag_workspace_bytes(int64_t n_frames) {
    const size_t rec = (size_t)std::max<int64_t>(n_frames, 1) * kMagRec * sizeof(double);
    return mag_map_bytes(n_frames) + ((rec + 255) & ~(size_t)255);
}

hipError_t launch_pair_mag(const MagParams& p, void* ws, bool frame_records, hipStream_t s) {
    int32_t* fb = static_cast<int32_t*>(ws);
    double* rec = frame_records ? reinterpret_cast<double*>(static_cast<char*>(ws) + mag_map_bytes(p.n_frames))
                                : nullptr;
    if (p.n_frames > 0) {
        const unsigned g = (unsigned)std::min<int64_t>((p.n_frames + 255) / 256, 4096);
        hipLaunchKernelGGL(k_mag_fill, dim3(g), dim3(256), 0, s, fb, p.n_frames);
        if (p.n_batch > 0)
            hipLaunchKernelGGL(k_mag_frame_batch, dim3((unsigned)((p.n_frames + 255) / 256)), dim3(256), 0, s, p,
                               fb);
        if (rec)
            hipLaunchKernelGGL(k_mag_frame_rec, dim3((unsigned)((p.n_frames + 255) / 256)), dim3(256), 0, s, p,
                               (const int32_t*)fb, rec);
    }
    if (p.n_pairs > 0)
        hipLaunchKernelGGL(k_pair_mag, dim3((unsigned)((p.n_pairs + 255) / 256)), dim3(256), 0, s, p,
                           (const int32_t*)fb, (const double*)rec);
    return hipGetLastError();
}

}  // namespace kete
