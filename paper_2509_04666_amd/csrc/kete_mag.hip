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

__global__ __launch_bounds__(256) void k_pair_mag(const MagParams p, const int32_t* __restrict__ fb) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= p.n_pairs) return;
    const int32_t f = p.pf[i], j = p.po[i];
    const int b = (f >= 0 && f < p.n_frames) ? fb[f] : -1;
    double v = kNaN, rh = kNaN, dl = kNaN, al = kNaN;
    if (b >= 0 && j >= 0 && j < p.n_obj) {
        const EphemArgs& E = p.eph;
        const double tr = p.t_ref[b], tf = p.ft[f];
        // the Sun at the epoch from the same chunked evaluation as its cubic
        // about the frame time: a few rounds of coefficient loads, not one
        // dependent load per coefficient
        const SunCubic s_ref = sun_cubic(E.coef, 0, E.deg1, tr, E.t_start, E.seg_days, E.inv_seg, 0, E.n_seg - 1);
        const double* st = p.x_epoch + 6 * ((int64_t)b * p.n_obj + j);
        const double r0[3] = {st[0] - s_ref.s[0], st[1] - s_ref.s[1], st[2] - s_ref.s[2]};
        const double v0[3] = {st[3] - s_ref.v[0], st[4] - s_ref.v[1], st[5] - s_ref.v[2]};
        double d[3], tau, ve[3];
        // a hop that ends on the Kepler iteration cap gives NaN, as a pair
        // outside the ephemeris does
        SunCubic sun_e = sun_cubic(E.coef, 0, E.deg1, tf, E.t_start, E.seg_days, E.inv_seg, 0, E.n_seg - 1);
        const int kst = lighttime(sun_e, E.gm[0], p.smu, p.c_light, p.lt_tol, p.lt_iter, tr, r0, v0, tf,
                                  p.fobs + 3 * (int64_t)f, d, tau, ve, nullptr, p.kepler_iter);
        const double te = tf - tau;
        if (kst == 0 && te >= p.t_lo && te <= p.t_hi) {
            // heliocentric emission point r = (d + o) - S(te)
            double Se[3], Sde[3];
            sun_e.eval(te, Se, Sde);
            const double* o = p.fobs + 3 * (int64_t)f;
            const double r[3] = {d[0] + o[0] - Se[0], d[1] + o[1] - Se[1], d[2] + o[2] - Se[2]};
            const double c = dot3(r, d);
            const double cx = r[1] * d[2] - r[2] * d[1];
            const double cy = r[2] * d[0] - r[0] * d[2];
            const double cz = r[0] * d[1] - r[1] * d[0];
            const double s = sqrt(cx * cx + cy * cy + cz * cz);
            rh = sqrt(dot3(r, r));
            dl = sqrt(dot3(d, d));
            al = atan2(s, c);
            const double t = s / (rh * dl + c);
            // t^B as exp(B log t); t = 0 (zero phase) gives Phi = 1
            const double lt = log(t);
            const double phi1 = t > 0.0 ? exp(-kA1 * exp(kB1 * lt)) : 1.0;
            const double phi2 = t > 0.0 ? exp(-kA2 * exp(kB2 * lt)) : 1.0;
            const double G = p.g_slope[j];
            v = p.h_mag[j] + 5.0 * log10(rh * dl) - 2.5 * log10((1.0 - G) * phi1 + G * phi2);
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

size_t mag_workspace_bytes(int64_t n_frames) {
    return ((size_t)std::max<int64_t>(n_frames, 1) * sizeof(int32_t) + 255) & ~(size_t)255;
}

hipError_t launch_pair_mag(const MagParams& p, void* ws, hipStream_t s) {
    int32_t* fb = static_cast<int32_t*>(ws);
    if (p.n_frames > 0) {
        const unsigned g = (unsigned)std::min<int64_t>((p.n_frames + 255) / 256, 4096);
        hipLaunchKernelGGL(k_mag_fill, dim3(g), dim3(256), 0, s, fb, p.n_frames);
        if (p.n_batch > 0)
            hipLaunchKernelGGL(k_mag_frame_batch, dim3((unsigned)((p.n_frames + 255) / 256)), dim3(256), 0, s, p,
                               fb);
    }
    if (p.n_pairs > 0)
        hipLaunchKernelGGL(k_pair_mag, dim3((unsigned)((p.n_pairs + 255) / 256)), dim3(256), 0, s, p,
                           (const int32_t*)fb);
    return hipGetLastError();
}

}  // namespace kete
