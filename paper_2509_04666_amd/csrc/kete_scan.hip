// Exclusive prefix sums of int32 counts (three passes: tile sums, a
// single-block scan of the tile sums, tile scans with their offsets).
#include "kete_internal.hpp"

namespace kete {
namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 4;
constexpr int kTile = kScanThreads * kScanItems;

// Inclusive scan of one value per thread over a 256-thread block.
__device__ __forceinline__ int block_inclusive(int v, int* sh) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        int u = __shfl_up(v, off, 64);
        if (lane >= off) v += u;
    }
    if (lane == 63) sh[wid] = v;
    __syncthreads();
    int add = 0;
    for (int w = 0; w < wid; ++w) add += sh[w];
    __syncthreads();
    return v + add;
}

__global__ __launch_bounds__(kScanThreads) void k_tile_sums(const int32_t* __restrict__ in, int64_t n,
                                                          int32_t* __restrict__ part) {
    __shared__ int sh[4];
    const int64_t base = (int64_t)blockIdx.x * kTile + threadIdx.x * kScanItems;
    int s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) if (base + k < n) s += in[base + k];
    s = block_inclusive(s, sh);
    if (threadIdx.x == kScanThreads - 1) part[blockIdx.x] = s;
}

// One block scans all tile sums (exclusive), carrying a running total.
__global__ __launch_bounds__(kScanThreads) void k_scan_parts(int32_t* __restrict__ part, int64_t np,
                                                           int32_t* __restrict__ total) {
    __shared__ int sh[4];
    __shared__ int carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t base = 0; base < np; base += kScanThreads) {
        const int64_t i = base + threadIdx.x;
        const int v = i < np ? part[i] : 0;
        const int inc = block_inclusive(v, sh);
        const int c = carry;
        if (i < np) part[i] = c + inc - v;
        __syncthreads();
        if (threadIdx.x == kScanThreads - 1) carry = c + inc;
        __syncthreads();
    }
    if (threadIdx.x == 0) *total = carry;
}

__global__ __launch_bounds__(kScanThreads) void k_tile_scan(const int32_t* __restrict__ in, int64_t n,
                                                          const int32_t* __restrict__ part,
                                                          int32_t* __restrict__ out) {
    __shared__ int sh[4];
    const int64_t base = (int64_t)blockIdx.x * kTile + threadIdx.x * kScanItems;
    int v[kScanItems];
    int s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) { v[k] = (base + k < n) ? in[base + k] : 0; s += v[k]; }
    const int inc = block_inclusive(s, sh);
    int run = part[blockIdx.x] + inc - s;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < n) out[base + k] = run;
        run += v[k];
    }
}

}  // namespace

size_t scan_scratch_bytes(int64_t n) {
    const int64_t np = (n + kTile - 1) / kTile;
    return (size_t)(np + 64) * sizeof(int32_t);
}

// out[0..n) = exclusive prefix sums of in, out[n] = total.  `in` may alias `out`.
hipError_t exclusive_scan_i32(const int32_t* in, int32_t* out, int64_t n, void* scratch, hipStream_t s) {
    int32_t* part = (int32_t*)scratch;
    const int64_t np = (n + kTile - 1) / kTile;
    if (n == 0) {
        hipLaunchKernelGGL(k_scan_parts, dim3(1), dim3(kScanThreads), 0, s, part, (int64_t)0, out);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_tile_sums, dim3((unsigned)np), dim3(kScanThreads), 0, s, in, n, part);
    hipLaunchKernelGGL(k_scan_parts, dim3(1), dim3(kScanThreads), 0, s, part, np, out + n);
    hipLaunchKernelGGL(k_tile_scan, dim3((unsigned)np), dim3(kScanThreads), 0, s, in, n, (const int32_t*)part, out);
    return hipGetLastError();
}

}  // namespace kete
