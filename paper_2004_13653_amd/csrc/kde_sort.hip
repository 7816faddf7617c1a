// Spatial sort of points (used by the support-culled LSCV pair sums).
//
// Every point gets the Morton (Z-order) code of the square cell it falls in,
// cells of side `cell` grid units over [0, 1024 cell)^2 (coordinates outside
// are clamped to the border cells), and the points are reordered by that code
// with a stable least-significant-digit radix sort, 10 bits per pass:
//
//   1. key:     code per point, and the point copied next to it;
//   2. count:   one wave per block of 1024 consecutive items counts the digits
//               of its items in LDS (integer atomics: order-independent) and
//               stores the 1024 counts digit-major, hist[digit][block];
//   3. scan:    exclusive prefix sum of hist (the work-efficient scan of the
//               support binning) gives each (digit, block) its first slot;
//   4. scatter: the wave walks its block in item order, 64 items per step;
//               lanes holding the same digit find each other with one ballot
//               per digit bit, take consecutive slots in lane order, and the
//               lowest of them advances the digit's running slot in LDS.
//
// Equal codes keep their input order, so the result is a fixed function of the
// input: consecutive 256-point blocks of it cover small regions, and the
// pair sums over blocks are the same on every run.
#include "kde_internal.h"

#include <algorithm>

namespace kde {

namespace {

constexpr int kDigitBits = 10;
constexpr int kBuckets = 1 << kDigitBits;
constexpr int kItems = 16;                 // items per lane and block
constexpr int kSortBlock = 64 * kItems;    // items per wave block
constexpr int kCellsPerSide = 1024;        // 10 bits per axis, 20-bit codes
constexpr int kPasses = 2;

__device__ __forceinline__ unsigned spread10(unsigned v) {
    v &= 0x3ffu;
    v = (v | (v << 8)) & 0x00ff00ffu;
    v = (v | (v << 4)) & 0x0f0f0f0fu;
    v = (v | (v << 2)) & 0x33333333u;
    v = (v | (v << 1)) & 0x55555555u;
    return v;
}

__device__ __forceinline__ unsigned cell_of(float x, float inv_cell) {
    const float c = floorf(x * inv_cell);  // NaN -> 0 below
    return (unsigned)fminf(fmaxf(c, 0.0f), (float)(kCellsPerSide - 1));
}

__global__ __launch_bounds__(256) void morton_key_kernel(const float2 *__restrict__ pts, int64_t n, float inv_cell,
                                                         unsigned *__restrict__ keys, float2 *__restrict__ vals) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float2 p = pts[i];
    keys[i] = spread10(cell_of(p.x, inv_cell)) | (spread10(cell_of(p.y, inv_cell)) << 1);
    vals[i] = p;
}

struct SortPass {
    const unsigned *kin;
    const float2 *vin;
    unsigned *kout;
    float2 *vout;
    int64_t n, blocks;
    int shift;
    unsigned *hist;  // [kBuckets][blocks]
};

__global__ __launch_bounds__(64) void radix_count_kernel(SortPass p) {
    __shared__ unsigned h[kBuckets];
    const int lane = threadIdx.x;
    const int64_t b = blockIdx.x;
    for (int d = lane; d < kBuckets; d += 64) h[d] = 0u;
    __syncthreads();
    const int64_t base = b * kSortBlock;
#pragma unroll 4
    for (int r = 0; r < kItems; ++r) {
        const int64_t i = base + r * 64 + lane;
        if (i < p.n) atomicAdd(&h[(p.kin[i] >> p.shift) & (kBuckets - 1)], 1u);
    }
    __syncthreads();
    for (int d = lane; d < kBuckets; d += 64) p.hist[(int64_t)d * p.blocks + b] = h[d];
}

__global__ __launch_bounds__(64) void radix_scatter_kernel(SortPass p) {
    __shared__ unsigned run[kBuckets];
    const int lane = threadIdx.x;
    const int64_t b = blockIdx.x;
    for (int d = lane; d < kBuckets; d += 64) run[d] = p.hist[(int64_t)d * p.blocks + b];
    __syncthreads();
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int64_t base = b * kSortBlock;
    for (int r = 0; r < kItems; ++r) {
        const int64_t i = base + r * 64 + lane;
        const bool valid = i < p.n;
        const unsigned key = valid ? p.kin[i] : 0u;
        const unsigned d = (key >> p.shift) & (kBuckets - 1);
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < kDigitBits; ++bit) {
            const uint64_t set = __ballot((d >> bit) & 1u);
            peers &= ((d >> bit) & 1u) ? set : ~set;
        }
        const unsigned first = run[d];  // every lane reads before the leaders write
        __syncthreads();
        if (valid) {
            const unsigned pos = first + (unsigned)__popcll(peers & below);
            p.kout[pos] = key;
            p.vout[pos] = p.vin[i];
            if ((peers & below) == 0ull) run[d] = first + (unsigned)__popcll(peers);  // lowest lane of the group
        }
        __syncthreads();
    }
}

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

struct SortPlan {
    int64_t blocks, hist_len;
    size_t keys_bytes, vals_bytes, hist_bytes, totals_bytes;
};

SortPlan sort_plan(int64_t n) {
    SortPlan pl;
    pl.blocks = (n + kSortBlock - 1) / kSortBlock;
    pl.hist_len = pl.blocks * kBuckets;
    pl.keys_bytes = align256((size_t)n * sizeof(unsigned));
    pl.vals_bytes = align256((size_t)n * sizeof(float2));
    pl.hist_bytes = align256((size_t)pl.hist_len * sizeof(unsigned));
    pl.totals_bytes = align256(scan_u32_totals_bytes(pl.hist_len));
    return pl;
}

}  // namespace

size_t spatial_sort_bytes(int64_t n) {
    const SortPlan pl = sort_plan(n);
    return 2 * pl.keys_bytes + pl.vals_bytes + pl.hist_bytes + pl.totals_bytes;
}

hipError_t launch_spatial_sort(const float2 *pts, int64_t n, float cell, void *ws, float2 *out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const SortPlan pl = sort_plan(n);
    char *w = static_cast<char *>(ws);
    unsigned *k0 = reinterpret_cast<unsigned *>(w);
    unsigned *k1 = reinterpret_cast<unsigned *>(w + pl.keys_bytes);
    float2 *v0 = reinterpret_cast<float2 *>(w + 2 * pl.keys_bytes);
    unsigned *hist = reinterpret_cast<unsigned *>(w + 2 * pl.keys_bytes + pl.vals_bytes);
    unsigned *totals = reinterpret_cast<unsigned *>(w + 2 * pl.keys_bytes + pl.vals_bytes + pl.hist_bytes);
    // Keys and points into (k0, out); pass 1 to (k1, v0); pass 2 back to (k0, out).
    hipLaunchKernelGGL(morton_key_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, pts, n,
                       1.0f / cell, k0, out);
    hipError_t e = hipGetLastError();
    unsigned *kin = k0, *kout = k1;
    float2 *vin = out, *vout = v0;
    for (int pass = 0; pass < kPasses && e == hipSuccess; ++pass) {
        SortPass p{kin, vin, kout, vout, n, pl.blocks, pass * kDigitBits, hist};
        hipLaunchKernelGGL(radix_count_kernel, dim3((unsigned)pl.blocks), dim3(64), 0, s, p);
        e = hipGetLastError();
        if (e == hipSuccess) e = launch_scan_u32(hist, pl.hist_len, totals, s);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(radix_scatter_kernel, dim3((unsigned)pl.blocks), dim3(64), 0, s, p);
            e = hipGetLastError();
        }
        std::swap(kin, kout);
        std::swap(vin, vout);
    }
    return e;
}

float spatial_sort_cell(float Hx, float Hy, int nx, int ny) {
    return std::max(std::max(Hx, Hy), (float)std::max(nx, ny) / (float)kCellsPerSide);
}

}  // namespace kde
