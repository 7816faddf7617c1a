// The paper's own binned visualisation (Sec. III-C and IV-B) on gfx950.
//
//   1. count matrix: each point adds 1 to the cell (ceil X, ceil Y) of the grid
//      (Eq. (5)-(6) with 0-based cells); points whose cell falls outside the
//      grid are dropped;
//   2. gap filling: consecutive points with equal labels, both inside, whose
//      cells are more than one cell apart are joined by the cells of the linear
//      interpolation of Eq. (12)-(13) (1-based coordinate rounded half up,
//      computed exactly in integers);
//   3. convolution of the counts with the separable table f(s, t) = k(s/Hx)
//      k(t/Hy), |s| <= a, |t| <= b (Eq. (7)-(8)), as a row pass and a column
//      pass, each through LDS tiles; the column pass applies the density scale
//      c^2 / (N hx hy), N the number of counted cells, read from the device.
//
// Counting uses integer atomics, so the count matrix and N do not depend on
// the order in which threads run.  The convolution sums run over taps in a
// fixed order: maps are bitwise reproducible.
#include "kde_tile.h"

#include <algorithm>

namespace kde {

namespace {

constexpr int kRowTileW = 256;  // row pass: outputs per row segment (one per thread)
constexpr int kRowTileH = 8;    // row pass: rows per workgroup
constexpr int kColTileW = 32;   // column pass: columns per workgroup
constexpr int kColTileH = 64;   // column pass: rows per workgroup (8 groups of 8)

// 0-based cell of a coordinate, or -1 outside [0, n) (NaN included).
__device__ __forceinline__ int cell_of(float X, int n) {
    const float c = ceilf(X);
    return (c >= 0.0f && c <= (float)(n - 1)) ? (int)c : -1;
}

__global__ __launch_bounds__(256) void zero_counts_kernel(uint32_t *counts, int64_t cells,
                                                          unsigned long long *total) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < cells) counts[i] = 0u;
    if (i == 0 && total != nullptr) *total = 0ull;
}

// One thread per point: its own cell, then the gap cells towards the next point.
// Consecutive points of a track often share a cell, so the point cells of a
// wave are combined first: one atomic per distinct cell, adding its
// multiplicity (integer sums, so the result is the same).
__global__ __launch_bounds__(256) void bin_points_kernel(const float2 *__restrict__ pts, int64_t n,
                                                         const int32_t *__restrict__ labels, int nx, int ny,
                                                         uint32_t *__restrict__ counts,
                                                         unsigned long long *__restrict__ total) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    unsigned mine = 0;
    int64_t key = -1;  // this point's cell, -1 if none
    int i = -1, j = -1;
    if (p < n) {
        const float2 v = pts[p];
        i = cell_of(v.x, nx);
        j = cell_of(v.y, ny);
        if (i >= 0 && j >= 0) key = (int64_t)j * nx + i;
    }
    uint64_t pending = __ballot(key >= 0);
    while (pending != 0ull) {  // uniform: every lane sees the same masks
        const int leader = __ffsll((unsigned long long)pending) - 1;
        const int64_t lkey = __shfl(key, leader);
        const uint64_t same = __ballot(key == lkey);
        if (lane == leader) atomicAdd(counts + lkey, (unsigned)__popcll(same));
        pending &= ~same;
    }
    if (key >= 0) {
        mine = 1;
        if (labels != nullptr && p + 1 < n && labels[p] == labels[p + 1]) {
            const float2 w = pts[p + 1];
            const int i2 = cell_of(w.x, nx), j2 = cell_of(w.y, ny);
            if (i2 >= 0 && j2 >= 0) {
                const int64_t di = i2 - i, dj = j2 - j;
                const int64_t cmax = max(di < 0 ? -di : di, dj < 0 ? -dj : dj);
                const int64_t bx = 2 * (int64_t)i * cmax + cmax, by = 2 * (int64_t)j * cmax + cmax;
                for (int64_t c = 1; c < cmax; ++c) {
                    // both numerators are positive: the cells lie between the end points
                    const int64_t ic = (bx + 2 * c * di) / (2 * cmax);
                    const int64_t jc = (by + 2 * c * dj) / (2 * cmax);
                    atomicAdd(counts + jc * nx + ic, 1u);
                }
                mine += (unsigned)(cmax > 1 ? cmax - 1 : 0);
            }
        }
    }
    // one 64-bit atomic per wave for the number of counted cells
    unsigned long long s = mine;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off);
    if (lane == 0 && s != 0ull) atomicAdd(total, s);
}

// One tap g(s / H) at integer offset s (g without the Table I constant).
template <int K>
__device__ __forceinline__ float tap(int s, float scale_arg, float H) {
    return tile::factor<K>((float)s, scale_arg, H);
}

// Row pass: tmp[j][i] = sum_{s=-a..a} g(s / Hx) counts[j][i - s].
template <int K>
__global__ __launch_bounds__(kRowTileW) void conv_rows_kernel(const uint32_t *__restrict__ counts, int nx, int ny,
                                                              int a, float Hx, float axs, float *__restrict__ tmp) {
    extern __shared__ float lds[];
    float *w = lds;                    // [2a + 1] taps
    float *row = lds + (2 * a + 1);    // [kRowTileW + 2a] counts of one row segment
    const int tid = threadIdx.x;
    const int i0 = blockIdx.x * kRowTileW, j0 = blockIdx.y * kRowTileH;
    for (int s = tid; s <= 2 * a; s += kRowTileW) w[s] = tap<K>(s - a, axs, Hx);
    const int span = kRowTileW + 2 * a;
    for (int r = 0; r < kRowTileH; ++r) {
        const int j = j0 + r;
        if (j >= ny) break;  // uniform across the workgroup
        __syncthreads();     // taps written / previous row consumed
        const uint32_t *src = counts + (int64_t)j * nx;
        for (int k = tid; k < span; k += kRowTileW) {
            const int i = i0 - a + k;
            row[k] = (i >= 0 && i < nx) ? (float)src[i] : 0.0f;
        }
        __syncthreads();
        const int i = i0 + tid;
        if (i < nx) {
            // output i reads counts[i - s], s = -a..a, i.e. row[tid + a - s]
            float acc = 0.0f;
            for (int s = -a; s <= a; ++s) acc = fmaf(w[s + a], row[tid + a - s], acc);
            tmp[(int64_t)j * nx + i] = acc;
        }
    }
}

// Column pass: out[j][i] = scale * sum_{t=-b..b} g(t / Hy) tmp[j - t][i].
template <int K>
__global__ __launch_bounds__(256) void conv_cols_kernel(const float *__restrict__ tmp, int nx, int ny, int b,
                                                        float Hy, float ays, double c2_over_hxhy, int raw,
                                                        const unsigned long long *__restrict__ total,
                                                        float *__restrict__ out) {
    extern __shared__ float lds[];
    float *w = lds;                          // [2b + 1]
    float *tile_ = lds + (2 * b + 1);        // [kColTileH + 2b][kColTileW]
    const int tid = threadIdx.x;
    const int i0 = blockIdx.x * kColTileW, j0 = blockIdx.y * kColTileH;
    for (int t = tid; t <= 2 * b; t += 256) w[t] = tap<K>(t - b, ays, Hy);
    const int rows = kColTileH + 2 * b;
    for (int k = tid; k < rows * kColTileW; k += 256) {
        const int rr = k / kColTileW, cc = k % kColTileW;
        const int j = j0 - b + rr, i = i0 + cc;
        tile_[k] = (j >= 0 && j < ny && i < nx) ? tmp[(int64_t)j * nx + i] : 0.0f;
    }
    __syncthreads();
    float scale;
    if (raw) {
        scale = (float)c2_over_hxhy;
    } else {
        const unsigned long long N = *total;
        scale = N == 0ull ? 0.0f : (float)(c2_over_hxhy / (double)N);
    }
    constexpr int kGroups = 256 / kColTileW, kRowsPer = kColTileH / kGroups;
    const int cc = tid % kColTileW, rg = tid / kColTileW;
    const int i = i0 + cc;
    if (i >= nx) return;
    for (int q = 0; q < kRowsPer; ++q) {
        const int rr = rg * kRowsPer + q, j = j0 + rr;
        if (j >= ny) break;
        // output row rr reads tmp rows rr + b - t, t = -b..b
        float acc = 0.0f;
        for (int t = -b; t <= b; ++t) acc = fmaf(w[t + b], tile_[(rr + b - t) * kColTileW + cc], acc);
        out[(int64_t)j * nx + i] = acc * scale;
    }
}

template <int K>
hipError_t launch_conv_k(const BinnedConvArgs &c, float *tmp, hipStream_t s) {
    const float axs = arg_scale(K, c.Hx), ays = arg_scale(K, c.Hy);
    dim3 g1((c.nx + kRowTileW - 1) / kRowTileW, (c.ny + kRowTileH - 1) / kRowTileH);
    const size_t lds1 = (size_t)(2 * c.a + 1 + kRowTileW + 2 * c.a) * sizeof(float);
    main_kernel_begin(s);
    hipLaunchKernelGGL((conv_rows_kernel<K>), g1, dim3(kRowTileW), lds1, s, c.counts, c.nx, c.ny, c.a, c.Hx, axs,
                       tmp);
    dim3 g2((c.nx + kColTileW - 1) / kColTileW, (c.ny + kColTileH - 1) / kColTileH);
    const size_t lds2 = (size_t)(2 * c.b + 1 + (kColTileH + 2 * c.b) * kColTileW) * sizeof(float);
    hipLaunchKernelGGL((conv_cols_kernel<K>), g2, dim3(256), lds2, s, tmp, c.nx, c.ny, c.b, c.Hy, ays,
                       c.c2_over_hxhy, c.raw ? 1 : 0, c.total, c.out);
    main_kernel_end(s);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_bin_counts(const float2 *pts, int64_t n, const int32_t *labels, int nx, int ny, uint32_t *counts,
                             unsigned long long *total, hipStream_t s) {
    const int64_t cells = (int64_t)nx * ny;
    hipLaunchKernelGGL(zero_counts_kernel, dim3((unsigned)((cells + 255) / 256)), dim3(256), 0, s, counts, cells,
                       total);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || n == 0) return e;
    hipLaunchKernelGGL(bin_points_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, pts, n, labels, nx, ny,
                       counts, total);
    return hipGetLastError();
}

size_t conv_workspace_bytes(int nx, int ny) { return (size_t)nx * ny * sizeof(float); }

hipError_t launch_conv_counts(const BinnedConvArgs &c, void *ws, hipStream_t s) {
    if (c.a < 0 || c.b < 0 || c.a > kMaxTapRadius || c.b > kMaxTapRadius) return hipErrorInvalidValue;
    float *tmp = static_cast<float *>(ws);
    switch (c.kernel_id) {
    case kUniform: return launch_conv_k<kUniform>(c, tmp, s);
    case kTriangular: return launch_conv_k<kTriangular>(c, tmp, s);
    case kEpanechnikov: return launch_conv_k<kEpanechnikov>(c, tmp, s);
    case kQuartic: return launch_conv_k<kQuartic>(c, tmp, s);
    case kTriweight: return launch_conv_k<kTriweight>(c, tmp, s);
    case kTricube: return launch_conv_k<kTricube>(c, tmp, s);
    case kGaussian: return launch_conv_k<kGaussian>(c, tmp, s);
    case kCosine: return launch_conv_k<kCosine>(c, tmp, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace kde
