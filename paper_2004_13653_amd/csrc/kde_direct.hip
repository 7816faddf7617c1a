// FP32 direct evaluation of the KDE heat map on gfx950.
//
// S[j][i] = sum_p g((i - X_p) a_x) g((j - Y_p) a_y) for the Table I product
// kernels (Sec. III-C, Eq. (7)-(8)), in grid units, FP32 arithmetic, every pair
// (compact kernels: pairs with |i - X_p| > Hx or |j - Y_p| > Hy contribute 0 and
// whole point tiles outside a workgroup's reach are skipped).
//
// Layout.  A workgroup of 256 threads (16 x 16) owns a TW x TH pixel tile, each
// thread an R x C register block (R = C = 2, 4 or 8, chosen per map) of R
// consecutive rows and C consecutive columns,
// so the 16 threads of a row of the thread grid store 16*C contiguous floats.
// Points stream through LDS 256 at a time and are read back as wave-wide
// broadcasts.  Per point a thread evaluates C + R one-dimensional factors and
// does R*C FMAs: the product form of Table I shares each factor across a row or
// column of the block.
//
// Accumulation.  Each LDS tile of points is summed into a fresh register block
// that is then added to the running total, so no FP32 sum runs over more than
// 256 terms before joining a partial of similar size.  Large maps split the
// points across workgroups ("splits"); a second kernel adds the per-split
// partial maps in split order and applies the density scale.  The order of every
// sum is fixed by the launch shape, so results are bitwise reproducible.
#include "kde_tile.h"

#include <algorithm>
#include <cmath>

namespace kde {

namespace {

using tile::kPointTile;
using tile::kThreads;

struct DirectLaunch {
    const float2 *pts;
    int64_t n;
    int64_t per_split;  // points per split (multiple of kPointTile)
    float Hx, Hy, ax, ay;
    int nx, ny, tiles_x;
    float *dst;         // final map (splits == 1) or partials [splits][ny][nx]
    float scale;        // applied only when writing the final map
    int64_t plane;      // nx * ny
};

// One workgroup: pixel tile blockIdx.x, point split blockIdx.y.
template <int K, int RC, bool kRuns>
__global__ __launch_bounds__(tile::kThreads) void direct_fp32_kernel(DirectLaunch p) {
    using S = tile::Shape<K, RC>;
    __shared__ float2 sp[tile::kPointTile];
    __shared__ int swave[tile::kThreads / 64];
    const int tid = threadIdx.x;
    const int tx = blockIdx.x % p.tiles_x, ty = blockIdx.x / p.tiles_x;
    const int x0 = tx * S::TW, y0 = ty * S::TH;
    const int ib = x0 + (tid & 15) * S::C, jb = y0 + (tid >> 4) * S::R;
    const int64_t beg = (int64_t)blockIdx.y * p.per_split;
    const int64_t end = min(p.n, beg + p.per_split);
    float tot[S::R][S::C];
    tile::tile_sums<K, S::R, S::C, S::kCull, kRuns>(p.pts, beg, end, p.Hx, p.Hy, p.ax, p.ay, ib, jb, (float)x0,
                                                    (float)(min(x0 + S::TW, p.nx) - 1), (float)y0,
                                                    (float)(min(y0 + S::TH, p.ny) - 1), sp, swave, tot);
    if constexpr (kRuns) tile::apply_run_q<S::R, S::C>(tot, p.ax, p.ay);
    float *dst = p.dst + (int64_t)blockIdx.y * p.plane;
    tile::store_block<S::R, S::C>(tot, dst, p.nx, p.ny, ib, jb, gridDim.y == 1 ? p.scale : 1.0f);
}

// out[i] = scale * sum_s part[s][i], s in order.
__global__ __launch_bounds__(256) void reduce_splits_kernel(const float *__restrict__ part, int splits,
                                                            int64_t plane, float scale,
                                                            float *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= plane) return;
    float s = 0.0f;
    for (int k = 0; k < splits; ++k) s += part[(int64_t)k * plane + i];
    out[i] = s * scale;
}

__global__ __launch_bounds__(256) void fill_zero_kernel(float *out, int64_t count) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) out[i] = 0.0f;
}

struct Plan {
    int tiles_x, tiles;
    int splits;
    int64_t per_split;
};

Plan plan_for(const MapArgs &a) {
    const int TW = 16 * a.rc, TH = 16 * a.rc;
    Plan pl;
    pl.tiles_x = (a.nx + TW - 1) / TW;
    pl.tiles = pl.tiles_x * ((a.ny + TH - 1) / TH);
    // Aim for about 4 workgroups per CU (256 CUs) with at least 2048 points each.
    const int64_t want = std::max<int64_t>(1, (1024 + pl.tiles - 1) / pl.tiles);
    const int64_t by_points = std::max<int64_t>(1, a.n / 2048);
    int64_t splits = std::min<int64_t>({want, by_points, 64});
    int64_t per = (a.n + splits - 1) / splits;
    per = (per + kPointTile - 1) / kPointTile * kPointTile;
    splits = (a.n + per - 1) / per;
    pl.splits = (int)std::max<int64_t>(1, splits);
    pl.per_split = std::max<int64_t>(per, kPointTile);
    return pl;
}

template <int K, int RC>
hipError_t launch_kr(const MapArgs &a, const Plan &pl, float *dst, hipStream_t stream) {
    DirectLaunch p{a.pts, a.n, pl.per_split, a.Hx, a.Hy, a.ax, a.ay, a.nx, a.ny, pl.tiles_x, dst, a.scale,
                   (int64_t)a.nx * a.ny};
    dim3 grid(pl.tiles, pl.splits);
    main_kernel_begin(stream);
    constexpr bool kGauss = K == kGaussian || K == kGaussTrunc;
    if (kGauss && a.ax <= kMaxRunScale && a.ay <= kMaxRunScale)
        hipLaunchKernelGGL((direct_fp32_kernel<K, RC, kGauss>), grid, dim3(kThreads), 0, stream, p);
    else
        hipLaunchKernelGGL((direct_fp32_kernel<K, RC, false>), grid, dim3(kThreads), 0, stream, p);
    main_kernel_end(stream);
    return hipGetLastError();
}

template <int K>
hipError_t launch_k(const MapArgs &a, const Plan &pl, float *dst, hipStream_t stream) {
    switch (a.rc) {
    case 2: return launch_kr<K, 2>(a, pl, dst, stream);
    case 4: return launch_kr<K, 4>(a, pl, dst, stream);
    case 8: return launch_kr<K, 8>(a, pl, dst, stream);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

double kernel_norm(int kernel_id) {
    const double pi = 3.14159265358979323846;
    switch (kernel_id) {
    case kUniform: return 0.5;
    case kTriangular: return 1.0;
    case kEpanechnikov: return 0.75;
    case kQuartic: return 15.0 / 16.0;
    case kTriweight: return 35.0 / 32.0;
    case kTricube: return 70.0 / 81.0;
    case kGaussian: return 1.0 / std::sqrt(2.0 * pi);
    case kCosine: return pi / 4.0;
    case kGaussTrunc: return 1.0 / std::sqrt(2.0 * pi);
    default: return 0.0;
    }
}

float arg_scale(int kernel_id, float H) {
    if (kernel_id == kGaussian) return (float)(std::sqrt(0.5 / std::log(2.0)) / (double)H);
    if (kernel_id == kGaussTrunc) return arg_scale(kGaussian, H / kTruncSigmas);  // H: the support
    return (float)(1.0 / (double)H);
}

size_t direct_workspace_bytes(const MapArgs &a) {
    if (!valid_rc(a.rc)) return 0;
    if (binning_applies(a)) return binned_workspace_bytes(a);
    const Plan pl = plan_for(a);
    return pl.splits > 1 ? (size_t)pl.splits * a.nx * a.ny * sizeof(float) : 0;
}

hipError_t launch_fill_zero(float *out, int64_t count, hipStream_t stream) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_zero_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, stream, out, count);
    return hipGetLastError();
}

hipError_t launch_direct(const MapArgs &a, void *ws, hipStream_t stream) {
    if (!valid_rc(a.rc)) return hipErrorInvalidValue;
    if (binning_applies(a)) return launch_binned(a, ws, stream);
    const Plan pl = plan_for(a);
    float *dst = pl.splits > 1 ? static_cast<float *>(ws) : a.out;
    hipError_t e;
    switch (a.kernel_id) {
    case kUniform: e = launch_k<kUniform>(a, pl, dst, stream); break;
    case kTriangular: e = launch_k<kTriangular>(a, pl, dst, stream); break;
    case kEpanechnikov: e = launch_k<kEpanechnikov>(a, pl, dst, stream); break;
    case kQuartic: e = launch_k<kQuartic>(a, pl, dst, stream); break;
    case kTriweight: e = launch_k<kTriweight>(a, pl, dst, stream); break;
    case kTricube: e = launch_k<kTricube>(a, pl, dst, stream); break;
    case kGaussian: e = launch_k<kGaussian>(a, pl, dst, stream); break;
    case kCosine: e = launch_k<kCosine>(a, pl, dst, stream); break;
    case kGaussTrunc: e = launch_k<kGaussTrunc>(a, pl, dst, stream); break;
    default: return hipErrorInvalidValue;
    }
    if (e != hipSuccess || pl.splits == 1) return e;
    return launch_reduce_splits(static_cast<const float *>(ws), pl.splits, (int64_t)a.nx * a.ny, a.scale, a.out,
                                stream);
}

hipError_t launch_reduce_splits(const float *part, int splits, int64_t plane, float scale, float *out,
                                hipStream_t stream) {
    hipLaunchKernelGGL(reduce_splits_kernel, dim3((unsigned)((plane + 255) / 256)), dim3(256), 0, stream, part,
                       splits, plane, scale, out);
    return hipGetLastError();
}

}  // namespace kde
