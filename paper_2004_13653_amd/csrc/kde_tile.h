// Device building blocks of the FP32 direct evaluation, shared by the single-map
// kernel (kde_direct.hip) and the batched persistent kernel (kde_batched.hip).
#pragma once

#include "kde_internal.h"

namespace kde {
namespace tile {

constexpr int kThreads = 256;    // threads per workgroup (16 x 16)
constexpr int kPointTile = 256;  // points staged in LDS per step

// g(d) for grid-unit difference d = node - point.  a is arg_scale(kernel, H).
template <int K>
__device__ __forceinline__ float factor(float d, float a, float H) {
    if constexpr (K == kGaussian) {
        const float t = d * a;
        return __builtin_amdgcn_exp2f(-t * t);
    } else if constexpr (K == kGaussTrunc) {  // H is the support half-width here
        const float t = d * a;
        return fabsf(d) <= H ? __builtin_amdgcn_exp2f(-t * t) : 0.0f;
    } else {
        const float u = fminf(fabsf(d) * a, 1.0f);  // |u|, clamped against rounding past 1
        float v;
        if constexpr (K == kUniform) {
            v = 1.0f;
        } else if constexpr (K == kTriangular) {
            v = 1.0f - u;
        } else if constexpr (K == kEpanechnikov) {
            v = 1.0f - u * u;
        } else if constexpr (K == kQuartic) {
            const float w = 1.0f - u * u;
            v = w * w;
        } else if constexpr (K == kTriweight) {
            const float w = 1.0f - u * u;
            v = w * w * w;
        } else if constexpr (K == kTricube) {
            const float w = 1.0f - u * u * u;
            v = w * w * w;
        } else {  // cosine: v_cos_f32 takes revolutions, cos(pi u / 2) = cos(2 pi (u / 4))
            v = __builtin_amdgcn_cosf(u * 0.25f);
        }
        return fabsf(d) <= H ? v : 0.0f;
    }
}

// Gaussian run of N consecutive nodes c0 .. c0+N-1 against one point: with the
// centre node c = c0 + (N-1)/2, t = (c - X) a and rho_r = r - (N-1)/2,
//     g(c0 + r) = exp2(-(t + rho_r a)^2) = P_r q_r,
//     P_r = exp2(-t^2 - 2 t a rho_r) = P_0 B^r,  B = exp2(-2 a t),  q_r = exp2(-(rho_r a)^2).
// v receives P_0 .. P_{N-1}: two exp2 and N-1 multiplies instead of N exp2.
// q_r depends only on r, so it multiplies the finished sums (run_q).  With
// a <= kMaxRunScale, P_r <= g / q_r <= 2^7.9 g; a P_0 that underflows means
// every factor of the run is negligible, and B is clamped to stay finite, so a
// run never produces NaN or turns a zero into a non-zero.
template <int N>
__device__ __forceinline__ void gauss_run(float t, float a, float (&v)[N]) {
    const float span = (float)(N - 1) * a;
    v[0] = __builtin_amdgcn_exp2f(t * (span - t));  // -t^2 + (N-1) a t
    const float ratio = __builtin_amdgcn_exp2f(fminf(-2.0f * a * t, 126.0f));
#pragma unroll
    for (int r = 1; r < N; ++r) v[r] = v[r - 1] * ratio;
}

template <int N>
__device__ __forceinline__ void run_q(float a, float (&q)[N]) {
#pragma unroll
    for (int r = 0; r < N; ++r) {
        const float rho = ((float)r - 0.5f * (float)(N - 1)) * a;
        q[r] = __builtin_amdgcn_exp2f(-rho * rho);
    }
}

// tot[r][c] *= q_y[r] q_x[c]: the position factors of Gaussian runs.
template <int R, int C>
__device__ __forceinline__ void apply_run_q(float (&tot)[R][C], float ax, float ay) {
    float qx[C], qy[R];
    run_q<C>(ax, qx);
    run_q<R>(ay, qy);
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int c = 0; c < C; ++c) tot[r][c] *= qy[r] * qx[c];
}

template <int R, int C>
__device__ __forceinline__ void store_block(float (&v)[R][C], float *dst, int nx, int ny, int ib, int jb,
                                            float scale) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int j = jb + r;
        if (j >= ny) break;
        float *row = dst + (int64_t)j * nx;
        if ((nx & 3) == 0 && ib + C <= nx && (C % 4) == 0) {
#pragma unroll
            for (int c = 0; c < C; c += 4) {
                float4 w = make_float4(v[r][c] * scale, v[r][c + 1] * scale, v[r][c + 2] * scale,
                                       v[r][c + 3] * scale);
                *reinterpret_cast<float4 *>(row + ib + c) = w;
            }
        } else {
#pragma unroll
            for (int c = 0; c < C; ++c)
                if (ib + c < nx) row[ib + c] = v[r][c] * scale;
        }
    }
}

// Adds the points [base, end) (at most kPointTile, one LDS tile) to tot, for
// the R x C register block at (jb, ib) of a 256-thread workgroup (16 x 16
// threads); tile reach x0..x1, y0..y1 (nodes) for culling.  The tile's points
// are summed into a fresh block before joining the total.  Every thread calls
// it (it contains workgroup barriers).
// sp: LDS [kPointTile] float2; swave: LDS [kThreads / 64] int.
// kRuns (Gaussian, truncated Gaussian): factors as Gaussian runs (the truncated
// one then masked to its support); the caller applies apply_run_q.
template <int K, int R, int C, bool kCull, bool kRuns = false>
__device__ __forceinline__ void chunk_sums(const float2 *__restrict__ pts, int64_t base, int64_t end, float Hx,
                                           float Hy, float ax, float ay, float fib, float fjb, float bx0, float bx1,
                                           float by0, float by1, float2 *sp, int *swave, float (&tot)[R][C]) {
    const int tid = threadIdx.x;
    const int64_t q = base + tid;
    float2 v = make_float2(0.0f, 0.0f);
    if (q < end) v = pts[q];
    int cnt;
    __syncthreads();  // previous tile fully consumed
    if constexpr (kCull) {
        const bool keep = q < end && v.x + Hx >= bx0 && v.x - Hx <= bx1 && v.y + Hy >= by0 && v.y - Hy <= by1;
        const uint64_t m = __ballot(keep);
        const int lane = tid & 63, w = tid >> 6;
        const int before = __popcll(m & ((1ull << lane) - 1ull));
        if (lane == 0) swave[w] = __popcll(m);
        __syncthreads();
        int off = 0;
        cnt = 0;
#pragma unroll
        for (int k = 0; k < kThreads / 64; ++k) {
            off += (k < w) ? swave[k] : 0;
            cnt += swave[k];
        }
        if (keep) sp[off + before] = v;  // survivors keep their index order
    } else {
        sp[tid] = v;
        cnt = (int)min((int64_t)kPointTile, end - base);
    }
    __syncthreads();
    if (cnt == 0) return;

    float acc[R][C];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int c = 0; c < C; ++c) acc[r][c] = 0.0f;

    for (int k = 0; k < cnt; ++k) {
        const float2 pt = sp[k];
        float kx[C], ky[R];
        if constexpr (kRuns) {
            // run centres: half-integer nodes, so (centre - X) is exact like dx0 below
            gauss_run<C>((fib + 0.5f * (float)(C - 1) - pt.x) * ax, ax, kx);
            gauss_run<R>((fjb + 0.5f * (float)(R - 1) - pt.y) * ay, ay, ky);
            if constexpr (K == kGaussTrunc) {  // the support test of factor<kGaussTrunc> (q_r > 0 keeps zeros)
                const float dx0 = fib - pt.x, dy0 = fjb - pt.y;
#pragma unroll
                for (int c = 0; c < C; ++c) kx[c] = fabsf(dx0 + (float)c) <= Hx ? kx[c] : 0.0f;
#pragma unroll
                for (int r = 0; r < R; ++r) ky[r] = fabsf(dy0 + (float)r) <= Hy ? ky[r] : 0.0f;
            }
        } else {
            const float dx0 = fib - pt.x, dy0 = fjb - pt.y;
#pragma unroll
            for (int c = 0; c < C; ++c) kx[c] = factor<K>(dx0 + (float)c, ax, Hx);
#pragma unroll
            for (int r = 0; r < R; ++r) ky[r] = factor<K>(dy0 + (float)r, ay, Hy);
        }
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int c = 0; c < C; ++c) acc[r][c] = fmaf(ky[r], kx[c], acc[r][c]);
    }
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int c = 0; c < C; ++c) tot[r][c] += acc[r][c];
}

// Raw sums of one pixel tile over points [beg, end), kPointTile at a time (see
// chunk_sums).
template <int K, int R, int C, bool kCull, bool kRuns = false>
__device__ __forceinline__ void tile_sums(const float2 *__restrict__ pts, int64_t beg, int64_t end, float Hx,
                                          float Hy, float ax, float ay, int ib, int jb, float bx0, float bx1,
                                          float by0, float by1, float2 *sp, int *swave, float (&tot)[R][C]) {
    // Node coordinates of the block's first column and row; the others are these
    // plus small integers, and (node - X) stays exact in FP32 for |X| < 2^24.
    const float fib = (float)ib, fjb = (float)jb;
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int c = 0; c < C; ++c) tot[r][c] = 0.0f;
    for (int64_t base = beg; base < end; base += kPointTile)
        chunk_sums<K, R, C, kCull, kRuns>(pts, base, end, Hx, Hy, ax, ay, fib, fjb, bx0, bx1, by0, by1, sp, swave,
                                          tot);
}

// Compact kernels over points [0, n) whose kPointTile-point chunks have
// bounding boxes (x min, x max, y min, y max) in boxes[]: the chunks are tested
// kThreads at a time, and only those whose box reaches the tile are loaded, in
// index order.  A chunk whose box misses the tile has no point that passes the
// per-point test of chunk_sums (x max + Hx >= x0 follows from x + Hx >= x0 by
// the monotonicity of rounding, and likewise for the other sides), so the sums
// equal tile_sums' bit for bit.  slist: LDS [kThreads] int.
template <int K, int R, int C>
__device__ __forceinline__ void tile_sums_boxed(const float2 *__restrict__ pts, int64_t n,
                                                const float4 *__restrict__ boxes, float Hx, float Hy, float ax,
                                                float ay, int ib, int jb, float bx0, float bx1, float by0, float by1,
                                                float2 *sp, int *swave, int *slist, float (&tot)[R][C]) {
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const float fib = (float)ib, fjb = (float)jb;
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int c = 0; c < C; ++c) tot[r][c] = 0.0f;
    const int64_t nch = (n + kPointTile - 1) / kPointTile;
    for (int64_t g0 = 0; g0 < nch; g0 += kThreads) {
        const int64_t c = g0 + tid;
        bool hit = false;
        if (c < nch) {
            const float4 b = boxes[c];
            hit = b.y + Hx >= bx0 && b.x - Hx <= bx1 && b.w + Hy >= by0 && b.z - Hy <= by1;
        }
        const uint64_t m = __ballot(hit);
        const int before = __popcll(m & ((1ull << lane) - 1ull));
        __syncthreads();  // the previous group's list and counts are consumed
        if (lane == 0) swave[w] = __popcll(m);
        __syncthreads();
        int off = 0, cnt = 0;
#pragma unroll
        for (int k = 0; k < kThreads / 64; ++k) {
            off += (k < w) ? swave[k] : 0;
            cnt += swave[k];
        }
        if (hit) slist[off + before] = (int)(c - g0);
        __syncthreads();
        for (int k = 0; k < cnt; ++k) {
            const int64_t base = (g0 + slist[k]) * kPointTile;
            chunk_sums<K, R, C, true, false>(pts, base, min(n, base + kPointTile), Hx, Hy, ax, ay, fib, fjb, bx0,
                                             bx1, by0, by1, sp, swave, tot);
        }
    }
}

// Fixed-point accumulation of compact kernels with small supports (support
// binning and batched tiles): a point adds its own terms g(s) g(t) at the nodes
// of its support inside a TW x TH tile at (x0, y0), as round(v 2^32) with 64-bit
// integer atomics into acc (LDS), so the sums are exact in the rounded terms and
// independent of the order the points arrive in (n < 2^31 terms of at most
// 2^32 cannot overflow).  Nodes are tried from floor(X - H) - 1 over
// floor(2 H) + 3 per axis with the factor's own support test, so rounding of
// X - H never drops a node of the support; the tile's nodes past the grid
// (nx, ny) are skipped.  The point's support must reach the tile (its
// coordinates then convert to int safely).
constexpr float kFixedOne = 4294967296.0f;  // 2^32
// Nodes tried per point, at most, on the single-map path: beyond, the gather is
// faster (the cosine's gather, with a transcendental per factor, later).
constexpr int kAccumMaxFootprint = 225;
constexpr int kAccumMaxFootprintCosine = 441;

// Batched tiles: every item already lists the chunks that reach its tile, and
// the gather there loses to the accumulation up to larger supports.
constexpr int kBatchAccumMaxFootprint = 441;

__host__ __device__ inline bool accum_footprint_fits(float Hx, float Hy, int limit = kAccumMaxFootprint) {
    if (!(Hx > 0.0f && Hy > 0.0f && Hx < 64.0f && Hy < 64.0f)) return false;  // NaN fails; int conversions safe
    return ((int)floorf(2.0f * Hx) + 3) * ((int)floorf(2.0f * Hy) + 3) <= limit;
}

__host__ __device__ inline bool accum_applies(int kernel_id, int rc, float Hx, float Hy) {
    return kernel_id != kGaussian && kernel_id != kGaussTrunc && rc <= 4 &&
           accum_footprint_fits(Hx, Hy, kernel_id == kCosine ? kAccumMaxFootprintCosine : kAccumMaxFootprint);
}

template <int K, int TW, int TH>
__device__ __forceinline__ void accum_point(float2 v, int x0, int y0, int nx, int ny, float Hx, float Hy, float ax,
                                            float ay, unsigned long long *acc) {
    const int j0 = (int)floorf(v.y - Hy) - 1, i0 = (int)floorf(v.x - Hx) - 1;
    const int jlo = max(j0, y0), jhi = min(min(j0 + (int)floorf(2.0f * Hy) + 3, y0 + TH), ny);
    const int ilo = max(i0, x0), ihi = min(min(i0 + (int)floorf(2.0f * Hx) + 3, x0 + TW), nx);
    for (int j = jlo; j < jhi; ++j) {
        const float ty = factor<K>((float)j - v.y, ay, Hy);
        if (!(ty > 0.0f)) continue;
        for (int i = ilo; i < ihi; ++i) {
            // the compact factors are >= 0; the FP32 cosine at the support edge can
            // round to a tiny negative, which the clamp turns into the exact 0
            const float w = fmaxf(ty * factor<K>((float)i - v.x, ax, Hx), 0.0f);
            if (w > 0.0f) atomicAdd(&acc[(j - y0) * TW + (i - x0)], __float2ull_rn(w * kFixedOne));
        }
    }
}

// Register-block shape: R x C = RC x RC per thread, so a workgroup covers a
// 16 RC x 16 RC pixel tile.  Larger blocks amortise each factor over more FMAs;
// smaller tiles waste fewer evaluations on pixels outside a compact kernel's
// support and give more workgroups.  The shape is chosen per map (autotuned or
// by default), among kTileShapes.
template <int K, int RC>
struct Shape {
    static constexpr int R = RC;
    static constexpr int C = RC;
    static constexpr bool kCull = K != kGaussian;
    static constexpr int TW = 16 * C, TH = 16 * R;
};

}  // namespace tile
}  // namespace kde
