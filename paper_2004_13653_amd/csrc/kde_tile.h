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

// Raw sums of one pixel tile over points [beg, end): workgroup of 256 threads
// (16 x 16), each an R x C register block of R consecutive rows and C consecutive
// columns starting at (jb, ib); tile reach x0..x1, y0..y1 (nodes) for culling.
// Each LDS tile of points is summed into a fresh block before joining the total.
// sp: LDS [kPointTile] float2; swave: LDS [kThreads / 64] int.
template <int K, int R, int C, bool kCull>
__device__ __forceinline__ void tile_sums(const float2 *__restrict__ pts, int64_t beg, int64_t end, float Hx,
                                          float Hy, float ax, float ay, int ib, int jb, float bx0, float bx1,
                                          float by0, float by1, float2 *sp, int *swave, float (&tot)[R][C]) {
    const int tid = threadIdx.x;
    // Node coordinates of the block's first column and row; the others are these
    // plus small integers, and (node - X) stays exact in FP32 for |X| < 2^24.
    const float fib = (float)ib, fjb = (float)jb;
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int c = 0; c < C; ++c) tot[r][c] = 0.0f;

    for (int64_t base = beg; base < end; base += kPointTile) {
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
        if (cnt == 0) continue;

        float acc[R][C];
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int c = 0; c < C; ++c) acc[r][c] = 0.0f;

        for (int k = 0; k < cnt; ++k) {
            const float2 pt = sp[k];
            const float dx0 = fib - pt.x, dy0 = fjb - pt.y;
            float kx[C], ky[R];
#pragma unroll
            for (int c = 0; c < C; ++c) kx[c] = factor<K>(dx0 + (float)c, ax, Hx);
#pragma unroll
            for (int r = 0; r < R; ++r) ky[r] = factor<K>(dy0 + (float)r, ay, Hy);
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
