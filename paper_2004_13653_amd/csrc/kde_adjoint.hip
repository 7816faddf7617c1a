// Adjoints of the KDE heat map on gfx950 (FP32 per pair, FP64 final sums).
//
// 1. Vector-Jacobian product of the map.  With S[j][i] = sum_p g(s_ip) g(t_jp),
//    s_ip = (i - X_p)/Hx, t_jp = (j - Y_p)/Hy (grid units) and a cotangent
//    Gbar[j][i], every point needs the bilinear sums
//      Tx_p = sum_{j,i} Gbar g'(s) g(t)      Ty_p = sum Gbar g(s) g'(t)
//      Ux_p = sum Gbar s g'(s) g(t)          Uy_p = sum Gbar g(s) t g'(t)
//      Q_p  = sum Gbar g(s) g(t)
//    from which the host-side chain rule forms dL/dX_p, dL/dY_p and the
//    bandwidth gradient (see kde_api.cpp).
//    Layout: one thread per point (a workgroup owns 256 consecutive points), so
//    no sum is shared between threads.  The grid is swept in strips of 32
//    columns: each thread keeps its point's 32 column factors g, g' and s g' in
//    registers, the workgroup stages the strip's Gbar rows in LDS, and every row
//    costs 96 FMAs against three LDS broadcast rows plus one row factor pair.
//    Compact kernels sweep only the strips and rows that the workgroup's points
//    can reach (their bounding box widened by the support).
//
// 2. Least-squares cross-validation sums over ordered point pairs (p, q):
//      SA = sum kb(u) kb(v)   SAX = sum (kb(u) + u kb'(u)) kb(v)   SAY likewise
//      SB = sum g(u) g(v)     SBX = sum (g(u) + u g'(u)) g(v)      SBY likewise
//    with u = (X_p - X_q)/Hx, v = (Y_p - Y_q)/Hy, kb the autoconvolution of g
//    (normalising constants are applied on the host).  One thread per p, q
//    streamed through LDS 256 at a time; FP32 partials per q tile are added to
//    FP64 accumulators and reduced per workgroup in FP64 in a fixed order.  The
//    p == q terms are included here and removed on the host (each contributes
//    exactly 1 to SB, SBX and SBY).
//
// 3. Support-culled LSCV for the compact kernels.  kb vanishes for |u| >= 2 and
//    g for |u| > 1, so a pair (p, q) adds nothing once |X_p - X_q| >= 2 Hx or
//    |Y_p - Y_q| >= 2 Hy; at vessel-track densities only a few per mille of the
//    pairs are that close.  The points are first put in spatial (Z-order) order
//    (kde_sort.hip), so that each 256-point block covers a small region; each
//    block's bounding box is taken, and a tile (p-block, q-block >= p-block) is
//    visited only if the boxes are closer than 2H on both axes.  The test is on
//    the FP32 values the pair terms use (gap * (1/H) >= 2 implies |d| * (1/H)
//    >= 2 for every pair of the two blocks, rounding being monotone), so a
//    skipped tile is one whose every term is exactly zero.  The visited tiles,
//    counted per p-block row and prefix-summed, form one sequence in row order
//    that a fixed grid of workgroups cuts into equal runs; each workgroup finds
//    its first tile by a binary search over the row offsets and walks the rows'
//    candidate q-blocks 256 at a time (a ballot compaction of the box tests).
//    Per tile the pair loop is that of (2).  All orders are fixed: the sums are
//    bitwise reproducible.
#include "kde_internal.h"

#include <algorithm>

#include <cmath>

namespace kde {

namespace {

constexpr int kAdjThreads = 256;
constexpr int kStrip = 32;        // columns per strip
constexpr int kRowChunk = 256;    // Gbar rows staged per LDS fill
constexpr float kFarAdj = 1.0e30f;

// g, g' and the support test for grid-unit difference d (u = d / H).
template <int K>
__device__ __forceinline__ void gdg(float d, float H, float inv, float &g, float &dg) {
    const float u = d * inv;
    if constexpr (K == kGaussian) {
        g = __builtin_amdgcn_exp2f(-0.72134752044448170368f * u * u);  // exp(-u^2/2)
        dg = -u * g;
        return;
    } else {
        const bool in = fabsf(d) <= H;
        const float a = fminf(fabsf(u), 1.0f);
        const float sg = u < 0.0f ? -1.0f : (u > 0.0f ? 1.0f : 0.0f);
        float v, w;
        if constexpr (K == kUniform) {
            v = 1.0f;
            w = 0.0f;
        } else if constexpr (K == kTriangular) {
            v = 1.0f - a;
            w = -sg;
        } else if constexpr (K == kEpanechnikov) {
            v = 1.0f - a * a;
            w = -2.0f * sg * a;
        } else if constexpr (K == kQuartic) {
            const float q = 1.0f - a * a;
            v = q * q;
            w = -4.0f * sg * a * q;
        } else if constexpr (K == kTriweight) {
            const float q = 1.0f - a * a;
            v = q * q * q;
            w = -6.0f * sg * a * q * q;
        } else if constexpr (K == kTricube) {
            const float q = 1.0f - a * a * a;
            v = q * q * q;
            w = -9.0f * sg * a * a * q * q;
        } else {  // cosine: g = cos(pi u / 2), g' = -(pi/2) sin(pi u / 2)
            v = __builtin_amdgcn_cosf(a * 0.25f);
            w = -1.57079632679489662f * sg * __builtin_amdgcn_sinf(a * 0.25f);
        }
        g = in ? v : 0.0f;
        dg = in ? w : 0.0f;
    }
}

struct VjpLaunch {
    const float2 *pts;
    int64_t n;
    const float *gbar;  // [ny][nx]
    int nx, ny;
    float Hx, Hy, ix, iy;  // bandwidths and their inverses (grid units)
    float fx, fy;          // output scales for dL/dX and dL/dY (host chain rule)
    float *grad;           // [n][2] or null
    double *part;          // [gridDim.x][3]: per-workgroup sums of Ux, Uy, Q
};

template <int K>
__global__ __launch_bounds__(kAdjThreads) void vjp_kernel(VjpLaunch p) {
    __shared__ float gs[kRowChunk][kStrip];
    __shared__ float box[4][kAdjThreads / 64];
    __shared__ double red[3][kAdjThreads];

    const int tid = threadIdx.x;
    const int64_t q = (int64_t)blockIdx.x * kAdjThreads + tid;
    const bool active = q < p.n;
    const float2 pt = active ? p.pts[q] : make_float2(kFarAdj, kFarAdj);

    // Reach of this workgroup's points (compact kernels only).
    int cx0 = 0, cx1 = p.nx - 1, ry0 = 0, ry1 = p.ny - 1;
    if constexpr (K != kGaussian) {
        float lox = active ? pt.x : 3.0e38f, hix = active ? pt.x : -3.0e38f;
        float loy = active ? pt.y : 3.0e38f, hiy = active ? pt.y : -3.0e38f;
        for (int off = 32; off > 0; off >>= 1) {
            lox = fminf(lox, __shfl_xor(lox, off));
            hix = fmaxf(hix, __shfl_xor(hix, off));
            loy = fminf(loy, __shfl_xor(loy, off));
            hiy = fmaxf(hiy, __shfl_xor(hiy, off));
        }
        if ((tid & 63) == 0) {
            box[0][tid >> 6] = lox;
            box[1][tid >> 6] = hix;
            box[2][tid >> 6] = loy;
            box[3][tid >> 6] = hiy;
        }
        __syncthreads();
        for (int w = 0; w < kAdjThreads / 64; ++w) {
            lox = fminf(lox, box[0][w]);
            hix = fmaxf(hix, box[1][w]);
            loy = fminf(loy, box[2][w]);
            hiy = fmaxf(hiy, box[3][w]);
        }
        // Nodes within H of the box (clamped to the grid; empty if none).
        cx0 = (int)fmaxf(0.0f, ceilf(lox - p.Hx));
        cx1 = (int)fminf((float)(p.nx - 1), floorf(hix + p.Hx));
        ry0 = (int)fmaxf(0.0f, ceilf(loy - p.Hy));
        ry1 = (int)fminf((float)(p.ny - 1), floorf(hiy + p.Hy));
    }

    float Tx = 0.0f, Ty = 0.0f, Ux = 0.0f, Uy = 0.0f, Q = 0.0f;
    if (cx0 <= cx1 && ry0 <= ry1) {
        const int s0 = cx0 / kStrip, s1 = cx1 / kStrip;
        for (int s = s0; s <= s1; ++s) {
            const int i0 = s * kStrip;
            // Column factors of this thread's point for the strip.
            float gx[kStrip], dgx[kStrip], sdgx[kStrip];
#pragma unroll
            for (int c = 0; c < kStrip; ++c) {
                const float d = (float)(i0 + c) - pt.x;
                float g, dg;
                gdg<K>(d, p.Hx, p.ix, g, dg);
                const bool in = i0 + c < p.nx;
                gx[c] = in ? g : 0.0f;
                dgx[c] = in ? dg : 0.0f;
                sdgx[c] = in ? d * p.ix * dg : 0.0f;
            }
            for (int r0 = ry0; r0 <= ry1; r0 += kRowChunk) {
                const int rows = min(kRowChunk, ry1 - r0 + 1);
                __syncthreads();  // previous chunk consumed
                for (int e = tid; e < rows * kStrip; e += kAdjThreads) {
                    const int rr = e / kStrip, cc = e % kStrip;
                    const int col = i0 + cc;
                    gs[rr][cc] = col < p.nx ? p.gbar[(int64_t)(r0 + rr) * p.nx + col] : 0.0f;
                }
                __syncthreads();
                for (int rr = 0; rr < rows; ++rr) {
                    float a1 = 0.0f, a2 = 0.0f, a3 = 0.0f;
#pragma unroll
                    for (int c = 0; c < kStrip; c += 4) {
                        const float4 gb = *reinterpret_cast<const float4 *>(&gs[rr][c]);
                        a1 = fmaf(gb.x, dgx[c], a1);
                        a2 = fmaf(gb.x, gx[c], a2);
                        a3 = fmaf(gb.x, sdgx[c], a3);
                        a1 = fmaf(gb.y, dgx[c + 1], a1);
                        a2 = fmaf(gb.y, gx[c + 1], a2);
                        a3 = fmaf(gb.y, sdgx[c + 1], a3);
                        a1 = fmaf(gb.z, dgx[c + 2], a1);
                        a2 = fmaf(gb.z, gx[c + 2], a2);
                        a3 = fmaf(gb.z, sdgx[c + 2], a3);
                        a1 = fmaf(gb.w, dgx[c + 3], a1);
                        a2 = fmaf(gb.w, gx[c + 3], a2);
                        a3 = fmaf(gb.w, sdgx[c + 3], a3);
                    }
                    const float dy = (float)(r0 + rr) - pt.y;
                    float gy, dgy;
                    gdg<K>(dy, p.Hy, p.iy, gy, dgy);
                    Tx = fmaf(gy, a1, Tx);
                    Ux = fmaf(gy, a3, Ux);
                    Q = fmaf(gy, a2, Q);
                    Ty = fmaf(dgy, a2, Ty);
                    Uy = fmaf(dy * p.iy * dgy, a2, Uy);
                }
            }
        }
    }
    if (active && p.grad != nullptr) {
        p.grad[2 * q] = p.fx * Tx;
        p.grad[2 * q + 1] = p.fy * Ty;
    }
    // Bandwidth sums: FP64 tree over the workgroup, fixed order.
    red[0][tid] = active ? (double)Ux : 0.0;
    red[1][tid] = active ? (double)Uy : 0.0;
    red[2][tid] = active ? (double)Q : 0.0;
    __syncthreads();
    for (int w = kAdjThreads / 2; w > 0; w >>= 1) {
        if (tid < w) {
            red[0][tid] += red[0][tid + w];
            red[1][tid] += red[1][tid + w];
            red[2][tid] += red[2][tid + w];
        }
        __syncthreads();
    }
    if (tid == 0) {
        p.part[3 * blockIdx.x + 0] = red[0][0];
        p.part[3 * blockIdx.x + 1] = red[1][0];
        p.part[3 * blockIdx.x + 2] = red[2][0];
    }
}

// Compact kernels with small supports: one thread per point over the nodes of
// its own support window (from ceil(X - H) - 1 to floor(X + H) + 1 per axis,
// clamped to the grid; gdg's support test decides), reading Gbar from the
// caches, instead of every thread of a workgroup sweeping the bounding box of
// all its points.  The same sums per point (columns within a row, then rows, in
// order) and the same FP64 tree for the bandwidth sums.
constexpr int kVjpLocalMaxWindow = 1024;  // nodes per point, at most

template <int K>
__global__ __launch_bounds__(kAdjThreads) void vjp_local_kernel(VjpLaunch p) {
    __shared__ double red[3][kAdjThreads];
    const int tid = threadIdx.x;
    const int64_t q = (int64_t)blockIdx.x * kAdjThreads + tid;
    const bool active = q < p.n;
    const float2 pt = active ? p.pts[q] : make_float2(kFarAdj, kFarAdj);
    float Tx = 0.0f, Ty = 0.0f, Ux = 0.0f, Uy = 0.0f, Q = 0.0f;
    // The window, or an empty one for points whose support misses the grid
    // (NaN coordinates fail every comparison).
    const bool near = pt.x + p.Hx >= 0.0f && pt.x - p.Hx <= (float)(p.nx - 1) && pt.y + p.Hy >= 0.0f &&
                      pt.y - p.Hy <= (float)(p.ny - 1);
    if (active && near) {
        const int i0 = max(0, (int)ceilf(pt.x - p.Hx) - 1), i1 = min(p.nx - 1, (int)floorf(pt.x + p.Hx) + 1);
        const int j0 = max(0, (int)ceilf(pt.y - p.Hy) - 1), j1 = min(p.ny - 1, (int)floorf(pt.y + p.Hy) + 1);
        for (int j = j0; j <= j1; ++j) {
            const float dy = (float)j - pt.y;
            float gy, dgy;
            gdg<K>(dy, p.Hy, p.iy, gy, dgy);
            if (gy == 0.0f && dgy == 0.0f) continue;  // outside the support: the row adds nothing
            const float *row = p.gbar + (int64_t)j * p.nx;
            float a1 = 0.0f, a2 = 0.0f, a3 = 0.0f;
            for (int i = i0; i <= i1; ++i) {
                const float d = (float)i - pt.x;
                float gx, dgx;
                gdg<K>(d, p.Hx, p.ix, gx, dgx);
                const float gb = row[i];
                a1 = fmaf(gb, dgx, a1);
                a2 = fmaf(gb, gx, a2);
                a3 = fmaf(gb, d * p.ix * dgx, a3);
            }
            Tx = fmaf(gy, a1, Tx);
            Ux = fmaf(gy, a3, Ux);
            Q = fmaf(gy, a2, Q);
            Ty = fmaf(dgy, a2, Ty);
            Uy = fmaf(dy * p.iy * dgy, a2, Uy);
        }
    }
    if (active && p.grad != nullptr) {
        p.grad[2 * q] = p.fx * Tx;
        p.grad[2 * q + 1] = p.fy * Ty;
    }
    red[0][tid] = active ? (double)Ux : 0.0;
    red[1][tid] = active ? (double)Uy : 0.0;
    red[2][tid] = active ? (double)Q : 0.0;
    __syncthreads();
    for (int w = kAdjThreads / 2; w > 0; w >>= 1) {
        if (tid < w) {
            red[0][tid] += red[0][tid + w];
            red[1][tid] += red[1][tid + w];
            red[2][tid] += red[2][tid + w];
        }
        __syncthreads();
    }
    if (tid == 0) {
        p.part[3 * blockIdx.x + 0] = red[0][0];
        p.part[3 * blockIdx.x + 1] = red[1][0];
        p.part[3 * blockIdx.x + 2] = red[2][0];
    }
}

struct LscvLaunch {
    const float2 *pts;
    int64_t n;
    float ix2, iy2;   // 1/H^2 (grid units)
    float ix, iy;     // 1/H
    double *part;     // [gridDim.x][6]
};

// Horner evaluation with compile-time coefficients, highest power first.
__device__ __forceinline__ float hp(float, float acc) { return acc; }
template <typename... C>
__device__ __forceinline__ float hp(float t, float acc, float c, C... rest) {
    return hp(t, fmaf(acc, t, c), rest...);
}

// Per pair and axis, from the grid-unit difference d (scaled u = d/H: the
// Gaussian through u^2 = d^2/H^2, the compact kernels through |u| = |d|/H) the four factors
// kb, kb + u kb', g, g + u g' (without normalising constants).  g is the Table I
// factor scaled to g(0) = 1 and kb its autoconvolution g * g (support |u| < 2)
// up to a constant; the launch's host code applies the constants.
//
// The autoconvolutions of the polynomial factors are piecewise polynomials:
// the integral over the overlap [a - 1, 1] (a = |u|) of g(v) g(a - v), one
// polynomial on 0 <= a <= 1 and one on 1 <= a <= 2 (for the even polynomial
// factors the two coincide).  They are evaluated in FP32 around each piece's
// midpoint (t = a - 1/2 or a - 3/2), where the terms stay within a few times
// the result; the coefficients below are those expansions, rounded to FP32.
template <int K>
__device__ __forceinline__ void lscv_axis(float d, float ih, float i2, float &kb, float &kbd, float &g, float &gd) {
    if constexpr (K == kGaussian) {
        const float w = fminf(d * d * i2, 1.0e4f);  // u^2, capped: every factor is 0 there and stays finite
        kb = __builtin_amdgcn_exp2f(-0.36067376022224085f * w);  // exp(-u^2/4)
        g = kb * kb;                                              // exp(-u^2/2)
        kbd = kb * fmaf(-0.5f, w, 1.0f);                          // (1 - u^2/2) kb
        gd = g * (1.0f - w);                                      // (1 - u^2) g
    } else if constexpr (K == kEpanechnikov) {  // kb ~ (2-a)^3 (a^2 + 6a + 4) on a <= 2, g = 1 - u^2 on a <= 1
        const float a = fminf(fabsf(d) * ih, 100.0f), w = a * a;  // |u|, capped: every factor is 0 there
        const float b = fmaxf(2.0f - a, 0.0f);
        const float b2 = b * b;
        kb = b2 * b * (w + 6.0f * a + 4.0f);
        kbd = kb - 5.0f * w * (a + 4.0f) * b2;
        const bool in = w <= 1.0f;
        g = in ? 1.0f - w : 0.0f;
        gd = in ? 1.0f - 3.0f * w : 0.0f;
    } else {
        const float a = fminf(fabsf(d) * ih, 100.0f), w = a * a;
        const bool reach = a < 2.0f, lo = a <= 1.0f, in = w <= 1.0f;
        float klo, khi, dlo, dhi;  // kb and kb + a kb' on each piece
        if constexpr (K == kUniform) {  // kb = 2 - a
            klo = khi = 2.0f - a;
            dlo = dhi = 2.0f - 2.0f * a;
            g = in ? 1.0f : 0.0f;
            gd = g;
        } else if constexpr (K == kTriangular) {  // the centred cubic B-spline
            const float b = 2.0f - a;
            klo = fmaf(w, fmaf(3.0f, a, -6.0f), 4.0f) * (1.0f / 6.0f);
            khi = b * b * b * (1.0f / 6.0f);
            dlo = fmaf(w, fmaf(12.0f, a, -18.0f), 4.0f) * (1.0f / 6.0f);
            dhi = b * b * fmaf(-4.0f, a, 2.0f) * (1.0f / 6.0f);
            g = in ? 1.0f - a : 0.0f;
            gd = in ? fmaf(-2.0f, a, 1.0f) : 0.0f;
        } else if constexpr (K == kQuartic) {
            const float tl = a - 0.5f, th = a - 1.5f;
            klo = hp(tl, -1.587301587e-03f, -7.142857143e-03f, 2.380952381e-02f, 1.166666667e-01f, -3.458333333e-01f,
                     -1.062500000e-01f, 8.812500000e-01f, -2.611607143e-01f, -8.482700893e-01f, 5.582310268e-01f);
            khi = hp(th, -1.587301587e-03f, -2.142857143e-02f, -9.047619048e-02f, -5.000000000e-02f, 2.541666667e-01f,
                     4.791666667e-02f, -3.687500000e-01f, 2.796130952e-01f, -8.577008929e-02f, 9.712921627e-03f);
            dlo = hp(tl, -1.587301587e-02f, -7.142857143e-02f, 1.619047619e-01f, 9.000000000e-01f, -1.725000000e+00f,
                     -1.395833333e+00f, 3.312500000e+00f, 5.383928571e-01f, -1.957700893e+00f, 1.340959821e-01f);
            dhi = hp(th, -1.587301587e-02f, -2.142857143e-01f, -9.809523810e-01f, -1.300000000e+00f, 1.075000000e+00f,
                     2.145833333e+00f, -1.187500000e+00f, -8.205357143e-01f, 6.672991071e-01f, -1.189422123e-01f);
            const float v = 1.0f - w;  // g = (1 - u^2)^2, u g' = -4 u^2 (1 - u^2)
            g = in ? v * v : 0.0f;
            gd = in ? v * fmaf(-5.0f, w, 1.0f) : 0.0f;
        } else if constexpr (K == kTriweight) {
            const float tl = a - 0.5f, th = a - 1.5f;
            klo = hp(tl, -8.325008325e-05f, -5.411255411e-04f, 9.740259740e-04f, 1.130952381e-02f, -6.101190476e-03f,
                     -1.212053571e-01f, 1.656250000e-01f, 3.220982143e-01f, -6.245256696e-01f, -3.529436384e-01f,
                     1.104031808e+00f, -6.887999696e-02f, -8.430865399e-01f, 4.149201933e-01f);
            khi = hp(th, -8.325008325e-05f, -1.623376623e-03f, -1.201298701e-02f, -3.750000000e-02f, -1.800595238e-02f,
                     1.185267857e-01f, 8.348214286e-02f, -2.426339286e-01f, -5.775669643e-03f, 2.686988467e-01f,
                     -2.391601563e-01f, 9.679446530e-02f, -1.950953100e-02f, 1.591997277e-03f);
            dlo = hp(tl, -1.165501166e-03f, -7.575757576e-03f, 8.441558442e-03f, 1.297619048e-01f, -4.464285714e-03f,
                     -1.118303571e+00f, 8.401785714e-01f, 2.834375000e+00f, -2.780859375e+00f, -3.326032366e+00f,
                     3.710239955e+00f, 1.449407721e+00f, -1.755053077e+00f, -6.623076630e-03f);
            dhi = hp(th, -1.165501166e-03f, -2.272727273e-02f, -1.733766234e-01f, -6.107142857e-01f, -7.425595238e-01f,
                     8.236607143e-01f, 2.090178571e+00f, -8.218750000e-01f, -2.218359375e+00f, 1.300176711e+00f,
                     6.555524554e-01f, -7.858373072e-01f, 2.513643339e-01f, -2.767229922e-02f);
            const float v = 1.0f - w;  // g = (1 - u^2)^3, u g' = -6 u^2 (1 - u^2)^2
            g = in ? v * v * v : 0.0f;
            gd = in ? v * v * fmaf(-7.0f, w, 1.0f) : 0.0f;
        } else if constexpr (K == kTricube) {
            const float tl = a - 0.5f, th = a - 1.5f;
            klo = hp(tl, 3.247526467e-06f, 3.085150144e-05f, 1.388317565e-04f, 3.184315684e-04f, 1.873126873e-04f,
                     -1.067682318e-03f, 1.676448551e-03f, 2.879464286e-02f, 9.884841721e-02f, -3.200334821e-02f,
                     2.913643973e-01f, -3.782207539e-01f, -6.789474685e-01f, 7.915561245e-01f, 1.970283257e-01f,
                     -5.366161487e-01f, 7.719792895e-01f, -2.202373705e-01f, -9.418320762e-01f, 6.534530266e-01f);
            khi = hp(th, -1.082508822e-06f, -3.085150144e-05f, -4.164952694e-04f, -3.465284715e-03f, -1.944305694e-02f,
                     -7.535589411e-02f, -1.957885864e-01f, -2.971387987e-01f, -1.113585633e-01f, 4.632533482e-01f,
                     7.370675223e-01f, -7.730379972e-02f, -9.847535765e-01f, -2.053903372e-01f, 8.611649215e-01f,
                     6.489563293e-02f, -6.115566235e-01f, 3.679434487e-01f, -9.104161577e-02f, 8.480808063e-03f);
            dlo = hp(tl, 6.495052935e-05f, 6.170300288e-04f, 2.776635130e-03f, 6.593406593e-03f, 5.544455544e-03f,
                     -1.461038961e-02f, 1.599650350e-02f, 3.852272727e-01f, 1.358948864e+00f, 1.916294643e-01f,
                     2.753627232e+00f, -2.092846997e+00f, -6.944462764e+00f, 3.164576732e+00f, 3.556838328e+00f,
                     -2.190509930e+00f, 2.014684860e+00f, 4.972568226e-01f, -2.103901523e+00f, 1.825369885e-01f);
            dhi = hp(th, -2.165017645e-05f, -6.170300288e-04f, -8.329905389e-03f, -6.953046953e-02f, -3.942557443e-01f,
                     -1.567807193e+00f, -4.323513986e+00f, -7.680681818e+00f, -6.684801136e+00f, 3.258370536e+00f,
                     1.431947545e+01f, 9.254677354e+00f, -8.805674209e+00f, -1.177764491e+01f, 3.318476494e+00f,
                     6.783215076e+00f, -2.056852696e+00f, -1.648174460e+00f, 9.217471144e-01f, -1.280816156e-01f);
            const float c3 = w * a, v = 1.0f - c3;  // g = (1 - a^3)^3, u g' = -9 a^3 (1 - a^3)^2
            g = in ? v * v * v : 0.0f;
            gd = in ? v * v * fmaf(-10.0f, c3, 1.0f) : 0.0f;
        } else {  // cosine: kb = ((2/pi) sin(pi a/2) + (2 - a) cos(pi a/2)) / 2, kb' = -(pi/4)(2 - a) sin(pi a/2)
            const float s = __builtin_amdgcn_sinf(a * 0.25f), c = __builtin_amdgcn_cosf(a * 0.25f);  // revolutions
            const float b = 2.0f - a;
            klo = khi = fmaf(0.5f * b, c, 0.31830988618379067f * s);
            dlo = dhi = klo - 0.78539816339744831f * a * b * s;
            g = in ? c : 0.0f;
            gd = in ? fmaf(-1.5707963267948966f * a, s, c) : 0.0f;
        }
        kb = reach ? (lo ? klo : khi) : 0.0f;
        kbd = reach ? (lo ? dlo : dhi) : 0.0f;
    }
}

// LSCV work plan.  Every pair term is symmetric in (p, q) (it depends on |dx|
// and |dy| only), so only the tiles (p-block, q-block) with q-block >= p-block
// are visited: an off-diagonal tile counts twice, and in a diagonal tile the
// pairs q > p count twice and p = q once, which gives the sums over all ordered
// pairs with half the work.  The row of tiles of p-block b is paired with that of
// p-block nb - 1 - b (together nb + 1 tiles, the same for every pair; the middle
// row of an odd nb stands alone), and each pair of rows is cut into `chunks`
// equal runs of tiles, one workgroup each.
struct LscvPlan {
    int64_t nb, units, chunks;
};

LscvPlan lscv_plan(int64_t n) {
    LscvPlan pl;
    pl.nb = (n + kAdjThreads - 1) / kAdjThreads;
    pl.units = (pl.nb + 1) / 2;
    const int64_t want = (2048 + pl.units - 1) / pl.units;                 // aim at ~2048 workgroups
    pl.chunks = std::max<int64_t>(1, std::min<int64_t>(want, (pl.nb + 1) / 4));  // at least ~4 tiles each
    return pl;
}

// Pair terms of one tile: thread tid holds point p of p-block pb (me, valid),
// the q-block's points are staged in qs; adds the tile's FP32 sums, doubled
// (symmetry), to S, and for a diagonal tile the pairs q > p only plus p = q once.
template <int K>
__device__ __forceinline__ void lscv_tile(const LscvLaunch &p, float2 me, bool diag, const float2 *qs, int tid,
                                          double (&S)[6], float4 reach = make_float4(-3.0e38f, 3.0e38f, -3.0e38f,
                                                                                     3.0e38f)) {
    float sa = 0.0f, sax = 0.0f, say = 0.0f, sb = 0.0f, sbx = 0.0f, sby = 0.0f;
    if constexpr (K == kGaussian) {
        // kb(u) kb(v) = exp(-(u^2 + v^2)/4) is one exp2 per pair, and g(u) g(v) =
        // exp(-(u^2 + v^2)/2) its square; the derivative factors are those of
        // lscv_axis, (1 - u^2/2) for kb and (1 - u^2) for g, applied after the
        // loop: the tile keeps sum e and sum u^2 e (sax, say, sbx, sby hold the
        // u^2- and v^2-weighted sums here), one FMA per derivative sum and pair.
        // wx, wy carry the exp2 scale c = log2(e) / 4: wx = c u^2 (capped), and the
        // derivative sums are divided by c after the loop.
        constexpr float c = 0.36067376022224085f;  // log2(e) / 4
        const float cx = c * p.ix2, cy = c * p.iy2, cap = c * 1.0e4f;
        auto pair = [&](float ox, float oy) {
            const float dx = me.x - ox, dy = me.y - oy;
            const float wx = fminf(dx * dx * cx, cap), wy = fminf(dy * dy * cy, cap);  // c u^2, c v^2, capped
            const float e = __builtin_amdgcn_exp2f(-(wx + wy));
            const float e2 = e * e;
            sa += e;
            sb += e2;
            sax = fmaf(wx, e, sax);
            say = fmaf(wy, e, say);
            sbx = fmaf(wx, e2, sbx);
            sby = fmaf(wy, e2, sby);
        };
        if (!diag) {  // the same q for every lane: a uniform loop, two points per LDS read
            const float4 *q2 = reinterpret_cast<const float4 *>(qs);
#pragma unroll 4
            for (int k = 0; k < kAdjThreads / 2; ++k) {
                const float4 o = q2[k];
                pair(o.x, o.y);
                pair(o.z, o.w);
            }
        } else {
            for (int k = tid + 1; k < kAdjThreads; ++k) pair(qs[k].x, qs[k].y);
        }
    } else {
        for (int k = diag ? tid + 1 : 0; k < kAdjThreads; ++k) {
            const float2 o = qs[k];
            // The same q for every lane of the wave: a q beyond the autoconvolution's
            // reach (2H) of all the wave's points adds exact zeros to every sum (the
            // uniform kernel's pair terms cost less than the test).
            if constexpr (K != kUniform)
                if (o.x < reach.x || o.x > reach.y || o.y < reach.z || o.y > reach.w) continue;
            float kbx, kbdx, gx, gdx, kby, kbdy, gy, gdy;
            lscv_axis<K>(me.x - o.x, p.ix, p.ix2, kbx, kbdx, gx, gdx);
            lscv_axis<K>(me.y - o.y, p.iy, p.iy2, kby, kbdy, gy, gdy);
            sa = fmaf(kbx, kby, sa);
            sax = fmaf(kbdx, kby, sax);
            say = fmaf(kbx, kbdy, say);
            sb = fmaf(gx, gy, sb);
            sbx = fmaf(gdx, gy, sbx);
            sby = fmaf(gx, gdy, sby);
        }
    }
    if constexpr (K == kGaussian) {  // sum (1 - u^2/2) e = sum e - sum u^2 e / 2, and so on, in FP64
        constexpr double ic = 1.0 / (double)0.36067376022224085f;  // the u^2 sums carry the FP32 c
        S[0] += 2.0 * sa;
        S[1] += 2.0 * ((double)sa - 0.5 * ic * (double)sax);
        S[2] += 2.0 * ((double)sa - 0.5 * ic * (double)say);
        S[3] += 2.0 * sb;
        S[4] += 2.0 * ((double)sb - ic * (double)sbx);
        S[5] += 2.0 * ((double)sb - ic * (double)sby);
    } else {
        S[0] += 2.0 * sa;
        S[1] += 2.0 * sax;
        S[2] += 2.0 * say;
        S[3] += 2.0 * sb;
        S[4] += 2.0 * sbx;
        S[5] += 2.0 * sby;
    }
    if (diag) {
        float kbx, kbdx, gx, gdx, kby, kbdy, gy, gdy;
        lscv_axis<K>(0.0f, p.ix, p.ix2, kbx, kbdx, gx, gdx);
        lscv_axis<K>(0.0f, p.iy, p.iy2, kby, kbdy, gy, gdy);
        S[0] += kbx * kby;
        S[1] += kbdx * kby;
        S[2] += kbx * kbdy;
        S[3] += gx * gy;
        S[4] += gdx * gy;
        S[5] += gx * gdy;
    }
}

// Workgroup sums of S in FP64, fixed order, into part[blockIdx.x][6].
__device__ __forceinline__ void lscv_store(double (&S)[6], double (*red)[kAdjThreads], double *part, int tid) {
#pragma unroll
    for (int k = 0; k < 6; ++k) red[k][tid] = S[k];
    __syncthreads();
    for (int w = kAdjThreads / 2; w > 0; w >>= 1) {
        if (tid < w) {
#pragma unroll
            for (int k = 0; k < 6; ++k) red[k][tid] += red[k][tid + w];
        }
        __syncthreads();
    }
    if (tid < 6) part[6 * blockIdx.x + tid] = red[tid][0];
}

// All-pairs LSCV (used for the Gaussian, whose every pair counts).
template <int K>
__global__ __launch_bounds__(kAdjThreads) void lscv_kernel(LscvLaunch p, int64_t nb, int64_t chunks) {
    __shared__ __align__(16) float2 qs[kAdjThreads];
    __shared__ double red[6][kAdjThreads];
    const int tid = threadIdx.x;
    const int64_t u = blockIdx.x / chunks, c = blockIdx.x % chunks;
    const int64_t b1 = u, b2 = nb - 1 - u;
    const int64_t len1 = nb - b1, len2 = b2 == b1 ? 0 : nb - b2;
    const int64_t L = len1 + len2, t0 = L * c / chunks, t1 = L * (c + 1) / chunks;
    double S[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int64_t t = t0; t < t1; ++t) {
        const int64_t pb = t < len1 ? b1 : b2, qb = t < len1 ? b1 + t : b2 + (t - len1);
        const int64_t pi = pb * kAdjThreads + tid, qi = qb * kAdjThreads + tid;
        const bool valid = pi < p.n;
        const float2 me = valid ? p.pts[pi] : make_float2(0.0f, 0.0f);
        __syncthreads();  // previous tile fully consumed
        qs[tid] = qi < p.n ? p.pts[qi] : make_float2(kFarAdj, kFarAdj);
        __syncthreads();
        if (valid) lscv_tile<K>(p, me, qb == pb, qs, tid, S);
    }
    lscv_store(S, red, p.part, tid);
}

// Bounding box (xmin, xmax, ymin, ymax) of each 256-point block.
__global__ __launch_bounds__(kAdjThreads) void block_box_kernel(const float2 *__restrict__ pts, int64_t n,
                                                               float4 *__restrict__ box) {
    __shared__ float4 wb[kAdjThreads / 64];
    const int tid = threadIdx.x;
    const int64_t i = (int64_t)blockIdx.x * kAdjThreads + tid;
    const bool ok = i < n;
    const float2 v = ok ? pts[i] : make_float2(0.0f, 0.0f);
    float x0 = ok ? v.x : 3.0e38f, x1 = ok ? v.x : -3.0e38f, y0 = ok ? v.y : 3.0e38f, y1 = ok ? v.y : -3.0e38f;
    for (int off = 32; off > 0; off >>= 1) {
        x0 = fminf(x0, __shfl_xor(x0, off));
        x1 = fmaxf(x1, __shfl_xor(x1, off));
        y0 = fminf(y0, __shfl_xor(y0, off));
        y1 = fmaxf(y1, __shfl_xor(y1, off));
    }
    if ((tid & 63) == 0) wb[tid >> 6] = make_float4(x0, x1, y0, y1);
    __syncthreads();
    if (tid == 0) {
        float4 b = wb[0];
        for (int w = 1; w < kAdjThreads / 64; ++w) {
            b.x = fminf(b.x, wb[w].x);
            b.y = fmaxf(b.y, wb[w].y);
            b.z = fminf(b.z, wb[w].z);
            b.w = fmaxf(b.w, wb[w].w);
        }
        box[blockIdx.x] = b;
    }
}

// Whether some pair of blocks a, b can be closer than 2H on both axes, as the
// pair terms compute it: false only if every pair has |d| * (1/H) >= 2 on an axis.
__device__ __forceinline__ bool boxes_meet(float4 a, float4 b, float ix, float iy) {
    const float gx = fmaxf(b.x - a.y, a.x - b.y);
    const float gy = fmaxf(b.z - a.w, a.z - b.w);
    return !(gx * ix >= 2.0f) && !(gy * iy >= 2.0f);
}

// rowcnt[pb] = number of q-blocks qb >= pb whose box meets pb's.
__global__ __launch_bounds__(kAdjThreads) void tile_count_kernel(const float4 *__restrict__ box, int64_t nb, float ix,
                                                                float iy, unsigned *__restrict__ rowcnt) {
    __shared__ unsigned wsum[kAdjThreads / 64];
    const int tid = threadIdx.x;
    const int64_t pb = blockIdx.x;
    const float4 a = box[pb];
    unsigned c = 0;
    for (int64_t qb = pb + tid; qb < nb; qb += kAdjThreads) c += boxes_meet(a, box[qb], ix, iy) ? 1u : 0u;
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off);
    if ((tid & 63) == 0) wsum[tid >> 6] = c;
    __syncthreads();
    if (tid == 0) {
        unsigned t = 0;
        for (int w = 0; w < kAdjThreads / 64; ++w) t += wsum[w];
        rowcnt[pb] = t;
    }
}

struct CullLaunch {
    const float4 *box;       // [nb]
    const unsigned *rowoff;  // [nb + 1]: exclusive prefix of rowcnt, rowoff[nb] = visited tiles
    int64_t nb;
};

template <int K>
__global__ __launch_bounds__(kAdjThreads) void lscv_cull_kernel(LscvLaunch p, CullLaunch c) {
    __shared__ __align__(16) float2 qs[kAdjThreads];
    __shared__ double red[6][kAdjThreads];
    __shared__ int64_t list[kAdjThreads];
    __shared__ unsigned wsum[kAdjThreads / 64];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    double S[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    const uint64_t total = c.rowoff[c.nb];
    const uint64_t t0 = total * blockIdx.x / gridDim.x, t1 = total * (blockIdx.x + 1) / gridDim.x;
    if (t0 < t1) {
        // Row holding tile t0: the last pb with rowoff[pb] <= t0.
        int64_t lo = 0, hi = c.nb - 1;
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) / 2;
            if ((uint64_t)c.rowoff[mid] <= t0) lo = mid;
            else hi = mid - 1;
        }
        int64_t pb = lo, cand = pb;
        uint64_t skip = t0 - c.rowoff[pb], t = t0;
        float4 a = c.box[pb];
        int64_t pi = pb * kAdjThreads + tid;
        float2 me = pi < p.n ? p.pts[pi] : make_float2(0.0f, 0.0f);
        // The wave's points' box, widened by the autoconvolution's reach 2H (with a
        // margin for rounding): q outside it meet none of the wave's points.
        const float rx = 2.0f / p.ix * 1.0001f + 1.0e-3f, ry = 2.0f / p.iy * 1.0001f + 1.0e-3f;
        auto wave_reach = [&](int64_t i, float2 v) {
            const bool ok = i < p.n;
            float x0 = ok ? v.x : 3.0e38f, x1 = ok ? v.x : -3.0e38f, y0 = ok ? v.y : 3.0e38f, y1 = ok ? v.y : -3.0e38f;
            for (int off = 32; off > 0; off >>= 1) {
                x0 = fminf(x0, __shfl_xor(x0, off));
                x1 = fmaxf(x1, __shfl_xor(x1, off));
                y0 = fminf(y0, __shfl_xor(y0, off));
                y1 = fmaxf(y1, __shfl_xor(y1, off));
            }
            return make_float4(x0 - rx, x1 + rx, y0 - ry, y1 + ry);
        };
        float4 reach = wave_reach(pi, me);
        while (t < t1) {
            if (cand >= c.nb) {  // row done: the next row starts at its diagonal tile
                if (++pb >= c.nb) break;  // not reached: every tile of [t0, t1) lies in a row below nb
                cand = pb;
                a = c.box[pb];
                pi = pb * kAdjThreads + tid;
                me = pi < p.n ? p.pts[pi] : make_float2(0.0f, 0.0f);
                reach = wave_reach(pi, me);
            }
            // Compact the next 256 candidates of the row that meet the p-block.
            const int64_t qb = cand + tid;
            const bool hit = qb < c.nb && boxes_meet(a, c.box[qb], p.ix, p.iy);
            const uint64_t bal = __ballot(hit);
            __syncthreads();  // list and wsum of the previous group consumed
            if (lane == 0) wsum[wave] = (unsigned)__popcll(bal);
            __syncthreads();
            unsigned before = 0, count = 0;
            for (int w = 0; w < kAdjThreads / 64; ++w) {
                before += w < wave ? wsum[w] : 0u;
                count += wsum[w];
            }
            if (hit) list[before + __popcll(bal & ((lane == 0) ? 0ull : (~0ull >> (64 - lane))))] = qb;
            __syncthreads();
            cand += kAdjThreads;
            if (skip >= count) {
                skip -= count;
                continue;
            }
            for (unsigned k = (unsigned)skip; k < count && t < t1; ++k, ++t) {
                const int64_t q = list[k];
                const int64_t qi = q * kAdjThreads + tid;
                __syncthreads();  // previous tile consumed
                qs[tid] = qi < p.n ? p.pts[qi] : make_float2(kFarAdj, kFarAdj);
                __syncthreads();
                if (pi < p.n) lscv_tile<K>(p, me, q == pb, qs, tid, S, reach);
            }
            skip = 0;
        }
    }
    lscv_store(S, red, p.part, tid);
}

}  // namespace

int64_t vjp_blocks(int64_t n) { return (n + kAdjThreads - 1) / kAdjThreads; }

hipError_t launch_vjp(const float2 *pts, int64_t n, int kernel_id, float Hx, float Hy, const float *gbar, int nx,
                      int ny, float fx, float fy, float *grad, double *part, hipStream_t stream) {
    VjpLaunch p{pts, n, gbar, nx, ny, Hx, Hy, (float)(1.0 / (double)Hx), (float)(1.0 / (double)Hy), fx, fy, grad,
                part};
    const dim3 grid((unsigned)vjp_blocks(n));
    main_kernel_begin(stream);
    // Small compact supports: each point over its own window.
    const double wx = std::floor(2.0 * (double)Hx) + 3.0, wy = std::floor(2.0 * (double)Hy) + 3.0;
    if (kernel_id != kGaussian && wx * wy <= (double)kVjpLocalMaxWindow) {
        switch (kernel_id) {
        case kUniform: hipLaunchKernelGGL(vjp_local_kernel<kUniform>, grid, dim3(kAdjThreads), 0, stream, p); break;
        case kTriangular:
            hipLaunchKernelGGL(vjp_local_kernel<kTriangular>, grid, dim3(kAdjThreads), 0, stream, p);
            break;
        case kEpanechnikov:
            hipLaunchKernelGGL(vjp_local_kernel<kEpanechnikov>, grid, dim3(kAdjThreads), 0, stream, p);
            break;
        case kQuartic: hipLaunchKernelGGL(vjp_local_kernel<kQuartic>, grid, dim3(kAdjThreads), 0, stream, p); break;
        case kTriweight:
            hipLaunchKernelGGL(vjp_local_kernel<kTriweight>, grid, dim3(kAdjThreads), 0, stream, p);
            break;
        case kTricube: hipLaunchKernelGGL(vjp_local_kernel<kTricube>, grid, dim3(kAdjThreads), 0, stream, p); break;
        case kCosine: hipLaunchKernelGGL(vjp_local_kernel<kCosine>, grid, dim3(kAdjThreads), 0, stream, p); break;
        default: return hipErrorInvalidValue;
        }
        main_kernel_end(stream);
        return hipGetLastError();
    }
    switch (kernel_id) {
    case kUniform: hipLaunchKernelGGL(vjp_kernel<kUniform>, grid, dim3(kAdjThreads), 0, stream, p); break;
    case kTriangular: hipLaunchKernelGGL(vjp_kernel<kTriangular>, grid, dim3(kAdjThreads), 0, stream, p); break;
    case kEpanechnikov: hipLaunchKernelGGL(vjp_kernel<kEpanechnikov>, grid, dim3(kAdjThreads), 0, stream, p); break;
    case kQuartic: hipLaunchKernelGGL(vjp_kernel<kQuartic>, grid, dim3(kAdjThreads), 0, stream, p); break;
    case kTriweight: hipLaunchKernelGGL(vjp_kernel<kTriweight>, grid, dim3(kAdjThreads), 0, stream, p); break;
    case kTricube: hipLaunchKernelGGL(vjp_kernel<kTricube>, grid, dim3(kAdjThreads), 0, stream, p); break;
    case kGaussian: hipLaunchKernelGGL(vjp_kernel<kGaussian>, grid, dim3(kAdjThreads), 0, stream, p); break;
    case kCosine: hipLaunchKernelGGL(vjp_kernel<kCosine>, grid, dim3(kAdjThreads), 0, stream, p); break;
    default: return hipErrorInvalidValue;
    }
    main_kernel_end(stream);
    return hipGetLastError();
}

namespace {

constexpr int64_t kCullGroups = 2048;  // workgroups of the culled pass (equal runs of the visited tiles)

// Compact kernels use the culled pass while the tile count fits the 32-bit scan.
bool lscv_culled(int64_t n, int kernel_id) {
    const int64_t nb = (n + kAdjThreads - 1) / kAdjThreads;
    return kernel_id != kGaussian && nb * (nb + 1) / 2 < (int64_t(1) << 32);
}

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

// Culled-pass workspace: [part][sorted points][boxes][row counts][scan totals][sort scratch].
struct CullPlan {
    int64_t nb, groups;
    size_t part, sorted, box, rowcnt, totals, sort;
};

CullPlan cull_plan(int64_t n) {
    CullPlan pl;
    pl.nb = (n + kAdjThreads - 1) / kAdjThreads;
    pl.groups = std::max<int64_t>(1, std::min<int64_t>(kCullGroups, pl.nb * (pl.nb + 1) / 2));
    pl.part = align256((size_t)pl.groups * 6 * sizeof(double));
    pl.sorted = align256((size_t)n * sizeof(float2));
    pl.box = align256((size_t)pl.nb * sizeof(float4));
    pl.rowcnt = align256((size_t)(pl.nb + 1) * sizeof(unsigned));
    pl.totals = align256(scan_u32_totals_bytes(pl.nb + 1));
    pl.sort = spatial_sort_bytes(n);
    return pl;
}

template <int K>
void launch_cull_k(const LscvLaunch &p, const CullLaunch &c, int64_t groups, hipStream_t s) {
    hipLaunchKernelGGL(lscv_cull_kernel<K>, dim3((unsigned)groups), dim3(kAdjThreads), 0, s, p, c);
}

template <int K>
void launch_all_k(const LscvLaunch &p, const LscvPlan &pl, hipStream_t s) {
    hipLaunchKernelGGL(lscv_kernel<K>, dim3((unsigned)(pl.units * pl.chunks)), dim3(kAdjThreads), 0, s, p, pl.nb,
                       pl.chunks);
}

template <template <int> class F, class... A>
hipError_t by_kernel(int kernel_id, A &&...args) {
    switch (kernel_id) {
    case kUniform: F<kUniform>::run(args...); break;
    case kTriangular: F<kTriangular>::run(args...); break;
    case kEpanechnikov: F<kEpanechnikov>::run(args...); break;
    case kQuartic: F<kQuartic>::run(args...); break;
    case kTriweight: F<kTriweight>::run(args...); break;
    case kTricube: F<kTricube>::run(args...); break;
    case kGaussian: F<kGaussian>::run(args...); break;
    case kCosine: F<kCosine>::run(args...); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int K>
struct CullRun {
    static void run(const LscvLaunch &p, const CullLaunch &c, int64_t groups, hipStream_t s) {
        launch_cull_k<K>(p, c, groups, s);
    }
};

template <int K>
struct AllRun {
    static void run(const LscvLaunch &p, const LscvPlan &pl, hipStream_t s) { launch_all_k<K>(p, pl, s); }
};

}  // namespace

int64_t lscv_blocks(int64_t n, int kernel_id) {
    if (lscv_culled(n, kernel_id)) return cull_plan(n).groups;
    const LscvPlan pl = lscv_plan(n);
    return pl.units * pl.chunks;
}

size_t lscv_workspace_bytes(int64_t n, int kernel_id) {
    if (!lscv_culled(n, kernel_id)) return (size_t)lscv_blocks(n, kernel_id) * 6 * sizeof(double);
    const CullPlan pl = cull_plan(n);
    return pl.part + pl.sorted + pl.box + pl.rowcnt + pl.totals + pl.sort;
}

hipError_t launch_lscv(const float2 *pts, int64_t n, int kernel_id, float Hx, float Hy, int nx, int ny, void *ws,
                       hipStream_t stream) {
    double *part = static_cast<double *>(ws);
    LscvLaunch p{pts, n, (float)(1.0 / ((double)Hx * Hx)), (float)(1.0 / ((double)Hy * Hy)), (float)(1.0 / (double)Hx),
                 (float)(1.0 / (double)Hy), part};
    if (!lscv_culled(n, kernel_id)) return by_kernel<AllRun>(kernel_id, p, lscv_plan(n), stream);
    const CullPlan pl = cull_plan(n);
    char *w = static_cast<char *>(ws) + pl.part;
    float2 *sorted = reinterpret_cast<float2 *>(w);
    float4 *box = reinterpret_cast<float4 *>(w + pl.sorted);
    unsigned *rowcnt = reinterpret_cast<unsigned *>(w + pl.sorted + pl.box);
    unsigned *totals = reinterpret_cast<unsigned *>(w + pl.sorted + pl.box + pl.rowcnt);
    void *sort_ws = w + pl.sorted + pl.box + pl.rowcnt + pl.totals;
    hipError_t e = launch_spatial_sort(pts, n, spatial_sort_cell(Hx, Hy, nx, ny), sort_ws, sorted, stream);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(block_box_kernel, dim3((unsigned)pl.nb), dim3(kAdjThreads), 0, stream, sorted, n, box);
    hipLaunchKernelGGL(tile_count_kernel, dim3((unsigned)pl.nb), dim3(kAdjThreads), 0, stream, box, pl.nb, p.ix, p.iy,
                       rowcnt);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = launch_fill_zero(reinterpret_cast<float *>(rowcnt + pl.nb), 1, stream)) != hipSuccess) return e;
    if ((e = launch_scan_u32(rowcnt, pl.nb + 1, totals, stream)) != hipSuccess) return e;
    p.pts = sorted;
    return by_kernel<CullRun>(kernel_id, p, CullLaunch{box, rowcnt, pl.nb}, pl.groups, stream);
}

}  // namespace kde
