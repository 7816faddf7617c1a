// Separable evaluation of the KDE heat map on gfx950 matrix cores.
//
// Every Table I kernel is a product f(s,t) = k(s) k(t) (Sec. III-C), so the raw
// map is a matrix product over the points:
//
//     S = Gy . Gx^T,   Gy[j][p] = g((j - Y_p)/Hy),   Gx[i][p] = g((i - X_p)/Hx),
//
// an [ny x n] by [n x nx] contraction.  The factors are produced inside the
// kernel, rounded to FP16 or BF16 (optionally as a hi + lo pair), and
// multiplied with v_mfma_f32_32x32x16_{f16,bf16} into FP32 accumulators; they
// never exist in HBM.
//
// Workgroup: 4 waves, a 256 x 256 output tile (wave w owns the 128 x 128 block
// (w >> 1, w & 1): 4 x 4 MFMA tiles, 256 accumulator registers per lane).  The
// points stream through in chunks of KC: for each chunk the workgroup writes the
// 256 x KC slices of Gy and Gx into LDS in the exact lane order the MFMA operand
// registers use (one 16-byte LDS word per lane and MFMA tile, conflict-free
// linear reads), double-buffered so that factor generation for chunk c + 1
// (VALU, v_exp_f32) and the MFMAs of chunk c come from the same basic block.
//
// Gaussian factors are evaluated tile-relative: with a = sqrt(log2(e)/2)/H,
// g = exp2(-(m a - (X - x0) a)^2) for node x0 + m, keeping every argument small.
// Compact kernels test |m - (X - x0)| <= H on the exact difference, as the FP32
// direct path does.
//
// Points are split across workgroups (split-K) so that a launch has about one
// workgroup per CU; per-split partial maps are added in split order by the
// reduction kernel of the direct path's file, which also applies the scale.
#include "kde_internal.h"

#include <algorithm>

namespace kde {

namespace {

constexpr int kTile = 256;     // output tile side (rows and columns)
constexpr int kThreadsSep = 256;
constexpr float kFar = 1.0e30f;

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float float8v __attribute__((ext_vector_type(8)));

template <int P>
struct PrecTraits;
template <>
struct PrecTraits<kPrecFp16> {
    static constexpr bool kSplit = false, kBf16 = false;
};
template <>
struct PrecTraits<kPrecBf16> {
    static constexpr bool kSplit = false, kBf16 = true;
};
template <>
struct PrecTraits<kPrecFp16x3> {
    static constexpr bool kSplit = true, kBf16 = false;
};
template <>
struct PrecTraits<kPrecBf16x3> {
    static constexpr bool kSplit = true, kBf16 = true;
};

struct SepLaunch {
    const float2 *pts;
    int64_t n;
    int64_t per_split;  // points per split, multiple of the chunk size
    float ax, ay;       // Gaussian argument scales sqrt(log2(e)/2)/H
    float Hx, Hy;       // compact kernels: support half-widths
    float ix, iy;       // compact kernels: 1/H
    int nx, ny, tiles_x;
    float *dst;         // final map (one split) or partials [splits][ny][nx]
    float scale;
    int64_t plane;
};

// g for a node offset m (Gaussian: pre-multiplied by a) and a tile-relative point
// coordinate pr (Gaussian: (X - x0) a; compact: X - x0).
template <int K>
__device__ __forceinline__ float sep_factor(float m, float pr, float H, float inv) {
    if constexpr (K == kGaussian) {
        const float t = m - pr;
        return __builtin_amdgcn_exp2f(-t * t);
    } else {
        const float d = m - pr;
        const float u = fminf(fabsf(d) * inv, 1.0f);
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
        } else {
            v = __builtin_amdgcn_cosf(u * 0.25f);
        }
        return fabsf(d) <= H ? v : 0.0f;
    }
}

template <bool kBf16>
__device__ __forceinline__ uint4 pack8(const float (&v)[8]) {
    uint4 r;
    if constexpr (kBf16) {
        bf16x8 h;
#pragma unroll
        for (int k = 0; k < 8; ++k) h[k] = (__bf16)v[k];
        r = __builtin_bit_cast(uint4, h);
    } else {
        half8 h;
#pragma unroll
        for (int k = 0; k < 8; ++k) h[k] = (_Float16)v[k];
        r = __builtin_bit_cast(uint4, h);
    }
    return r;
}

// Residual v - (float)round16(v), for the lo half of a split.
template <bool kBf16>
__device__ __forceinline__ void residual8(const float (&v)[8], uint4 hi, float (&lo)[8]) {
    if constexpr (kBf16) {
        const bf16x8 h = __builtin_bit_cast(bf16x8, hi);
#pragma unroll
        for (int k = 0; k < 8; ++k) lo[k] = v[k] - (float)h[k];
    } else {
        const half8 h = __builtin_bit_cast(half8, hi);
#pragma unroll
        for (int k = 0; k < 8; ++k) lo[k] = v[k] - (float)h[k];
    }
}

template <bool kBf16>
__device__ __forceinline__ f32x16 mfma(uint4 a, uint4 b, f32x16 c) {
    if constexpr (kBf16)
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b),
                                                       c, 0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(half8, a), __builtin_bit_cast(half8, b), c,
                                                      0, 0, 0);
}

template <int P>
struct SepConfig {
    static constexpr bool kSplit = PrecTraits<P>::kSplit;
    static constexpr int KC = kSplit ? 32 : 64;         // points per chunk
    static constexpr int G = KC / 8;                    // 8-point groups per chunk
    static constexpr int KK = KC / 16;                  // MFMA k-steps per chunk
    static constexpr int kWords = (kTile / 32) * KK * 64;  // 16-byte LDS words per operand slice
    static constexpr int kRowsPerThread = G;            // rows (and columns) each thread generates
    static constexpr int kRowStride = kTile / G;
};

// Generates chunk `c` of this split into LDS buffer words: A (rows, from Y) and B
// (columns, from X), hi and optionally lo.
template <int K, int P>
__device__ __forceinline__ void generate_chunk(const SepLaunch &p, int64_t beg, int64_t end, int64_t c, int tid,
                                               float x0, float y0, const float (&mrow)[SepConfig<P>::G],
                                               const float (&mcol)[SepConfig<P>::G], uint4 *Ahi, uint4 *Bhi,
                                               uint4 *Alo, uint4 *Blo) {
    using Cfg = SepConfig<P>;
    constexpr bool kBf16 = PrecTraits<P>::kBf16;
    const int g = tid % Cfg::G, s = tid / Cfg::G;
    const int64_t q0 = beg + c * Cfg::KC + 8 * g;
    float px[8], py[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const int64_t q = q0 + k;
        float2 v = make_float2(kFar, kFar);
        if (q < end) v = p.pts[q];
        if constexpr (K == kGaussian) {
            px[k] = (v.x - x0) * p.ax;
            py[k] = (v.y - y0) * p.ay;
        } else {
            px[k] = v.x - x0;
            py[k] = v.y - y0;
        }
    }
    const int kk = g >> 1, hh = g & 1;
#pragma unroll
    for (int r = 0; r < Cfg::G; ++r) {
        const int m = s + Cfg::kRowStride * r;  // row (A) and column (B) index within the tile
        const int word = ((m >> 5) * Cfg::KK + kk) * 64 + (m & 31) + 32 * hh;
        float va[8], vb[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            va[k] = sep_factor<K>(mrow[r], py[k], p.Hy, p.iy);
            vb[k] = sep_factor<K>(mcol[r], px[k], p.Hx, p.ix);
        }
        const uint4 ha = pack8<kBf16>(va), hb = pack8<kBf16>(vb);
        Ahi[word] = ha;
        Bhi[word] = hb;
        if constexpr (Cfg::kSplit) {
            float la[8], lb[8];
            residual8<kBf16>(va, ha, la);
            residual8<kBf16>(vb, hb, lb);
            Alo[word] = pack8<kBf16>(la);
            Blo[word] = pack8<kBf16>(lb);
        }
    }
}

template <int K, int P>
__global__ __launch_bounds__(kThreadsSep, 1) void sep_mfma_kernel(SepLaunch p) {
    using Cfg = SepConfig<P>;
    constexpr bool kBf16 = PrecTraits<P>::kBf16;
    constexpr int W = Cfg::kWords;
    constexpr int kOps = Cfg::kSplit ? 4 : 2;  // operand slices per buffer
    __shared__ uint4 lds[2 * kOps * W];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int tx = blockIdx.x % p.tiles_x, ty = blockIdx.x / p.tiles_x;
    const int col0 = tx * kTile, row0 = ty * kTile;
    const float x0 = (float)col0, y0 = (float)row0;

    // Node offsets of the rows/columns this thread generates.
    float mrow[Cfg::G], mcol[Cfg::G];
    {
        const int s = tid / Cfg::G;
#pragma unroll
        for (int r = 0; r < Cfg::G; ++r) {
            const float m = (float)(s + Cfg::kRowStride * r);
            if constexpr (K == kGaussian) {
                mrow[r] = m * p.ay;
                mcol[r] = m * p.ax;
            } else {
                mrow[r] = m;
                mcol[r] = m;
            }
        }
    }

    f32x16 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.0f;

    const int64_t beg = (int64_t)blockIdx.y * p.per_split;
    const int64_t end = min(p.n, beg + p.per_split);
    const int64_t nch = (end - beg + Cfg::KC - 1) / Cfg::KC;

    auto slices = [&](int buf, uint4 *&Ah, uint4 *&Bh, uint4 *&Al, uint4 *&Bl) {
        uint4 *base = lds + buf * kOps * W;
        Ah = base;
        Bh = base + W;
        Al = Cfg::kSplit ? base + 2 * W : nullptr;
        Bl = Cfg::kSplit ? base + 3 * W : nullptr;
    };

    {
        uint4 *Ah, *Bh, *Al, *Bl;
        slices(0, Ah, Bh, Al, Bl);
        generate_chunk<K, P>(p, beg, end, 0, tid, x0, y0, mrow, mcol, Ah, Bh, Al, Bl);
    }
    __syncthreads();

    const int ta0 = 4 * (wave >> 1), tb0 = 4 * (wave & 1);  // first MFMA row / column tile of this wave
    for (int64_t c = 0; c < nch; ++c) {
        const int cur = (int)(c & 1);
        {
            uint4 *Ah, *Bh, *Al, *Bl;
            slices(cur ^ 1, Ah, Bh, Al, Bl);
            generate_chunk<K, P>(p, beg, end, c + 1, tid, x0, y0, mrow, mcol, Ah, Bh, Al, Bl);
        }
        uint4 *Ah, *Bh, *Al, *Bl;
        slices(cur, Ah, Bh, Al, Bl);
#pragma unroll
        for (int kk = 0; kk < Cfg::KK; ++kk) {
            uint4 fa[4], fb[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) fa[a] = Ah[((ta0 + a) * Cfg::KK + kk) * 64 + lane];
#pragma unroll
            for (int b = 0; b < 4; ++b) fb[b] = Bh[((tb0 + b) * Cfg::KK + kk) * 64 + lane];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) acc[a][b] = mfma<kBf16>(fa[a], fb[b], acc[a][b]);
            if constexpr (Cfg::kSplit) {
                uint4 la[4], lb[4];
#pragma unroll
                for (int a = 0; a < 4; ++a) la[a] = Al[((ta0 + a) * Cfg::KK + kk) * 64 + lane];
#pragma unroll
                for (int b = 0; b < 4; ++b) lb[b] = Bl[((tb0 + b) * Cfg::KK + kk) * 64 + lane];
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int b = 0; b < 4; ++b) {
                        acc[a][b] = mfma<kBf16>(fa[a], lb[b], acc[a][b]);
                        acc[a][b] = mfma<kBf16>(la[a], fb[b], acc[a][b]);
                    }
            }
        }
        __syncthreads();
    }

    // Epilogue: register r of lane l in a 32 x 32 tile holds row 8 (r / 4) + 4 (l / 32) + r % 4,
    // column l % 32.
    float *dst = p.dst + (int64_t)blockIdx.y * p.plane;
    const float sc = gridDim.y == 1 ? p.scale : 1.0f;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int col = col0 + 32 * (tb0 + b) + (lane & 31);
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int row = row0 + 32 * (ta0 + a) + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                if (row < p.ny && col < p.nx) dst[(int64_t)row * p.nx + col] = acc[a][b][r] * sc;
            }
        }
    }
}

struct SepPlan {
    int tiles_x, tiles, splits;
    int64_t per_split;
};

SepPlan sep_plan(const MapArgs &a, int kc) {
    SepPlan pl;
    pl.tiles_x = (a.nx + kTile - 1) / kTile;
    pl.tiles = pl.tiles_x * ((a.ny + kTile - 1) / kTile);
    // One 4-wave workgroup per CU (256 CUs); at least 4 chunks per split.
    int64_t splits = std::max<int64_t>(1, 256 / pl.tiles);
    splits = std::min<int64_t>(splits, std::max<int64_t>(1, a.n / (4 * kc)));
    int64_t per = (a.n + splits - 1) / splits;
    per = (per + kc - 1) / kc * kc;
    pl.splits = (int)std::max<int64_t>(1, (a.n + per - 1) / per);
    pl.per_split = per;
    return pl;
}

template <int P>
int chunk_of() {
    return SepConfig<P>::KC;
}

int chunk_for(int precision) {
    switch (precision) {
    case kPrecFp16: return chunk_of<kPrecFp16>();
    case kPrecBf16: return chunk_of<kPrecBf16>();
    case kPrecFp16x3: return chunk_of<kPrecFp16x3>();
    default: return chunk_of<kPrecBf16x3>();
    }
}

template <int K, int P>
hipError_t launch_sep_kp(const MapArgs &a, const SepPlan &pl, float *dst, hipStream_t stream) {
    SepLaunch p;
    p.pts = a.pts;
    p.n = a.n;
    p.per_split = pl.per_split;
    p.ax = arg_scale(kGaussian, a.Hx);
    p.ay = arg_scale(kGaussian, a.Hy);
    p.Hx = a.Hx;
    p.Hy = a.Hy;
    p.ix = (float)(1.0 / (double)a.Hx);
    p.iy = (float)(1.0 / (double)a.Hy);
    p.nx = a.nx;
    p.ny = a.ny;
    p.tiles_x = pl.tiles_x;
    p.dst = dst;
    p.scale = a.scale;
    p.plane = (int64_t)a.nx * a.ny;
    hipLaunchKernelGGL((sep_mfma_kernel<K, P>), dim3(pl.tiles, pl.splits), dim3(kThreadsSep), 0, stream, p);
    return hipGetLastError();
}

template <int P>
hipError_t launch_sep_p(const MapArgs &a, const SepPlan &pl, float *dst, hipStream_t stream) {
    switch (a.kernel_id) {
    case kUniform: return launch_sep_kp<kUniform, P>(a, pl, dst, stream);
    case kTriangular: return launch_sep_kp<kTriangular, P>(a, pl, dst, stream);
    case kEpanechnikov: return launch_sep_kp<kEpanechnikov, P>(a, pl, dst, stream);
    case kQuartic: return launch_sep_kp<kQuartic, P>(a, pl, dst, stream);
    case kTriweight: return launch_sep_kp<kTriweight, P>(a, pl, dst, stream);
    case kTricube: return launch_sep_kp<kTricube, P>(a, pl, dst, stream);
    case kGaussian: return launch_sep_kp<kGaussian, P>(a, pl, dst, stream);
    case kCosine: return launch_sep_kp<kCosine, P>(a, pl, dst, stream);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

size_t sep_workspace_bytes(const MapArgs &a, int precision) {
    const SepPlan pl = sep_plan(a, chunk_for(precision));
    return pl.splits > 1 ? (size_t)pl.splits * a.nx * a.ny * sizeof(float) : 0;
}

hipError_t launch_sep(const MapArgs &a, int precision, void *ws, hipStream_t stream) {
    const SepPlan pl = sep_plan(a, chunk_for(precision));
    float *dst = pl.splits > 1 ? static_cast<float *>(ws) : a.out;
    hipError_t e;
    switch (precision) {
    case kPrecFp16: e = launch_sep_p<kPrecFp16>(a, pl, dst, stream); break;
    case kPrecBf16: e = launch_sep_p<kPrecBf16>(a, pl, dst, stream); break;
    case kPrecFp16x3: e = launch_sep_p<kPrecFp16x3>(a, pl, dst, stream); break;
    case kPrecBf16x3: e = launch_sep_p<kPrecBf16x3>(a, pl, dst, stream); break;
    default: return hipErrorInvalidValue;
    }
    if (e != hipSuccess || pl.splits == 1) return e;
    return launch_reduce_splits(static_cast<const float *>(ws), pl.splits, (int64_t)a.nx * a.ny, a.scale, a.out,
                                stream);
}

}  // namespace kde
