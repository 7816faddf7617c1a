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
// 256 x KC slices of Gy and Gx into LDS as row-major rows of 16-byte words (8
// factors each, one pad word per row so that neither the stores nor the MFMA
// fragment reads conflict on LDS banks), double-buffered in two arrays so that
// factor generation for chunk c + 1 (VALU) and the MFMAs of chunk c share a basic
// block and can interleave.
//
// Gaussian factors are evaluated tile-relative: with a = sqrt(log2(e)/2)/H,
// g = exp2(-(m a - (X - x0) a)^2) for node x0 + m, keeping every argument small.
// Compact kernels test |m - (X - x0)| <= H on the exact difference, as the FP32
// direct path does.
//
// Points are split across workgroups (split-K) so that a launch has about one
// workgroup per CU; per-split partial maps are added in split order by the
// reduction kernel of the direct path's file, which also applies the scale.
//
// Dense Gaussian maps with multiplicative runs (the common case) run an 8-wave
// variant, sep_mfma8_kernel, with two waves per SIMD; see there.
#include "kde_internal.h"
#include "kde_mfma.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

namespace kde {

namespace {

constexpr int kTile = 256;     // output tile side (rows and columns)
constexpr int kThreadsSep = 256;
constexpr float kFar = 1.0e30f;

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

// Banded work item: the points of one 256 x 256 tile's bin (or a share of
// them), copied padded to pts[pad_off ..]; its partial tile goes to slot
// (the item's index).
struct SepItem {
    int tile, pad_;
    int64_t begin;    // first point in the tile bins
    int64_t len;      // points
    int64_t pad_off;  // first point of the padded copy
};

struct SepLaunch {
    const SepItem *items;  // banded: the work item of each workgroup; nullptr: dense splits
    const int *n_items;    // banded: number of valid items (device)
    const float2 *pts;  // padded copy: split s owns [s * pad_stride, (s + 1) * pad_stride)
    int64_t n;
    int64_t per_split;  // points per split, multiple of the chunk size
    int64_t pad_stride; // per_split + 4 chunks of far-away points
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
    } else if constexpr (K == kGaussTrunc) {  // H: support 8 h; inv: the Gaussian argument scale
        const float d = m - pr, t = d * inv;
        return fabsf(d) <= H ? __builtin_amdgcn_exp2f(-t * t) : 0.0f;
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

template <int P>
struct SepConfig {
    static constexpr bool kSplit = PrecTraits<P>::kSplit;
    static constexpr int KC = kSplit ? 32 : 64;            // points per chunk
    static constexpr int G = KC / 8;                       // 8-point groups per chunk
    static constexpr int KK = KC / 16;                     // MFMA k-steps per chunk
    // Operand slice in LDS: row-major [kTile rows][G + 1] 16-byte words (8 factors
    // each); the one-word pad per row makes both the generators' stores (8
    // consecutive rows per thread, lanes varying the point group) and the MFMA
    // fragment reads (lanes varying the row) hit distinct bank groups.
    static constexpr int kRowWords = G + 1;
    static constexpr int kWords = kTile * kRowWords;  // 16-byte LDS words per operand slice
    static constexpr int R = G;                            // consecutive rows (and columns) per thread
};

// The 8 points of one group: 64 contiguous bytes of the padded copy (points
// past the split's end are far away, so every factor they produce is 0).
__device__ __forceinline__ void load_points(const float2 *q, float2 (&v)[8]) {
    const float4 *q4 = reinterpret_cast<const float4 *>(q);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float4 w = q4[k];
        v[2 * k] = make_float2(w.x, w.y);
        v[2 * k + 1] = make_float2(w.z, w.w);
    }
}

// Copies each split's points into a padded array: split s gets [s * stride,
// (s + 1) * stride), its points first, then far-away points up to the stride.
__global__ __launch_bounds__(256) void pad_points_kernel(const float2 *__restrict__ pts, int64_t n,
                                                         int64_t per_split, int64_t stride, int64_t total,
                                                         float2 *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const int64_t s = i / stride, k = i - s * stride;
    const int64_t q = s * per_split + k;
    out[i] = (k < per_split && q < n) ? pts[q] : make_float2(kFar, kFar);
}

// Writes one row (A) or column (B) of 8 factors: hi, and lo for splits.
template <int P>
__device__ __forceinline__ void put8(const float (&v)[8], uint4 *hi, uint4 *lo, int word) {
    constexpr bool kBf16 = PrecTraits<P>::kBf16;
    const uint4 h = pack8<kBf16>(v);
    hi[word] = h;
    if constexpr (PrecTraits<P>::kSplit) {
        float l[8];
        residual8<kBf16>(v, h, l);
        lo[word] = pack8<kBf16>(l);
    }
}

// Factors of one operand slice for this thread: R consecutive nodes m0 .. m0+R-1
// (rows of A or columns of B) against the 8 points `pr` (tile-relative; Gaussian
// scaled by a), each evaluated on its own.
template <int K, int P>
__device__ __forceinline__ void gen_slice(const float (&pr)[8], float m0, float a, float H, float inv, uint4 *hi,
                                          uint4 *lo, int word0, int stride) {
    constexpr int R = SepConfig<P>::R;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const float m = K == kGaussian ? m0 + (float)r * a : m0 + (float)r;
        float v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = sep_factor<K>(m, pr[k], H, inv);
        put8<P>(v, hi, lo, word0 + r * stride);
    }
}

// Generates one chunk (8 points per thread, given) into an LDS buffer: A (rows,
// from Y) and B (columns, from X).
template <int K, int P>
__device__ __forceinline__ void generate_chunk(const SepLaunch &p, const float2 (&v)[8], int tid, float x0,
                                               float y0, float mrow0, float mcol0, uint4 *Ahi, uint4 *Bhi,
                                               uint4 *Alo, uint4 *Blo) {
    using Cfg = SepConfig<P>;
    const int g = tid % Cfg::G, s = tid / Cfg::G;
    const int m = Cfg::R * s;  // first row / column of this thread; R consecutive ones, within one 32-block
    const int word0 = m * Cfg::kRowWords + g;
    float px[8], py[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        if constexpr (K == kGaussian) {
            px[k] = (v[k].x - x0) * p.ax;
            py[k] = (v[k].y - y0) * p.ay;
        } else {
            px[k] = v[k].x - x0;
            py[k] = v[k].y - y0;
        }
    }
    const float ga_y = K == kGaussian ? p.ay : 1.0f, ga_x = K == kGaussian ? p.ax : 1.0f;
    gen_slice<K, P>(py, mrow0, ga_y, p.Hy, p.iy, Ahi, Alo, word0, Cfg::kRowWords);
    gen_slice<K, P>(px, mcol0, ga_x, p.Hx, p.ix, Bhi, Blo, word0, Cfg::kRowWords);
}

// A batch of dense maps in one launch: map m owns workgroups [wg0, wg0 + tiles
// x splits) of the grid (tile fastest), found by binary search.
struct DenseEntry {
    SepLaunch p;          // dst: the map (one split) or its partial planes
    int64_t wg0;          // first workgroup of the map
    int64_t tiles;
    int splits;           // point splits of the map
    // padding: split s of the map's points -> p.pts + s * p.pad_stride
    const float2 *src;
    int64_t pad0;         // first padded point of the map in the batch's padded array
    // split reduction (maps with more than one split; 0 cells otherwise)
    int64_t red0;         // first cell of the map in the batch's reduction range
    float *out;
};

__device__ __forceinline__ int find_entry(const DenseEntry *e, int n, int64_t key, int which) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        const int64_t v = which == 0 ? e[mid].wg0 : which == 1 ? e[mid].pad0 : e[mid].red0;
        if (v <= key) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// kBatch: one launch over the maps of a DenseEntry table (dense Gaussian maps
// too narrow for multiplicative runs); p is then each workgroup's entry's.
template <int K, int P, bool kBatch>
__global__ __launch_bounds__(kThreadsSep, 1) void sep_mfma_kernel(SepLaunch p, const DenseEntry *__restrict__ batch,
                                                                 int n_batch) {
    using Cfg = SepConfig<P>;
    constexpr bool kBf16 = PrecTraits<P>::kBf16;
    constexpr int W = Cfg::kWords;
    constexpr int kOps = Cfg::kSplit ? 4 : 2;  // operand slices per buffer
    // Two separate LDS buffers, so the compiler can see that the factor stores of
    // one chunk never alias the fragment reads of the other and may interleave them.
    __shared__ uint4 lds0[kOps * W];
    __shared__ uint4 lds1[kOps * W];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // Dense: tile blockIdx.x, point split blockIdx.y.  Banded: the item's tile
    // and points (workgroups past the last item leave at once).
    bool one_split = gridDim.y == 1;  // a single point split: write the map scaled
    int bm = 0;                       // the workgroup's entry (kBatch)
    if constexpr (kBatch) {
        bm = find_entry(batch, n_batch, blockIdx.x, 0);
        p = batch[bm].p;
        one_split = batch[bm].splits == 1;
    }
    const bool banded = !kBatch && p.items != nullptr;
    int tile_idx = blockIdx.x;
    int64_t split = 0;
    int64_t count;
    const float2 *qbase;
    if constexpr (kBatch) {  // the item's tile and split, tile fastest
        const int64_t local = (int64_t)blockIdx.x - batch[bm].wg0;
        tile_idx = (int)(local % batch[bm].tiles);
        split = local / batch[bm].tiles;
        const int64_t beg = split * p.per_split;
        count = min(p.n, beg + p.per_split) - beg;
        qbase = p.pts + split * p.pad_stride;
    } else if (banded) {
        if ((int)blockIdx.x >= *p.n_items) return;
        const SepItem it = p.items[blockIdx.x];
        tile_idx = it.tile;
        count = it.len;
        qbase = p.pts + it.pad_off;
    } else {
        // Workgroups go to the 8 XCDs in turn (dispatch index mod 8), each XCD
        // with its own L2.  Numbering the (tile, split) items split-major and
        // giving each XCD one contiguous eighth of them keeps every split's points
        // in the L2s of the few XCDs that sweep it, instead of streaming every
        // split through all eight (a bijection, so any dispatch order stays correct).
        const int64_t L = blockIdx.x + (int64_t)blockIdx.y * gridDim.x, TS = (int64_t)gridDim.x * gridDim.y;
        const int64_t w = TS % 8 == 0 ? (L % 8) * (TS / 8) + L / 8 : L;
        tile_idx = (int)(w % gridDim.x);
        split = w / gridDim.x;
        const int64_t beg = split * p.per_split;
        count = min(p.n, beg + p.per_split) - beg;
        qbase = p.pts + split * p.pad_stride;
    }
    const int tx = tile_idx % p.tiles_x, ty = tile_idx / p.tiles_x;
    const int col0 = tx * kTile, row0 = ty * kTile;
    const float x0 = (float)col0, y0 = (float)row0;

    // First node offset of the rows / columns this thread generates (Gaussian:
    // pre-multiplied by a).
    const float m0 = (float)(Cfg::R * (tid / Cfg::G));
    const float mrow0 = K == kGaussian ? m0 * p.ay : m0;
    const float mcol0 = K == kGaussian ? m0 * p.ax : m0;

    f32x16 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.0f;

    // Chunks of this split, rounded up to even so that the loop below runs whole
    // pairs of steps (the padded copy holds far-away points past the end).
    const int64_t nch = ((count + Cfg::KC - 1) / Cfg::KC + 1) & ~int64_t(1);
    const float2 *qg = qbase + 8 * (tid % Cfg::G);  // this thread's group, chunk 0
    const int ta0 = 4 * (wave >> 1), tb0 = 4 * (wave & 1);  // first MFMA row / column tile of this wave
    // Fragment word of lane `lane` for MFMA tile t (32 rows) and k-step kk: row
    // 32 t + lane % 32, point group 2 kk + lane / 32.
    const int frag0 = (lane & 31) * Cfg::kRowWords + (lane >> 5);
    auto frag = [&](int t, int kk) { return frag0 + 32 * t * Cfg::kRowWords + 2 * kk; };

    float2 pts[8], nxt[8];
    load_points(qg, pts);
    load_points(qg + Cfg::KC, nxt);
    generate_chunk<K, P>(p, pts, tid, x0, y0, mrow0, mcol0, lds0, lds0 + W, lds0 + 2 * W, lds0 + 3 * W);
    __syncthreads();

    // One chunk: generate chunk c + 1 into `gen` while the MFMAs consume chunk c
    // from `use`.
    auto step = [&](int64_t c, uint4 *gen, const uint4 *use) {
#pragma unroll
        for (int k = 0; k < 8; ++k) pts[k] = nxt[k];
        load_points(qg + (c + 2) * Cfg::KC, nxt);  // consumed one chunk later
        generate_chunk<K, P>(p, pts, tid, x0, y0, mrow0, mcol0, gen, gen + W, gen + 2 * W, gen + 3 * W);
        const uint4 *Ah = use, *Bh = use + W, *Al = use + 2 * W, *Bl = use + 3 * W;
#pragma unroll
        for (int kk = 0; kk < Cfg::KK; ++kk) {
            uint4 fa[4], fb[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) fa[a] = Ah[frag(ta0 + a, kk)];
#pragma unroll
            for (int b = 0; b < 4; ++b) fb[b] = Bh[frag(tb0 + b, kk)];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) acc[a][b] = mfma<kBf16>(fa[a], fb[b], acc[a][b]);
            if constexpr (Cfg::kSplit) {
                uint4 la[4], lb[4];
#pragma unroll
                for (int a = 0; a < 4; ++a) la[a] = Al[frag(ta0 + a, kk)];
#pragma unroll
                for (int b = 0; b < 4; ++b) lb[b] = Bl[frag(tb0 + b, kk)];
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
    };

    for (int64_t c = 0; c < nch; c += 2) {
        step(c, lds1, lds0);
        step(c + 1, lds0, lds1);
    }

    // Epilogue: register r of lane l in a 32 x 32 tile holds row 8 (r / 4) + 4 (l / 32) + r % 4,
    // column l % 32.
    if (banded) {  // raw partial tile, row-major 256 x 256, in the item's slot
        float *slot = p.dst + (int64_t)blockIdx.x * (kTile * kTile);
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b)
#pragma unroll
                for (int r = 0; r < 16; ++r)
                    slot[(32 * (ta0 + a) + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3)) * kTile + 32 * (tb0 + b) +
                         (lane & 31)] = acc[a][b][r];
        return;
    }
    float *dst = p.dst + split * p.plane;
    const float sc = one_split ? p.scale : 1.0f;
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

// Dense Gaussian maps with multiplicative runs, every precision: 8 waves, two
// per SIMD, so that one wave's factor generation (VALU) overlaps the other's
// MFMAs (a single wave per SIMD issues its VALU work mostly between its own
// MFMAs and leaves the matrix core idle meanwhile).  Wave w owns the 128 x 64
// block (w / 4, w % 4) of the 256 x 256 tile: 4 x 2 MFMA tiles, 128
// accumulator registers per lane, which leaves room for two waves per SIMD.
// Threads 0-255 generate the row factors (A, from Y), threads 256-511 the
// column factors (B, from X): per chunk one R-node run of 8 points each (R = 8
// single, 4 for the hi/lo splits, whose chunks are half as long).  Every phase
// (one MFMA k-step) emits R / KK rows of the next chunk's run and starts 8 / KK
// points of the run after it, so the VALU work is spread evenly over the
// phases; single precision reads the fragments of phase kk + 1 during phase kk
// (the splits have no registers left for that).  Same LDS layout, chunking,
// split-K and tile order as sep_mfma_kernel; the point loads run three chunks
// ahead (the padded copy holds four chunks of far-away points past each split).
// kBatch: the launch runs the (tile, split) items of several maps, each
// workgroup taking its map's arguments from a table (DenseEntry) instead of the
// kernel argument; every map is split and summed as its own launch would.
constexpr int kThreads8 = 512;

// The entry of element i, starting from entry m (elements of a workgroup lie in
// one or a few consecutive entries: one search per workgroup, then steps).
__device__ __forceinline__ int advance_entry(const DenseEntry *e, int n, int64_t i, int m, int which) {
    while (m + 1 < n && (which == 1 ? e[m + 1].pad0 : e[m + 1].red0) <= i) ++m;
    return m;
}

// pad_points_kernel over every map of the batch.
__global__ __launch_bounds__(256) void pad_batch_kernel(const DenseEntry *__restrict__ e, int n, int64_t total,
                                                        float2 *__restrict__ padded) {
    __shared__ int s_m;
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x, i = i0 + threadIdx.x;
    if (threadIdx.x == 0) s_m = find_entry(e, n, i0, 1);
    __syncthreads();
    if (i >= total) return;
    const int m = advance_entry(e, n, i, s_m, 1);
    const SepLaunch &p = e[m].p;
    const int64_t k0 = i - e[m].pad0, s = k0 / p.pad_stride, k = k0 - s * p.pad_stride;
    const int64_t q = s * p.per_split + k;
    padded[i] = (k < p.per_split && q < p.n) ? e[m].src[q] : make_float2(kFar, kFar);
}

// reduce_splits_kernel over the maps of the batch with more than one split,
// kReduceCells cells per workgroup.
constexpr int kReduceCells = 1024;

__global__ __launch_bounds__(256) void reduce_batch_kernel(const DenseEntry *__restrict__ e, int n, int64_t total) {
    __shared__ int s_m;
    const int64_t i0 = (int64_t)blockIdx.x * kReduceCells;
    if (threadIdx.x == 0) s_m = find_entry(e, n, i0, 2);
    __syncthreads();
    int m = s_m;
    for (int r = 0; r < kReduceCells / 256; ++r) {
        const int64_t i = i0 + r * 256 + threadIdx.x;
        if (i >= total) return;
        m = advance_entry(e, n, i, m, 2);
        const SepLaunch &p = e[m].p;
        const int64_t c = i - e[m].red0;
        const int splits = e[m].splits;
        float v = 0.0f;
#pragma unroll 8
        for (int k = 0; k < splits; ++k) v += p.dst[(int64_t)k * p.plane + c];
        e[m].out[c] = v * p.scale;
    }
}

template <int P, bool kBatch>
__global__ __launch_bounds__(kThreads8, 1) void sep_mfma8_kernel(SepLaunch p, const DenseEntry *__restrict__ batch,
                                                                  int n_batch) {
    using Cfg = SepConfig<P>;
    constexpr bool kSplit = Cfg::kSplit;
    constexpr bool kBf16 = PrecTraits<P>::kBf16;
    constexpr int W = Cfg::kWords;
    constexpr int KK = Cfg::KK;
    constexpr int kOps = kSplit ? 4 : 2;       // operand slices per buffer (hi, and lo for splits)
    constexpr int kRowsPh = Cfg::R / KK;       // run rows emitted per phase
    constexpr int kPtsPh = 8 / KK;             // points of the next run started per phase
    static_assert(Cfg::R == kRowsPh * KK && 8 == kPtsPh * KK, "even spread over the phases");
    __shared__ uint4 lds0[kOps * W];
    __shared__ uint4 lds1[kOps * W];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    int tile_idx;
    int64_t split;
    bool one_split;  // the map has a single point split: write it scaled
    if constexpr (kBatch) {  // the item's map, tile and split from the batch table
        const int m = find_entry(batch, n_batch, blockIdx.x, 0);
        p = batch[m].p;
        const int64_t local = (int64_t)blockIdx.x - batch[m].wg0;
        tile_idx = (int)(local % batch[m].tiles);
        split = local / batch[m].tiles;
        one_split = batch[m].splits == 1;
    } else {
        // XCD-aware order of the (tile, split) items, as in sep_mfma_kernel.
        const int64_t L = blockIdx.x + (int64_t)blockIdx.y * gridDim.x, TS = (int64_t)gridDim.x * gridDim.y;
        const int64_t wl = TS % 8 == 0 ? (L % 8) * (TS / 8) + L / 8 : L;
        tile_idx = (int)(wl % gridDim.x);
        split = wl / gridDim.x;
        one_split = gridDim.y == 1;
    }
    const int64_t beg = split * p.per_split;
    const int64_t count = min(p.n, beg + p.per_split) - beg;
    const float2 *qbase = p.pts + split * p.pad_stride;
    const int tx = tile_idx % p.tiles_x, ty = tile_idx / p.tiles_x;
    const int col0 = tx * kTile, row0 = ty * kTile;

    // Generation role: A (rows, Y) for threads 0-255, B (columns, X) for 256-511.
    const bool genB = tid >= 256;
    const int gt = tid & 255;
    const int g8 = gt % Cfg::G, mrun = Cfg::R * (gt / Cfg::G);
    const float a = genB ? p.ax : p.ay;
    const float origin = genB ? (float)col0 : (float)row0;
    const float m0 = (float)mrun * a;
    const int word0 = mrun * Cfg::kRowWords + g8;
    const int slice = genB ? W : 0;  // hi slice; lo (splits) at slice + 2 W
    const float mc = m0 + 0.5f * (float)(Cfg::R - 1) * a, span = (float)(Cfg::R - 1) * a;

    f32x16 acc[4][2];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;

    const int64_t nch = ((count + Cfg::KC - 1) / Cfg::KC + 1) & ~int64_t(1);
    const float2 *qg = qbase + 8 * g8;
    const int ta0 = 4 * (wave >> 2), tb0 = 2 * (wave & 3);  // first 32-row / 32-column MFMA tile
    const int frag0 = (lane & 31) * Cfg::kRowWords + (lane >> 5);
    auto frag = [&](int t, int kk) { return frag0 + 32 * t * Cfg::kRowWords + 2 * kk; };

    // This thread's coordinate of 8 points, scaled and tile-relative.
    auto coords = [&](const float2 (&v)[8], float (&pc)[8]) {
#pragma unroll
        for (int k = 0; k < 8; ++k) pc[k] = ((genB ? v[k].x : v[k].y) - origin) * a;
    };
    // Gaussian runs.  With the run centre c = m0 + (R-1)/2, t_c = (c - X) a and
    // offsets rho_r = r - (R-1)/2,
    //     g(m0 + r) = exp2(-(t_c + rho_r a)^2) = P_r q_r,
    //     P_r = exp2(-t_c^2 - 2 t_c a rho_r),   q_r = exp2(-(rho_r a)^2).
    // q_r depends only on the node's position in its run (row or column index
    // mod R), so it factors out of the contraction and is applied once per
    // output in the epilogue; the operands carry P_r = P_0 B^r, B = exp2(-2 a
    // t_c): two exp2 per point and run, then one multiply per factor.  P_r <= g
    // q_r^-1 <= 2^((R-1)^2 a^2 / 4) stays inside FP16 range for a <= 0.8; a start
    // value P_0 that underflows implies every factor of the run is below 2^-31 of
    // the peak, and B is clamped to stay finite, so a run never turns a zero into
    // a non-zero or produces NaN.
    // start_pts: the run start for points k0 .. k1-1; emit: one row, then the
    // next row's values.
    auto start_pts = [&](float (&e)[8], float (&ratio)[8], const float (&pc)[8], int k0, int k1) {
#pragma unroll
        for (int k = k0; k < k1; ++k) {
            const float tc = mc - pc[k];
            e[k] = __builtin_amdgcn_exp2f(tc * (span - tc));
            ratio[k] = __builtin_amdgcn_exp2f(fminf(-2.0f * a * tc, 126.0f));
        }
    };
    auto emit = [&](float (&e)[8], const float (&ratio)[8], uint4 *buf, int word) {
        put8<P>(e, buf + slice, buf + slice + 2 * W, word);
#pragma unroll
        for (int k = 0; k < 8; ++k) e[k] *= ratio[k];
    };

    float2 raw[8];  // points of the chunk whose run starts next
    float eA[8], rA[8], eB[8], rB[8];
    {
        float2 v[8];
        float pc[8];
        load_points(qg, v);
        coords(v, pc);
        start_pts(eA, rA, pc, 0, 8);
#pragma unroll
        for (int r = 0; r < Cfg::R; ++r) emit(eA, rA, lds0, word0 + r * Cfg::kRowWords);
        load_points(qg + Cfg::KC, v);
        coords(v, pc);
        start_pts(eA, rA, pc, 0, 8);          // chunk 1's run
        load_points(qg + 2 * Cfg::KC, raw);  // chunk 2's points
    }
    __syncthreads();

    // Step c: MFMAs on chunk c (use), emission of chunk c + 1 (run e, r) into
    // gen, start of chunk c + 2's run (en, rn); raw then takes chunk c + 3.
    auto step = [&](int64_t c, uint4 *gen, const uint4 *use, float (&e)[8], float (&r)[8], float (&en)[8],
                    float (&rn)[8]) {
        float pc[8];
        coords(raw, pc);
        load_points(qg + (c + 3) * Cfg::KC, raw);
        const uint4 *Ah = use, *Bh = use + W, *Al = use + 2 * W, *Bl = use + 3 * W;
        uint4 na[4], nb[2];
        if constexpr (!kSplit) {
#pragma unroll
            for (int i = 0; i < 4; ++i) na[i] = Ah[frag(ta0 + i, 0)];
#pragma unroll
            for (int j = 0; j < 2; ++j) nb[j] = Bh[frag(tb0 + j, 0)];
        }
#pragma unroll
        for (int kk = 0; kk < KK; ++kk) {
            uint4 fa[4], fb[2];
            if constexpr (!kSplit) {
#pragma unroll
                for (int i = 0; i < 4; ++i) fa[i] = na[i];
#pragma unroll
                for (int j = 0; j < 2; ++j) fb[j] = nb[j];
                if (kk + 1 < KK) {
#pragma unroll
                    for (int i = 0; i < 4; ++i) na[i] = Ah[frag(ta0 + i, kk + 1)];
#pragma unroll
                    for (int j = 0; j < 2; ++j) nb[j] = Bh[frag(tb0 + j, kk + 1)];
                }
            } else {
#pragma unroll
                for (int i = 0; i < 4; ++i) fa[i] = Ah[frag(ta0 + i, kk)];
#pragma unroll
                for (int j = 0; j < 2; ++j) fb[j] = Bh[frag(tb0 + j, kk)];
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) acc[i][j] = mfma<kBf16>(fa[i], fb[j], acc[i][j]);
            if constexpr (kSplit) {
                uint4 la[4], lb[2];
#pragma unroll
                for (int i = 0; i < 4; ++i) la[i] = Al[frag(ta0 + i, kk)];
#pragma unroll
                for (int j = 0; j < 2; ++j) lb[j] = Bl[frag(tb0 + j, kk)];
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 2; ++j) {
                        acc[i][j] = mfma<kBf16>(fa[i], lb[j], acc[i][j]);
                        acc[i][j] = mfma<kBf16>(la[i], fb[j], acc[i][j]);
                    }
            }
#pragma unroll
            for (int q = 0; q < kRowsPh; ++q) emit(e, r, gen, word0 + (kRowsPh * kk + q) * Cfg::kRowWords);
            start_pts(en, rn, pc, kPtsPh * kk, kPtsPh * (kk + 1));
            __builtin_amdgcn_sched_barrier(0);
        }
        __syncthreads();
    };
    for (int64_t c = 0; c < nch; c += 2) {
        step(c, lds1, lds0, eA, rA, eB, rB);
        step(c + 1, lds0, lds1, eB, rB, eA, rA);
    }

    // Epilogue: register r of lane l in a 32 x 32 tile holds row 8 (r / 4) + 4 (l / 32) + r % 4,
    // column l % 32; the runs' position factors q(row mod 8) q(column mod 8).
    float *dst = p.dst + split * p.plane;
    const float sc = one_split ? p.scale : 1.0f;
    constexpr float hc = 0.5f * (float)(Cfg::R - 1);
    const float rcq = ((float)(lane % Cfg::R) - hc) * p.ax;
    const float qcol = __builtin_amdgcn_exp2f(-rcq * rcq);
    float qrow[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const float rr = ((float)((4 * (lane >> 5) + r) % Cfg::R) - hc) * p.ay;
        qrow[r] = __builtin_amdgcn_exp2f(-rr * rr);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int col = col0 + 32 * (tb0 + j) + (lane & 31);
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int row = row0 + 32 * (ta0 + i) + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                if (row < p.ny && col < p.nx)
                    dst[(int64_t)row * p.nx + col] = acc[i][j][r] * (qrow[r & 3] * qcol * sc);
            }
        }
    }
}

struct SepPlan {
    int tiles_x, tiles, splits;
    int64_t per_split;
    int64_t pad_stride;   // padded points per split
    size_t partial_bytes; // split partial planes (0 with one split), 256-byte aligned
};

// max_splits caps the point splits (maps of a batch, which fill the GPU together).
SepPlan sep_plan(const MapArgs &a, int kc, int64_t max_splits = INT64_MAX) {
    SepPlan pl;
    pl.tiles_x = (a.nx + kTile - 1) / kTile;
    pl.tiles = pl.tiles_x * ((a.ny + kTile - 1) / kTile);
    // One 4-wave workgroup per CU (256 CUs); at least 4 chunks per split.
    int64_t splits = std::max<int64_t>(1, 256 / pl.tiles);
    splits = std::min<int64_t>(splits, std::max<int64_t>(1, a.n / (4 * kc)));
    splits = std::max<int64_t>(1, std::min<int64_t>(splits, max_splits));
    int64_t per = (a.n + splits - 1) / splits;
    per = (per + kc - 1) / kc * kc;
    pl.splits = (int)std::max<int64_t>(1, (a.n + per - 1) / per);
    pl.per_split = per;
    // Four extra chunks: the chunk count is rounded up to even and the point
    // loads run up to three chunks ahead of the MFMAs (sep_mfma8_kernel).
    pl.pad_stride = per + 4 * kc;
    pl.partial_bytes = pl.splits > 1 ? ((size_t)pl.splits * a.nx * a.ny * sizeof(float) + 255) / 256 * 256 : 0;
    return pl;
}

size_t padded_bytes(const SepPlan &pl) { return (size_t)pl.splits * pl.pad_stride * sizeof(float2); }

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

// Banded launch: one workgroup per possible item.
struct BandedItems {
    const SepItem *items;
    const int *n_items;
    int max_items;
};

template <int K, int P>
hipError_t launch_sep_kp(const MapArgs &a, const SepPlan &pl, const float2 *padded, float *dst,
                         hipStream_t stream, const BandedItems *bi = nullptr) {
    SepLaunch p;
    p.pts = padded;
    p.n = a.n;
    p.per_split = pl.per_split;
    p.pad_stride = pl.pad_stride;
    p.items = bi ? bi->items : nullptr;
    p.n_items = bi ? bi->n_items : nullptr;
    const dim3 grid = bi ? dim3((unsigned)bi->max_items, 1) : dim3(pl.tiles, pl.splits);
    p.ax = arg_scale(kGaussian, a.Hx);
    p.ay = arg_scale(kGaussian, a.Hy);
    p.Hx = a.Hx;
    p.Hy = a.Hy;
    p.ix = (float)(1.0 / (double)a.Hx);
    p.iy = (float)(1.0 / (double)a.Hy);
    if constexpr (K == kGaussTrunc) {  // support in H, Gaussian argument scale in ix, iy
        p.ix = a.ax;
        p.iy = a.ay;
    }
    p.nx = a.nx;
    p.ny = a.ny;
    p.tiles_x = pl.tiles_x;
    p.dst = dst;
    p.scale = a.scale;
    p.plane = (int64_t)a.nx * a.ny;
    // The Gaussian's multiplicative runs need a <= 0.8 (H >= 1.05 px); narrower
    // bandwidths evaluate every factor with its own exp2.
    bool recur = false;
    if constexpr (K == kGaussian) recur = p.ax <= kMaxRunScale && p.ay <= kMaxRunScale;
    // (The full Gaussian is never banded: only compact supports and the truncated
    // Gaussian are, so a dense launch is the only one with runs.)
    if constexpr (K == kGaussian) {
        if (recur && bi == nullptr) {  // the 8-wave kernel
            main_kernel_begin(stream);
            hipLaunchKernelGGL((sep_mfma8_kernel<P, false>), grid, dim3(kThreads8), 0, stream, p,
                               static_cast<const DenseEntry *>(nullptr), 0);
            main_kernel_end(stream);
            return hipGetLastError();
        }
    }
    main_kernel_begin(stream);
    hipLaunchKernelGGL((sep_mfma_kernel<K, P, false>), grid, dim3(kThreadsSep), 0, stream, p,
                       static_cast<const DenseEntry *>(nullptr), 0);
    main_kernel_end(stream);
    return hipGetLastError();
}

template <int P>
hipError_t launch_sep_p(const MapArgs &a, const SepPlan &pl, const float2 *padded, float *dst,
                        hipStream_t stream, const BandedItems *bi = nullptr) {
    switch (a.kernel_id) {
    case kUniform: return launch_sep_kp<kUniform, P>(a, pl, padded, dst, stream, bi);
    case kTriangular: return launch_sep_kp<kTriangular, P>(a, pl, padded, dst, stream, bi);
    case kEpanechnikov: return launch_sep_kp<kEpanechnikov, P>(a, pl, padded, dst, stream, bi);
    case kQuartic: return launch_sep_kp<kQuartic, P>(a, pl, padded, dst, stream, bi);
    case kTriweight: return launch_sep_kp<kTriweight, P>(a, pl, padded, dst, stream, bi);
    case kTricube: return launch_sep_kp<kTricube, P>(a, pl, padded, dst, stream, bi);
    case kGaussian: return launch_sep_kp<kGaussian, P>(a, pl, padded, dst, stream, bi);
    case kCosine: return launch_sep_kp<kCosine, P>(a, pl, padded, dst, stream, bi);
    case kGaussTrunc: return launch_sep_kp<kGaussTrunc, P>(a, pl, padded, dst, stream, bi);
    default: return hipErrorInvalidValue;
    }
}

template <int P>
hipError_t launch_sep_prec(int precision, const MapArgs &a, const SepPlan &pl, const float2 *padded, float *dst,
                           hipStream_t stream, const BandedItems *bi) {
    (void)precision;
    return launch_sep_p<P>(a, pl, padded, dst, stream, bi);
}

hipError_t launch_sep_any(int precision, const MapArgs &a, const SepPlan &pl, const float2 *padded, float *dst,
                          hipStream_t stream, const BandedItems *bi = nullptr) {
    switch (precision) {
    case kPrecFp16: return launch_sep_p<kPrecFp16>(a, pl, padded, dst, stream, bi);
    case kPrecBf16: return launch_sep_p<kPrecBf16>(a, pl, padded, dst, stream, bi);
    case kPrecFp16x3: return launch_sep_p<kPrecFp16x3>(a, pl, padded, dst, stream, bi);
    case kPrecBf16x3: return launch_sep_p<kPrecBf16x3>(a, pl, padded, dst, stream, bi);
    default: return hipErrorInvalidValue;
    }
}

// ------------------------------------------------------------------ banded path
// Compact supports (and the truncated Gaussian) reach few 256 x 256 tiles, so
// instead of every tile streaming every point, the points are binned by tile
// (support binning at tile side 256), each tile's bin is cut into items of
// about equal length (so that about kBandTarget workgroups share the work) and
// padded like a dense split, the contraction kernel runs one workgroup per item
// writing a raw partial tile, and a last pass adds each tile's partials in item
// order and applies the scale.  Every sum keeps a fixed order: deterministic.

constexpr int kBandTarget = 256;  // items aimed at (one workgroup per CU)

__host__ __device__ inline int64_t band_padded_len(int64_t len, int kc) {
    return ((((len + kc - 1) / kc) + 1) & ~int64_t(1)) * kc + 2 * kc;
}

// One workgroup: tile counts from the bin ends, the points per item, the items
// (tile-major), each tile's first item and item count, the padded offsets.
__global__ __launch_bounds__(256) void band_assign_kernel(const unsigned *__restrict__ end, int64_t wblocks, int tiles,
                                                          int kc, SepItem *__restrict__ items,
                                                          int *__restrict__ first_item, int *__restrict__ nsplit,
                                                          int *__restrict__ n_items) {
    __shared__ long long sh[256];
    __shared__ long long s_per;
    const int tid = threadIdx.x;
    const int t0 = (int)((int64_t)tiles * tid / 256), t1 = (int)((int64_t)tiles * (tid + 1) / 256);
    auto bin_begin = [&](int t) -> int64_t { return t > 0 ? (int64_t)end[(int64_t)t * wblocks - 1] : 0; };
    auto bin_end = [&](int t) -> int64_t { return (int64_t)end[(int64_t)t * wblocks + wblocks - 1]; };
    long long local = 0;
    for (int t = t0; t < t1; ++t) local += bin_end(t) - bin_begin(t);
    sh[tid] = local;
    __syncthreads();
    if (tid == 0) {
        long long tot = 0;
        for (int k = 0; k < 256; ++k) tot += sh[k];
        long long per = (tot + kBandTarget - 1) / kBandTarget;
        per = (per + kc - 1) / kc * kc;
        s_per = per < 4 * kc ? 4 * kc : per;
    }
    __syncthreads();
    const long long per = s_per;
    auto splits_of = [&](int64_t c) -> int64_t { return c == 0 ? 0 : (c + per - 1) / per; };
    local = 0;
    for (int t = t0; t < t1; ++t) local += splits_of(bin_end(t) - bin_begin(t));
    __syncthreads();
    sh[tid] = local;
    __syncthreads();
    if (tid == 0) {  // exclusive scan of the item counts
        long long run = 0;
        for (int k = 0; k < 256; ++k) {
            const long long v = sh[k];
            sh[k] = run;
            run += v;
        }
        *n_items = (int)run;
    }
    __syncthreads();
    int64_t item = sh[tid];
    long long padded = 0;
    for (int t = t0; t < t1; ++t) {
        const int64_t b = bin_begin(t), c = bin_end(t) - b, ns = splits_of(c);
        first_item[t] = (int)item;
        nsplit[t] = (int)ns;
        for (int64_t q = 0; q < ns; ++q) {
            SepItem it;
            it.tile = t;
            it.pad_ = 0;
            it.begin = b + c * q / ns;
            it.len = b + c * (q + 1) / ns - it.begin;
            it.pad_off = padded;  // local for now
            items[item + q] = it;
            padded += band_padded_len(it.len, kc);
        }
        item += ns;
    }
    __syncthreads();
    sh[tid] = padded;
    __syncthreads();
    if (tid == 0) {
        long long run = 0;
        for (int k = 0; k < 256; ++k) {
            const long long v = sh[k];
            sh[k] = run;
            run += v;
        }
    }
    __syncthreads();
    const long long base = sh[tid];
    for (int64_t i = (t0 < t1 ? first_item[t0] : 0), e = item; t0 < t1 && i < e; ++i) items[i].pad_off += base;
}

// One workgroup per item slot: the item's points then far-away points.
__global__ __launch_bounds__(256) void band_pad_kernel(const SepItem *__restrict__ items, const int *__restrict__ n_items,
                                                       const float2 *__restrict__ bins, int kc,
                                                       float2 *__restrict__ out) {
    if ((int)blockIdx.x >= *n_items) return;
    const SepItem it = items[blockIdx.x];
    const int64_t plen = band_padded_len(it.len, kc);
    for (int64_t k = threadIdx.x; k < plen; k += blockDim.x)
        out[it.pad_off + k] = k < it.len ? bins[it.begin + k] : make_float2(kFar, kFar);
}

// out[j][i] = scale * sum of the tile's partials (items in order), 0 for tiles without points.
__global__ __launch_bounds__(256) void band_reduce_kernel(const float *__restrict__ part,
                                                          const int *__restrict__ first_item,
                                                          const int *__restrict__ nsplit, int nx, int ny, int tiles_x,
                                                          float scale, float *__restrict__ out) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)nx * ny) return;
    const int j = (int)(idx / nx), i = (int)(idx % nx);
    const int t = (j / kTile) * tiles_x + i / kTile;
    const int64_t loc = (int64_t)(j % kTile) * kTile + i % kTile;
    const int f = first_item[t], ns = nsplit[t];
    float s = 0.0f;
    for (int k = 0; k < ns; ++k) s += part[(int64_t)(f + k) * (kTile * kTile) + loc];
    out[idx] = s * scale;
}

struct BandPlan {
    int tiles, tiles_x, max_items, kc;
    size_t bins_bytes, items_off, first_off, nsplit_off, nitems_off, padded_off, part_off, total;
};

size_t align256z(size_t x) { return (x + 255) / 256 * 256; }

BandPlan band_plan(const MapArgs &a, int kc) {
    BandPlan b;
    b.kc = kc;
    b.tiles_x = (a.nx + kTile - 1) / kTile;
    b.tiles = b.tiles_x * ((a.ny + kTile - 1) / kTile);
    b.max_items = b.tiles + kBandTarget;
    b.bins_bytes = align256z(tile_bins_bytes(a, kTile));
    // registrations per point: at most 3 x 3 tiles (support <= tile side)
    const int64_t entries = std::min<int64_t>(a.n * 9, a.n * (int64_t)b.tiles);
    b.items_off = b.bins_bytes;
    b.first_off = b.items_off + align256z((size_t)b.max_items * sizeof(SepItem));
    b.nsplit_off = b.first_off + align256z((size_t)b.tiles * sizeof(int));
    b.nitems_off = b.nsplit_off + align256z((size_t)b.tiles * sizeof(int));
    b.padded_off = b.nitems_off + 256;
    b.part_off = b.padded_off + align256z((size_t)(entries + (int64_t)b.max_items * 4 * kc) * sizeof(float2));
    b.total = b.part_off + (size_t)b.max_items * kTile * kTile * sizeof(float);
    return b;
}

bool banded_applies(const MapArgs &a) {
    if (a.kernel_id == kGaussian || a.n < 1) return false;  // the full Gaussian reaches every tile
    return a.Hx <= (float)kTile && a.Hy <= (float)kTile && tile_bins_fit(a, kTile);
}

hipError_t launch_sep_banded(const MapArgs &a, int precision, void *ws, hipStream_t s) {
    const int kc = chunk_for(precision);
    const BandPlan b = band_plan(a, kc);
    char *w = static_cast<char *>(ws);
    TileBins tb;
    hipError_t e = launch_tile_bins(a, kTile, w, s, &tb);
    if (e != hipSuccess) return e;
    SepItem *items = reinterpret_cast<SepItem *>(w + b.items_off);
    int *first_item = reinterpret_cast<int *>(w + b.first_off);
    int *nsplit = reinterpret_cast<int *>(w + b.nsplit_off);
    int *n_items = reinterpret_cast<int *>(w + b.nitems_off);
    float2 *padded = reinterpret_cast<float2 *>(w + b.padded_off);
    float *part = reinterpret_cast<float *>(w + b.part_off);
    hipLaunchKernelGGL(band_assign_kernel, dim3(1), dim3(256), 0, s, tb.end, tb.wblocks, b.tiles, kc, items,
                       first_item, nsplit, n_items);
    hipLaunchKernelGGL(band_pad_kernel, dim3((unsigned)b.max_items), dim3(256), 0, s, items,
                       static_cast<const int *>(n_items), tb.bins, kc, padded);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    SepPlan pl{};
    pl.tiles_x = b.tiles_x;
    pl.tiles = b.tiles;
    pl.splits = 1;
    const BandedItems bi{items, n_items, b.max_items};
    e = launch_sep_any(precision, a, pl, padded, part, s, &bi);
    if (e != hipSuccess) return e;
    const int64_t cells = (int64_t)a.nx * a.ny;
    hipLaunchKernelGGL(band_reduce_kernel, dim3((unsigned)((cells + 255) / 256)), dim3(256), 0, s,
                       static_cast<const float *>(part), static_cast<const int *>(first_item),
                       static_cast<const int *>(nsplit), a.nx, a.ny, b.tiles_x, a.scale, a.out);
    return hipGetLastError();
}

}  // namespace

size_t sep_workspace_bytes(const MapArgs &a, int precision) {
    if (banded_applies(a)) return band_plan(a, chunk_for(precision)).total;
    const SepPlan pl = sep_plan(a, chunk_for(precision));
    return pl.partial_bytes + padded_bytes(pl);
}

// ------------------------------------------------------------------ dense batches

namespace {

// Library-owned pinned staging for the batch tables: a ring of kStageSlots
// buffers per device, each with an event marking the completion of the last
// copy out of it, so that a call waits only for the copy issued kStageSlots
// calls earlier.
constexpr int kStageSlots = 4;
struct DenseStage {
    char *host = nullptr;
    size_t cap = 0;
    hipEvent_t done = nullptr;
};
struct DenseRing {
    DenseStage slot[kStageSlots];
    int next = 0;
};
std::mutex g_stage_mu;
std::map<int, DenseRing> g_stage;

struct DenseLayout {
    std::vector<DenseEntry> entries;
    int64_t wgs = 0, padded = 0, cells = 0;
    size_t table_bytes = 0, padded_off = 0, part_off = 0, total = 0;
};

// Point splits in a batch: the maps fill the GPU together, so a map is split
// only as far as its share of the batch's (point, tile) work asks for, about
// kBatchWgs workgroups in all, never further than alone (split partial planes
// cost a write and a read of the map each).
constexpr int64_t kBatchWgs = 1024;

DenseLayout dense_layout(const MapArgs *maps, int n, int precision) {
    DenseLayout L;
    const int kc = chunk_for(precision);
    L.entries.resize(n);
    double work = 0.0;  // (point, tile) pairs of the batch
    for (int m = 0; m < n; ++m) work += (double)maps[m].n * (double)sep_plan(maps[m], kc).tiles;
    // Points per workgroup: the batch's share of kBatchWgs workgroups, raised
    // until the rounding of the splits leaves at most kBatchWgs of them (one
    // workgroup per CU at a time: a few past a multiple of the CU count would
    // run as a nearly empty last round).
    double per_wg = std::max(4.0 * kc, work / (double)kBatchWgs);
    std::vector<SepPlan> plans(n);
    for (int pass = 0; pass < 64; ++pass) {
        int64_t wgs = 0;
        for (int m = 0; m < n; ++m) {
            plans[m] = sep_plan(maps[m], kc, (int64_t)std::ceil((double)maps[m].n / per_wg));
            wgs += (int64_t)plans[m].tiles * plans[m].splits;
        }
        if (wgs <= kBatchWgs) break;
        per_wg *= 1.03;
    }
    std::vector<int> order(n);
    for (int m = 0; m < n; ++m) order[m] = m;
    // Workgroups are dispatched in index order: the maps with the longest
    // workgroups (most points per split) first, the short ones fill the tail.
    std::stable_sort(order.begin(), order.end(),
                     [&](int x, int y) { return plans[x].per_split > plans[y].per_split; });
    size_t part = 0;
    for (int k = 0; k < n; ++k) {
        const int m = order[k];
        const MapArgs &a = maps[m];
        const SepPlan &pl = plans[m];
        DenseEntry &e = L.entries[k];
        e.wg0 = L.wgs;
        e.tiles = pl.tiles;
        L.wgs += (int64_t)pl.tiles * pl.splits;
        e.src = a.pts;
        e.pad0 = L.padded;
        L.padded += (int64_t)pl.splits * pl.pad_stride;
        e.red0 = L.cells;
        if (pl.splits > 1) L.cells += (int64_t)a.nx * a.ny;
        e.out = a.out;
        SepLaunch &p = e.p;
        p = SepLaunch{};
        p.n = a.n;
        p.per_split = pl.per_split;
        p.pad_stride = pl.pad_stride;
        p.ax = arg_scale(kGaussian, a.Hx);
        p.ay = arg_scale(kGaussian, a.Hy);
        p.Hx = a.Hx;
        p.Hy = a.Hy;
        p.ix = (float)(1.0 / (double)a.Hx);
        p.iy = (float)(1.0 / (double)a.Hy);
        p.nx = a.nx;
        p.ny = a.ny;
        p.tiles_x = pl.tiles_x;
        p.scale = a.scale;
        p.plane = (int64_t)a.nx * a.ny;
        e.splits = pl.splits;
        p.pts = reinterpret_cast<const float2 *>((uintptr_t)e.pad0);  // offsets until the base is known
        p.dst = pl.splits > 1 ? reinterpret_cast<float *>((uintptr_t)part) : a.out;
        part += pl.partial_bytes;
    }
    L.table_bytes = ((size_t)n * sizeof(DenseEntry) + 255) / 256 * 256;
    L.padded_off = L.table_bytes;
    L.part_off = L.padded_off + (((size_t)L.padded * sizeof(float2) + 255) / 256 * 256);
    L.total = L.part_off + part;
    return L;
}

template <int P>
hipError_t launch_dense_batch_p(const DenseEntry *dev, int n, const DenseLayout &L, bool runs, hipStream_t s) {
    if (runs)
        hipLaunchKernelGGL((sep_mfma8_kernel<P, true>), dim3((unsigned)L.wgs), dim3(kThreads8), 0, s, SepLaunch{},
                           dev, n);
    else
        hipLaunchKernelGGL((sep_mfma_kernel<kGaussian, P, true>), dim3((unsigned)L.wgs), dim3(kThreadsSep), 0, s,
                           SepLaunch{}, dev, n);
    return hipGetLastError();
}

}  // namespace

int sep_dense_batchable(const MapArgs &a) {
    if (a.kernel_id != kGaussian || a.n <= 0) return 0;
    return arg_scale(kGaussian, a.Hx) <= kMaxRunScale && arg_scale(kGaussian, a.Hy) <= kMaxRunScale ? 1 : 2;
}

size_t sep_dense_batch_bytes(const MapArgs *maps, int n, int precision) {
    return n > 0 ? dense_layout(maps, n, precision).total : 0;
}

hipError_t launch_sep_dense_batch(const MapArgs *maps, int n, int precision, bool runs, void *ws, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    DenseLayout L = dense_layout(maps, n, precision);
    char *w = static_cast<char *>(ws);
    for (DenseEntry &e : L.entries) {  // offsets -> device addresses
        e.p.pts = reinterpret_cast<const float2 *>(w + L.padded_off) + (uintptr_t)e.p.pts;
        if (e.splits > 1) e.p.dst = reinterpret_cast<float *>(w + L.part_off + (uintptr_t)e.p.dst);
    }
    int dev = 0;
    hipError_t err = hipGetDevice(&dev);
    if (err != hipSuccess) return err;
    const size_t bytes = (size_t)n * sizeof(DenseEntry);
    {
        std::lock_guard<std::mutex> lock(g_stage_mu);
        DenseRing &ring = g_stage[dev];
        DenseStage &st = ring.slot[ring.next];
        ring.next = (ring.next + 1) % kStageSlots;
        if (st.done == nullptr && (err = hipEventCreateWithFlags(&st.done, hipEventDisableTiming)) != hipSuccess)
            return err;
        if ((err = hipEventSynchronize(st.done)) != hipSuccess) return err;  // the last copy has read the buffer
        if (st.cap < bytes) {
            if (st.host) (void)hipHostFree(st.host);
            st.host = nullptr;
            st.cap = 0;
            if ((err = hipHostMalloc(&st.host, bytes, hipHostMallocDefault)) != hipSuccess) return err;
            st.cap = bytes;
        }
        std::memcpy(st.host, L.entries.data(), bytes);
        if ((err = hipMemcpyAsync(w, st.host, bytes, hipMemcpyHostToDevice, s)) != hipSuccess) return err;
        if ((err = hipEventRecord(st.done, s)) != hipSuccess) return err;
    }
    const DenseEntry *table = reinterpret_cast<const DenseEntry *>(w);
    hipLaunchKernelGGL(pad_batch_kernel, dim3((unsigned)((L.padded + 255) / 256)), dim3(256), 0, s, table, n,
                       L.padded, reinterpret_cast<float2 *>(w + L.padded_off));
    if ((err = hipGetLastError()) != hipSuccess) return err;
    switch (precision) {
    case kPrecFp16: err = launch_dense_batch_p<kPrecFp16>(table, n, L, runs, s); break;
    case kPrecBf16: err = launch_dense_batch_p<kPrecBf16>(table, n, L, runs, s); break;
    case kPrecFp16x3: err = launch_dense_batch_p<kPrecFp16x3>(table, n, L, runs, s); break;
    case kPrecBf16x3: err = launch_dense_batch_p<kPrecBf16x3>(table, n, L, runs, s); break;
    default: return hipErrorInvalidValue;
    }
    if (err != hipSuccess || L.cells == 0) return err;
    hipLaunchKernelGGL(reduce_batch_kernel, dim3((unsigned)((L.cells + kReduceCells - 1) / kReduceCells)), dim3(256), 0,
                       s, table, n,
                       L.cells);
    return hipGetLastError();
}

void release_dense_stage() {
    std::lock_guard<std::mutex> lock(g_stage_mu);
    for (auto &kv : g_stage) {
        for (DenseStage &st : kv.second.slot) {
            if (st.done) {
                (void)hipEventSynchronize(st.done);
                (void)hipEventDestroy(st.done);
            }
            if (st.host) (void)hipHostFree(st.host);
        }
    }
    g_stage.clear();
}

// Workspace: [split partial planes][padded points] (dense) or the banded layout.
hipError_t launch_sep(const MapArgs &a, int precision, void *ws, hipStream_t stream) {
    if (banded_applies(a)) return launch_sep_banded(a, precision, ws, stream);
    const SepPlan pl = sep_plan(a, chunk_for(precision));
    float *dst = pl.splits > 1 ? static_cast<float *>(ws) : a.out;
    float2 *padded = reinterpret_cast<float2 *>(static_cast<char *>(ws) + pl.partial_bytes);
    const int64_t total = (int64_t)pl.splits * pl.pad_stride;
    hipLaunchKernelGGL(pad_points_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, stream, a.pts, a.n,
                       pl.per_split, pl.pad_stride, total, padded);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    switch (precision) {
    case kPrecFp16: e = launch_sep_p<kPrecFp16>(a, pl, padded, dst, stream); break;
    case kPrecBf16: e = launch_sep_p<kPrecBf16>(a, pl, padded, dst, stream); break;
    case kPrecFp16x3: e = launch_sep_p<kPrecFp16x3>(a, pl, padded, dst, stream); break;
    case kPrecBf16x3: e = launch_sep_p<kPrecBf16x3>(a, pl, padded, dst, stream); break;
    default: return hipErrorInvalidValue;
    }
    if (e != hipSuccess || pl.splits == 1) return e;
    return launch_reduce_splits(static_cast<const float *>(ws), pl.splits, (int64_t)a.nx * a.ny, a.scale, a.out,
                                stream);
}

}  // namespace kde
