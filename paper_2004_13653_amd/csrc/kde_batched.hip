// Many heat maps in one persistent launch (FP32 direct path).
//
// The work of a batch is cut into items (map, pixel tile, point range): tiles
// of the per-kernel register-block shape, and Gaussian tiles whose point count
// would make one item long are split into point ranges of about 2^26 pairs.
// Items are sorted by estimated cost, longest first.  A persistent grid of
// workgroups (about one per SIMD slot the kernel can occupy) pulls item indices
// from an atomic counter until the list is exhausted, so uneven maps balance
// across the CUs.  An item that covers a whole tile writes the scaled tile to
// its map; split items write raw partial tiles, and the last of a tile's splits
// to finish (a per-tile atomic count, with device-scope fences) adds the
// partials in split order and writes the scaled tile: results do not depend on
// which workgroup finishes last.
//
// Compact maps are whole-tile items over all of the map's points; a first
// kernel of the launch takes the bounding box of every 256-point chunk of those
// points, and a tile item loads only the chunks whose box reaches the tile.
// Tracks are stored in order, so a chunk is a short stretch of one or two
// tracks and most chunks miss most tiles.  Small supports accumulate the
// reaching points' terms in 64-bit fixed point (run_accum_item: exact, so equal
// to kde_eval's fixed-point maps bit for bit); larger ones are gathered
// (tile::tile_sums_boxed, the same sums as the full scan bit for bit).
//
// Host side: a batch shape (per map: kernel, tile side, grid, point count)
// fixes the item list and the static map fields.  The first call of a shape
// builds them, uploads the item list once and captures into a hipGraph the copy
// of the map descriptors from a pinned staging buffer, a counter reset kernel,
// the box kernel and the persistent kernel; later calls of the shape only write
// the descriptors (new pointers and bandwidths) and replay the graph.  Eager
// calls copy descriptors and items and launch the same kernels.
#include "kde_tile.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

namespace kde {

namespace {

using tile::kPointTile;
using tile::kThreads;

constexpr int64_t kPairsPerItem = int64_t(1) << 26;

struct BMap {
    const float2 *pts;
    float *out;
    int64_t n;
    int64_t box0;     // first of this map's chunk boxes (compact maps; running count)
    int kernel, rc;   // kernel id, register-block side (tile side 16 rc)
    int nx, ny, tiles_x;
    float Hx, Hy, ax, ay, scale;
};

struct BItem {
    int map, tile, split, nsplit;
    int64_t p0, p1;
    int64_t slot;      // first float of this split's partial tile (split items only)
    int tile_global;   // index of the tile's finish counter (split items only)
    int pad;
};

struct BatchLaunch {
    const BMap *maps;
    const BItem *items;
    int n_items, n_maps;
    int *counter;   // [1 + n_split_tiles]: next item, then per-tile finish counts
    float *partials;
    float4 *boxes;  // [n_boxes]: (x min, x max, y min, y max) per 256-point chunk of the compact maps
    int64_t n_boxes;
};

// One wave per chunk box: its map is the last whose box0 is at most the box
// index (maps without chunks repeat the next map's box0).
__global__ __launch_bounds__(256) void batch_box_kernel(BatchLaunch b) {
    const int64_t gc = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (gc >= b.n_boxes) return;  // uniform per wave
    int lo = 0, hi = b.n_maps - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (b.maps[mid].box0 <= gc) lo = mid;
        else hi = mid - 1;
    }
    const BMap m = b.maps[lo];
    const int64_t base = (gc - m.box0) * kPointTile;
    const int lane = threadIdx.x & 63;
    float x0 = 3.0e38f, x1 = -3.0e38f, y0 = 3.0e38f, y1 = -3.0e38f;
#pragma unroll
    for (int k = 0; k < kPointTile / 64; ++k) {
        const int64_t q = base + lane + 64 * k;
        if (q < m.n) {
            const float2 v = m.pts[q];
            x0 = fminf(x0, v.x);
            x1 = fmaxf(x1, v.x);
            y0 = fminf(y0, v.y);
            y1 = fmaxf(y1, v.y);
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        x0 = fminf(x0, __shfl_xor(x0, off));
        x1 = fmaxf(x1, __shfl_xor(x1, off));
        y0 = fminf(y0, __shfl_xor(y0, off));
        y1 = fmaxf(y1, __shfl_xor(y1, off));
    }
    if (lane == 0) b.boxes[gc] = make_float4(x0, x1, y0, y1);
}

template <int K, int RC, bool kRuns>
__device__ __forceinline__ void run_item(const BMap &m, const BItem &w, const BatchLaunch &b, float2 *sp,
                                         int *swave, int *slist, int *s_last) {
    using S = tile::Shape<K, RC>;
    const int tid = threadIdx.x;
    const int tx = w.tile % m.tiles_x, ty = w.tile / m.tiles_x;
    const int x0 = tx * S::TW, y0 = ty * S::TH;
    const int lib = (tid & 15) * S::C, ljb = (tid >> 4) * S::R;  // tile-local block origin
    const int ib = x0 + lib, jb = y0 + ljb;
    float tot[S::R][S::C];
    const float bx0 = (float)x0, bx1 = (float)(min(x0 + S::TW, m.nx) - 1);
    const float by0 = (float)y0, by1 = (float)(min(y0 + S::TH, m.ny) - 1);
    if constexpr (S::kCull)  // whole-tile item over all the map's points
        tile::tile_sums_boxed<K, S::R, S::C>(m.pts, m.n, b.boxes + m.box0, m.Hx, m.Hy, m.ax, m.ay, ib, jb, bx0, bx1,
                                             by0, by1, sp, swave, slist, tot);
    else
        tile::tile_sums<K, S::R, S::C, false, kRuns>(m.pts, w.p0, w.p1, m.Hx, m.Hy, m.ax, m.ay, ib, jb, bx0, bx1,
                                                     by0, by1, sp, swave, tot);
    if constexpr (kRuns) tile::apply_run_q<S::R, S::C>(tot, m.ax, m.ay);
    if (w.nsplit == 1) {
        tile::store_block<S::R, S::C>(tot, m.out, m.nx, m.ny, ib, jb, m.scale);
        return;
    }
    // Partial tile, row-major TW x TH.
    constexpr int kTileElems = S::TW * S::TH;
    float *mine = b.partials + w.slot;
#pragma unroll
    for (int r = 0; r < S::R; ++r)
#pragma unroll
        for (int c = 0; c < S::C; ++c) mine[(ljb + r) * S::TW + lib + c] = tot[r][c];
    __threadfence();  // release the partial before counting this split as done
    __syncthreads();
    if (tid == 0) *s_last = atomicAdd(b.counter + 1 + w.tile_global, 1) == w.nsplit - 1;
    __syncthreads();
    if (!*s_last) return;
    __threadfence();  // acquire the other splits' partials
    const float *first = b.partials + (w.slot - (int64_t)w.split * kTileElems);
#pragma unroll
    for (int r = 0; r < S::R; ++r)
#pragma unroll
        for (int c = 0; c < S::C; ++c) {
            float v = 0.0f;
            for (int s = 0; s < w.nsplit; ++s) v += first[s * kTileElems + (ljb + r) * S::TW + lib + c];
            tot[r][c] = v;
        }
    tile::store_block<S::R, S::C>(tot, m.out, m.nx, m.ny, ib, jb, m.scale);
}

// Compact maps whose supports span at most tile::kBatchAccumMaxFootprint tried
// nodes (tile::accum_footprint_fits): the item's tile is taken as sub-tiles of
// side at most kAccMaxSide (such maps get tiles of that side, so one pass; 32
// in the general variant, which has no registers to spare).  For each, the
// chunks whose box reaches it are listed; their points are read (coalesced)
// and those whose support can reach the sub-tile are gathered into a list in
// LDS, which, when nearly full, is worked through point by point: each adds its
// own terms (tile::accum_point) to a fixed-point tile in LDS.  Integer sums
// depend neither on the order nor on the tiling the points come in, so the maps
// that kde_eval sums in fixed point too (tile::accum_applies) equal its maps bit
// for bit.  In the list, the
// lanes of a wave take entries kThreads / 64 apart (list entries keep track
// order), so that they seldom start in one node at once and their atomics
// seldom collide.
constexpr int kAccMaxSide = 64;
constexpr int kAccGroup = 1;    // listed chunks read per step
constexpr int kAccList = 768;   // float2 entries; the point tile of the gather items shares the array

template <int K, int AS>
__device__ __forceinline__ void accum_list(const BMap &m, const float2 *lst, int cnt, int x0, int y0,
                                           unsigned long long *acc) {
    const int spread = (threadIdx.x & 63) * (kThreads / 64) + (threadIdx.x >> 6);
    for (int e0 = 0; e0 < cnt; e0 += kThreads) {
        const int e = e0 + spread;
        if (e < cnt) tile::accum_point<K, AS, AS>(lst[e], x0, y0, m.nx, m.ny, m.Hx, m.Hy, m.ax, m.ay, acc);
    }
}

template <int K, int RC, int G, int kMaxSide>
__device__ __forceinline__ void run_accum_item(const BMap &m, const BItem &w, const BatchLaunch &b,
                                               unsigned long long *acc, float2 *lst, int *swave, int *slist,
                                               int *sgrp) {
    constexpr int TS = 16 * RC, AS = TS < kMaxSide ? TS : kMaxSide, NS = TS / AS;
    static_assert(kMaxSide <= kAccMaxSide, "the accumulation tile holds kAccMaxSide^2 nodes");
    static_assert(TS % AS == 0, "tile side must be a multiple of the accumulation side");
    // one point per thread per chunk; a flushed list holds more than kThreads points
    static_assert(kPointTile == kThreads && G <= kAccGroup && kAccList >= (G + 1) * kThreads, "list too short");
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const uint64_t below = (1ull << lane) - 1ull;
    const int tx = w.tile % m.tiles_x, ty = w.tile / m.tiles_x;
    const int64_t nch = (m.n + kPointTile - 1) / kPointTile;
    const float4 *boxes = b.boxes + m.box0;
    const double unit = (1.0 / (double)tile::kFixedOne) * m.scale;
    for (int sub = 0; sub < NS * NS; ++sub) {
        const int x0 = tx * TS + (sub % NS) * AS, y0 = ty * TS + (sub / NS) * AS;
        if (x0 >= m.nx || y0 >= m.ny) continue;  // uniform: the sub-tile lies past the grid
        // Points reaching the sub-tile lie within H + 1 of its nodes (the margin
        // of one node covers the rounding of the factors' support tests).
        const float lx = (float)x0 - m.Hx - 1.0f, hx = (float)(min(x0 + AS, m.nx) - 1) + m.Hx + 1.0f;
        const float ly = (float)y0 - m.Hy - 1.0f, hy = (float)(min(y0 + AS, m.ny) - 1) + m.Hy + 1.0f;
        __syncthreads();  // the previous sub-tile has been written out
        for (int i = tid; i < AS * AS; i += kThreads) acc[i] = 0ull;
        int fill = 0;  // list entries (the same in every thread)
        for (int64_t g0 = 0; g0 < nch; g0 += kThreads) {
            const int64_t c = g0 + tid;
            bool hit = false;
            if (c < nch) {
                const float4 bx = boxes[c];
                hit = bx.y >= lx && bx.x <= hx && bx.w >= ly && bx.z <= hy;
            }
            const uint64_t mk = __ballot(hit);
            __syncthreads();  // the previous group's list and counts are consumed; acc is cleared
            if (lane == 0) swave[wv] = __popcll(mk);
            __syncthreads();
            int off = 0, cnt = 0;
#pragma unroll
            for (int k = 0; k < kThreads / 64; ++k) {
                off += (k < wv) ? swave[k] : 0;
                cnt += swave[k];
            }
            if (hit) slist[off + __popcll(mk & below)] = (int)(c - g0);
            __syncthreads();
            for (int k = 0; k < cnt; k += G) {  // G chunks a step: their loads overlap
                float2 v[G];
                bool take[G];
                uint64_t mt[G];
#pragma unroll
                for (int j = 0; j < G; ++j) {
                    const int64_t q = k + j < cnt ? (g0 + slist[k + j]) * kPointTile + tid : m.n;
                    v[j] = q < m.n ? m.pts[q] : make_float2(0.0f, 0.0f);
                    take[j] = q < m.n && v[j].x >= lx && v[j].x <= hx && v[j].y >= ly && v[j].y <= hy;  // NaN fails
                    mt[j] = __ballot(take[j]);
                }
                __syncthreads();  // every thread has read the counts of the previous step
                if (lane == 0)
#pragma unroll
                    for (int j = 0; j < G; ++j) sgrp[j * (kThreads / 64) + wv] = __popcll(mt[j]);
                __syncthreads();
#pragma unroll
                for (int j = 0; j < G; ++j) {  // list order: chunk by chunk, wave by wave, lane by lane
                    int at = fill;
#pragma unroll
                    for (int kk = 0; kk < kThreads / 64; ++kk) {
                        const int c = sgrp[j * (kThreads / 64) + kk];
                        at += (kk < wv) ? c : 0;
                        fill += c;
                    }
                    if (take[j]) lst[at + __popcll(mt[j] & below)] = v[j];
                }
                if (fill > kAccList - G * kThreads) {  // no room for another step's points
                    __syncthreads();
                    accum_list<K, AS>(m, lst, fill, x0, y0, acc);
                    fill = 0;  // the next writes to the list follow two barriers
                }
            }
        }
        __syncthreads();
        accum_list<K, AS>(m, lst, fill, x0, y0, acc);
        __syncthreads();
        for (int i = tid; i < AS * AS; i += kThreads) {
            const int gi = x0 + i % AS, gj = y0 + i / AS;
            if (gi < m.nx && gj < m.ny) m.out[(int64_t)gj * m.nx + gi] = (float)((double)acc[i] * unit);
        }
    }
}

template <int K, int kMaxRc>
__device__ __forceinline__ void run_shape(const BMap &m, const BItem &w, const BatchLaunch &b, float2 *sp,
                                          int *swave, int *slist, int *s_last, unsigned long long *acc,
                                          int *sgrp) {
    if constexpr (K != kGaussian) {
        // the general variant has no registers to spare: one chunk a step, sub-tiles of 32
        constexpr int kG = kMaxRc < 8 ? kAccGroup : 1, kSide = kMaxRc < 8 ? kAccMaxSide : 32;
        // as batch_accumulates; whole-tile items over all points
        if (tile::accum_footprint_fits(m.Hx, m.Hy, tile::kBatchAccumMaxFootprint)) {
            if (m.rc == 2)
                run_accum_item<K, 2, kG, kSide>(m, w, b, acc, sp, swave, slist, sgrp);
            else if (kMaxRc < 8 || m.rc == 4)
                run_accum_item<K, 4, kG, kSide>(m, w, b, acc, sp, swave, slist, sgrp);
            else
                run_accum_item<K, kMaxRc, kG, kSide>(m, w, b, acc, sp, swave, slist, sgrp);
            return;
        }
    }
    if constexpr (kMaxRc < 8) {  // lean variant: register blocks of side 2 and 4 only
        if (m.rc == 2)
            run_item<K, 2, false>(m, w, b, sp, swave, slist, s_last);
        else
            run_item<K, 4, false>(m, w, b, sp, swave, slist, s_last);
        return;
    }
    if constexpr (K == kGaussian) {
        if (m.ax <= kMaxRunScale && m.ay <= kMaxRunScale) {
            if (m.rc == 2)
                run_item<K, 2, true>(m, w, b, sp, swave, slist, s_last);
            else if (m.rc == 4)
                run_item<K, 4, true>(m, w, b, sp, swave, slist, s_last);
            else
                run_item<K, 8, true>(m, w, b, sp, swave, slist, s_last);
            return;
        }
    }
    if (m.rc == 2)
        run_item<K, 2, false>(m, w, b, sp, swave, slist, s_last);
    else if (m.rc == 4)
        run_item<K, 4, false>(m, w, b, sp, swave, slist, s_last);
    else
        run_item<K, 8, false>(m, w, b, sp, swave, slist, s_last);
}

// The general variant (kLean false) runs every kernel and register-block side.
// Batches of compact maps with blocks of side 2 or 4 (the usual case: Gaussian
// maps go to the matrix cores) use the lean variant, built without the Gaussian
// paths and the 8 x 8 blocks that set the register count of the general one,
// so that more workgroups fit on a CU.
template <bool kLean>
__global__ __launch_bounds__(kThreads, 2) void batched_kernel(BatchLaunch b) {  // at least 2 waves per SIMD
    constexpr int R = kLean ? 4 : 8;
    __shared__ float2 sp[kAccList];  // point tile of the gather items, point list of the accumulating ones
    __shared__ int swave[kThreads / 64];
    __shared__ int slist[kThreads];
    __shared__ int sgrp[kAccGroup * (kThreads / 64)];
    __shared__ int s_item, s_last;
    __shared__ unsigned long long acc[kAccMaxSide * kAccMaxSide];
    for (;;) {
        __syncthreads();  // every thread has read the previous s_item
        if (threadIdx.x == 0) s_item = atomicAdd(b.counter, 1);
        __syncthreads();
        const int it = s_item;
        if (it >= b.n_items) return;  // the counter only grows: every workgroup reaches this
        const BItem w = b.items[it];
        const BMap m = b.maps[w.map];
        switch (m.kernel) {
        case kUniform: run_shape<kUniform, R>(m, w, b, sp, swave, slist, &s_last, acc, sgrp); break;
        case kTriangular: run_shape<kTriangular, R>(m, w, b, sp, swave, slist, &s_last, acc, sgrp); break;
        case kEpanechnikov: run_shape<kEpanechnikov, R>(m, w, b, sp, swave, slist, &s_last, acc, sgrp); break;
        case kQuartic: run_shape<kQuartic, R>(m, w, b, sp, swave, slist, &s_last, acc, sgrp); break;
        case kTriweight: run_shape<kTriweight, R>(m, w, b, sp, swave, slist, &s_last, acc, sgrp); break;
        case kTricube: run_shape<kTricube, R>(m, w, b, sp, swave, slist, &s_last, acc, sgrp); break;
        case kGaussian:
            if constexpr (!kLean) run_shape<kGaussian, R>(m, w, b, sp, swave, slist, &s_last, acc, sgrp);
            break;
        default: run_shape<kCosine, R>(m, w, b, sp, swave, slist, &s_last, acc, sgrp); break;
        }
    }
}

__global__ void zero_ints_kernel(int *p, int count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0;
}

// ------------------------------------------------------------------ host side

struct Plan {
    std::vector<BMap> maps;
    std::vector<BItem> items;
    int n_split_tiles = 0;
    int64_t n_slots = 0;  // floats of partial tiles
    int64_t n_boxes = 0;  // chunk boxes of the compact maps
    bool lean = true;     // no Gaussian map and no register block of side 8
};

// Everything a batch's item list and static map fields depend on: per map the
// kernel, register-block side, grid and point count.  Pointers and the
// bandwidth-dependent scalars are per-call values.
std::string shape_key(const MapArgs *args, int n_maps) {
    std::string k;
    k.reserve((size_t)n_maps * 24);
    for (int m = 0; m < n_maps; ++m) {
        const int32_t st[4] = {args[m].kernel_id, args[m].rc, args[m].nx, args[m].ny};
        k.append(reinterpret_cast<const char *>(st), sizeof st);
        k.append(reinterpret_cast<const char *>(&args[m].n), sizeof args[m].n);
    }
    return k;
}

// The per-call map descriptors: the plan's static fields, this call's values.
void fill_maps(const MapArgs *args, const std::vector<BMap> &tmpl, BMap *dst) {
    for (size_t m = 0; m < tmpl.size(); ++m) {
        BMap bm = tmpl[m];
        const MapArgs &a = args[m];
        bm.pts = a.pts;
        bm.out = a.out;
        bm.Hx = a.Hx;
        bm.Hy = a.Hy;
        bm.ax = a.ax;
        bm.ay = a.ay;
        bm.scale = a.scale;
        dst[m] = bm;
    }
}

Plan make_plan(const MapArgs *args, int n_maps) {
    Plan pl;
    pl.maps.resize(n_maps);
    struct Costed {
        double cost;
        int order;
        BItem item;
    };
    std::vector<Costed> cs;
    for (int m = 0; m < n_maps; ++m) {
        const MapArgs &a = args[m];
        const int TW = 16 * a.rc, TH = 16 * a.rc;
        BMap &bm = pl.maps[m];
        bm.pts = a.pts;
        bm.out = a.out;
        bm.n = a.n;
        bm.kernel = a.kernel_id;
        bm.rc = a.rc;
        bm.nx = a.nx;
        bm.ny = a.ny;
        bm.tiles_x = (a.nx + TW - 1) / TW;
        bm.Hx = a.Hx;
        bm.Hy = a.Hy;
        bm.ax = a.ax;
        bm.ay = a.ay;
        bm.scale = a.scale;
        const int tiles = bm.tiles_x * ((a.ny + TH - 1) / TH);
        const bool dense = a.kernel_id == kGaussian;
        bm.box0 = pl.n_boxes;
        if (!dense) pl.n_boxes += (a.n + kPointTile - 1) / kPointTile;
        pl.lean = pl.lean && !dense && a.rc <= 4;
        int64_t per = a.n;
        if (dense) {
            per = std::max<int64_t>(kPointTile, kPairsPerItem / ((int64_t)TW * TH));
            per = (per + kPointTile - 1) / kPointTile * kPointTile;
        }
        const int nsplit = a.n == 0 ? 1 : (int)((a.n + per - 1) / per);
        for (int t = 0; t < tiles; ++t) {
            const int tg = nsplit > 1 ? pl.n_split_tiles++ : -1;
            for (int s = 0; s < nsplit; ++s) {
                BItem it{};
                it.map = m;
                it.tile = t;
                it.split = s;
                it.nsplit = nsplit;
                it.p0 = std::min<int64_t>(a.n, s * per);
                it.p1 = std::min<int64_t>(a.n, (s + 1) * per);
                it.slot = -1;
                if (nsplit > 1) {
                    it.slot = pl.n_slots;
                    pl.n_slots += (int64_t)TW * TH;
                }
                it.tile_global = tg;
                // Dense tiles cost pairs; compact tiles the box scan (about one
                // 256-pixel pass per chunk box) plus their mean share of the
                // points, each against the whole tile.
                const double npts = (double)(it.p1 - it.p0);
                const double cost = dense ? npts * TW * TH
                                          : npts / kPointTile * 256.0 + npts / tiles * TW * TH;
                cs.push_back({cost, (int)cs.size(), it});
            }
        }
    }
    std::stable_sort(cs.begin(), cs.end(), [](const Costed &x, const Costed &y) { return x.cost > y.cost; });
    pl.items.reserve(cs.size());
    for (const auto &c : cs) pl.items.push_back(c.item);
    return pl;
}

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

struct Layout {
    size_t maps_off, items_off, stage_bytes;  // staged (copied) part
    size_t counters_off, partials_off, boxes_off, total;
    int n_counters;
};

Layout layout_of(const Plan &pl) {
    Layout L;
    L.maps_off = 0;
    L.items_off = align256(pl.maps.size() * sizeof(BMap));
    L.stage_bytes = align256(L.items_off + pl.items.size() * sizeof(BItem));
    L.counters_off = L.stage_bytes;
    L.n_counters = 1 + pl.n_split_tiles;
    L.partials_off = align256(L.counters_off + (size_t)L.n_counters * sizeof(int));
    L.boxes_off = align256(L.partials_off + (size_t)pl.n_slots * sizeof(float));
    L.total = align256(L.boxes_off + (size_t)pl.n_boxes * sizeof(float4));
    return L;
}

// Workgroups of the persistent launch: as many as can be resident at once
// (occupancy of the kernel variant times the CUs), at most one per item.
template <bool kLean>
int persistent_grid(int n_items) {
    static int resident = 0;
    if (resident == 0) {
        int dev = 0, cus = 0, per_cu = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batched_kernel<kLean>, kThreads, 0) !=
                hipSuccess || per_cu <= 0)
            per_cu = 2;
        resident = per_cu * cus;
    }
    return std::max(1, std::min(n_items, resident));
}

// copy_bytes of the staging buffer go to the device first: the map descriptors
// and item list (eager runs), or the map descriptors only (graph replays, whose
// item list was uploaded when the graph was made).
hipError_t enqueue(const Plan &pl, const Layout &L, const void *host_stage, size_t copy_bytes, char *dev,
                   hipStream_t s) {
    hipError_t e = hipMemcpyAsync(dev, host_stage, copy_bytes, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(zero_ints_kernel, dim3((L.n_counters + 255) / 256), dim3(256), 0, s,
                       reinterpret_cast<int *>(dev + L.counters_off), L.n_counters);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    BatchLaunch b;
    b.maps = reinterpret_cast<const BMap *>(dev + L.maps_off);
    b.items = reinterpret_cast<const BItem *>(dev + L.items_off);
    b.n_items = (int)pl.items.size();
    b.n_maps = (int)pl.maps.size();
    b.counter = reinterpret_cast<int *>(dev + L.counters_off);
    b.partials = reinterpret_cast<float *>(dev + L.partials_off);
    b.boxes = reinterpret_cast<float4 *>(dev + L.boxes_off);
    b.n_boxes = pl.n_boxes;
    if (pl.n_boxes > 0) {
        hipLaunchKernelGGL(batch_box_kernel, dim3((unsigned)((pl.n_boxes + 3) / 4)), dim3(256), 0, s, b);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (pl.lean)
        hipLaunchKernelGGL(batched_kernel<true>, dim3(persistent_grid<true>(b.n_items)), dim3(kThreads), 0, s, b);
    else
        hipLaunchKernelGGL(batched_kernel<false>, dim3(persistent_grid<false>(b.n_items)), dim3(kThreads), 0, s, b);
    return hipGetLastError();
}

// A captured batch: device buffer (item list uploaded once), pinned staging
// buffer of the map descriptors, executable graph, and the plan's static map
// fields.
struct Captured {
    char *dev = nullptr;
    char *stage = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t done = nullptr;
    Layout L;
    std::vector<BMap> maps;
    ~Captured() {
        if (done) (void)hipEventSynchronize(done);
        if (exec) (void)hipGraphExecDestroy(exec);
        if (done) (void)hipEventDestroy(done);
        if (stage) (void)hipHostFree(stage);
        if (dev) (void)hipFree(dev);
    }
};

std::mutex g_mu;
std::map<std::pair<int, std::string>, std::unique_ptr<Captured>> g_graphs;  // (device, signature)

}  // namespace

hipError_t run_batched(const MapArgs *args, int n_maps, bool use_graph, void *ws_eager, size_t ws_bytes,
                       hipStream_t stream) {
    for (int m = 0; m < n_maps; ++m)
        if (!valid_rc(args[m].rc)) return hipErrorInvalidValue;
    if (!use_graph) {
        const Plan pl = make_plan(args, n_maps);
        if (pl.items.empty()) return hipSuccess;
        const Layout L = layout_of(pl);
        if (ws_bytes < L.total) return hipErrorInvalidValue;
        std::vector<char> stage(L.stage_bytes);
        std::memcpy(stage.data() + L.maps_off, pl.maps.data(), pl.maps.size() * sizeof(BMap));
        std::memcpy(stage.data() + L.items_off, pl.items.data(), pl.items.size() * sizeof(BItem));
        hipError_t e = enqueue(pl, L, stage.data(), L.stage_bytes, static_cast<char *>(ws_eager), stream);
        if (e != hipSuccess) return e;
        return hipStreamSynchronize(stream);  // the pageable staging buffer dies here
    }
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lock(g_mu);
    auto &slot = g_graphs[{dev, shape_key(args, n_maps)}];
    if (!slot) {
        const Plan pl = make_plan(args, n_maps);
        if (pl.items.empty()) return hipSuccess;
        auto c = std::make_unique<Captured>();
        c->L = layout_of(pl);
        c->maps = pl.maps;
        const size_t map_bytes = pl.maps.size() * sizeof(BMap);
        if ((e = hipMalloc(&c->dev, c->L.total)) != hipSuccess) return e;
        if ((e = hipHostMalloc(&c->stage, map_bytes, hipHostMallocDefault)) != hipSuccess) return e;
        if ((e = hipEventCreateWithFlags(&c->done, hipEventDisableTiming)) != hipSuccess) return e;
        if ((e = hipMemcpy(c->dev + c->L.items_off, pl.items.data(), pl.items.size() * sizeof(BItem),
                           hipMemcpyHostToDevice)) != hipSuccess)
            return e;
        hipStream_t cap = nullptr;
        if ((e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking)) != hipSuccess) return e;
        hipGraph_t graph = nullptr;
        e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            const hipError_t e1 = enqueue(pl, c->L, c->stage, map_bytes, c->dev, cap);
            e = hipStreamEndCapture(cap, &graph);
            if (e1 != hipSuccess) e = e1;
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&c->exec, graph, nullptr, nullptr, 0);
        if (graph) (void)hipGraphDestroy(graph);
        (void)hipStreamDestroy(cap);
        if (e != hipSuccess) return e;
        slot = std::move(c);
    }
    Captured &c = *slot;
    // The previous replay's copy must have read the staging buffer before it is
    // overwritten.
    if ((e = hipEventSynchronize(c.done)) != hipSuccess) return e;
    fill_maps(args, c.maps, reinterpret_cast<BMap *>(c.stage));
    if ((e = hipGraphLaunch(c.exec, stream)) != hipSuccess) return e;
    return hipEventRecord(c.done, stream);
}

bool batch_accumulates(const MapArgs &a) {
    return a.kernel_id != kGaussian && tile::accum_footprint_fits(a.Hx, a.Hy, tile::kBatchAccumMaxFootprint);
}

size_t batched_workspace_bytes(const MapArgs *args, int n_maps) {
    const Plan pl = make_plan(args, n_maps);
    return pl.items.empty() ? 0 : layout_of(pl).total;
}

void release_batched_graphs() {
    std::lock_guard<std::mutex> lock(g_mu);
    g_graphs.clear();
}

}  // namespace kde
