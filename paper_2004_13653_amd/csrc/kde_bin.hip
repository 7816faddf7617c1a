// Support binning for the compact kernels (FP32 direct path).
//
// A point contributes only to nodes within H of it, so each T x T output tile
// (T = 16 rc, the map's register-block tile) needs only the points whose support square [X +- Hx] x [Y +- Hy] reaches one
// of its nodes.  Instead of every tile scanning all points, the points are
// counting-sorted into per-tile bins:
//
//   1. count:   every point adds 1 to cnt[tile][w] for each tile it reaches,
//               where w is its block of 1024 consecutive points (integer
//               atomics: the counts do not depend on their order);
//   2. scan:    exclusive prefix sum over cnt in tile-major order gives each
//               (tile, wave block) its first slot (the paper's work-efficient
//               scan pattern, Sec. IV-A: per-block scans, a scan of the block
//               totals, then a propagation pass);
//   3. scatter: for the gather, one wave per block walks its points 64 at a
//               time, and each 64's tiles in a fixed order, assigning slots with
//               ballots (lanes with the same tile take consecutive slots in lane
//               order), so the bin contents and their order (point order) are
//               the same on every run; for the fixed-point accumulation, whose
//               sums do not depend on order, one thread per point takes its
//               slots with atomics on the same table;
//   4. items:   each tile's bin is cut into items of at most M entries (dense
//               tiles, e.g. at anchorages, get many; M from the bound on all
//               entries, aiming at ~2048 items), one workgroup per item;
//   5. sums:    small compact supports accumulate per point in 64-bit fixed
//               point (bin_accum_kernel), the others are gathered with the
//               register-tiled kernel of the direct path (no culling needed;
//               the per-pair support test remains); a tile with one item writes
//               the map directly, the others write partial tiles that a last
//               pass adds in item order (as integers for the fixed point).
#include "kde_tile.h"

#include <algorithm>
#include <cmath>

namespace kde {

namespace {

constexpr int kScanBlock = 1024;
constexpr int kColBlock = 1024;   // points per count column (one wave each in the scatter)
constexpr int kTargetItems = 2048;

struct BinGeom {
    int nx, ny, tiles_x, tiles_y;
    int tile;  // tile side in nodes
    float Hx, Hy;
    int64_t n, wblocks;  // points, kColBlock-point blocks (count columns)
};

// Tile rectangle a point reaches (empty when tx0 > tx1 or ty0 > ty1).
__device__ __forceinline__ void reach(const BinGeom &g, float2 v, int &tx0, int &tx1, int &ty0, int &ty1) {
    const float i0 = fmaxf(0.0f, ceilf(v.x - g.Hx)), i1 = fminf((float)(g.nx - 1), floorf(v.x + g.Hx));
    const float j0 = fmaxf(0.0f, ceilf(v.y - g.Hy)), j1 = fminf((float)(g.ny - 1), floorf(v.y + g.Hy));
    if (!(i0 <= i1 && j0 <= j1)) {  // also false for NaN coordinates
        tx0 = ty0 = 1;
        tx1 = ty1 = 0;
        return;
    }
    tx0 = (int)i0 / g.tile;
    tx1 = (int)i1 / g.tile;
    ty0 = (int)j0 / g.tile;
    ty1 = (int)j1 / g.tile;
}

// Counts per (tile, column); lanes of a wave that register in the same tile
// combine into one atomic (tracks are stored in order, so neighbouring points
// mostly share their tiles).
__global__ __launch_bounds__(256) void bin_count_kernel(BinGeom g, const float2 *__restrict__ pts,
                                                        unsigned *__restrict__ cnt) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    if (p - lane >= g.n) return;  // whole wave past the end
    const int64_t w = p / kColBlock;  // one column per wave (kColBlock is a multiple of 64)
    int tx0 = 1, tx1 = 0, ty0 = 1, ty1 = 0;
    if (p < g.n) reach(g, pts[p], tx0, tx1, ty0, ty1);
    const int ncols = tx1 >= tx0 ? tx1 - tx0 + 1 : 0;
    const int ntl = ncols > 0 && ty1 >= ty0 ? ncols * (ty1 - ty0 + 1) : 0;
    int most = ntl;
    for (int o = 32; o > 0; o >>= 1) most = max(most, __shfl_xor(most, o));
    for (int j = 0; j < most; ++j) {
        const int key = j < ntl ? (ty0 + j / ncols) * g.tiles_x + tx0 + j % ncols : -1;
        uint64_t pending = __ballot(key >= 0);
        while (pending) {
            const int leader = __ffsll((unsigned long long)pending) - 1;
            const int lkey = __shfl(key, leader);
            const uint64_t same = __ballot(key == lkey);
            if (lane == leader) atomicAdd(&cnt[(int64_t)lkey * g.wblocks + w], (unsigned)__popcll(same));
            pending &= ~same;
        }
    }
}

// Exclusive scan, pass 1: each block scans kScanBlock entries in place and
// stores its total.
__global__ __launch_bounds__(256) void scan_blocks_kernel(unsigned *__restrict__ a, int64_t len,
                                                          unsigned *__restrict__ totals) {
    __shared__ unsigned s[256];
    const int tid = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * kScanBlock + 4 * tid;
    unsigned v[4], sum = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        v[k] = base + k < len ? a[base + k] : 0u;
        sum += v[k];
    }
    s[tid] = sum;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {  // inclusive Hillis-Steele over thread sums
        const unsigned t = tid >= off ? s[tid - off] : 0u;
        __syncthreads();
        s[tid] += t;
        __syncthreads();
    }
    unsigned run = s[tid] - sum;  // exclusive prefix of this thread
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (base + k < len) a[base + k] = run;
        run += v[k];
    }
    if (tid == 255) totals[blockIdx.x] = s[255];
}

// Pass 2: exclusive scan of the block totals by one workgroup (sequential over
// 256-entry segments); writes the grand total to totals[nblocks].
__global__ __launch_bounds__(256) void scan_totals_kernel(unsigned *__restrict__ totals, int64_t nblocks) {
    __shared__ unsigned s[256];
    __shared__ unsigned carry;
    const int tid = threadIdx.x;
    if (tid == 0) carry = 0;
    __syncthreads();
    for (int64_t seg = 0; seg < nblocks; seg += 256) {
        const int64_t i = seg + tid;
        const unsigned v = i < nblocks ? totals[i] : 0u;
        s[tid] = v;
        __syncthreads();
        for (int off = 1; off < 256; off <<= 1) {
            const unsigned t = tid >= off ? s[tid - off] : 0u;
            __syncthreads();
            s[tid] += t;
            __syncthreads();
        }
        if (i < nblocks) totals[i] = carry + s[tid] - v;
        __syncthreads();
        if (tid == 0) carry += s[255];
        __syncthreads();
    }
    if (tid == 0) totals[nblocks] = carry;
}

// Pass 3: add each block's offset.
__global__ __launch_bounds__(256) void scan_add_kernel(unsigned *__restrict__ a, int64_t len,
                                                       const unsigned *__restrict__ totals) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < len) a[i] += totals[i / kScanBlock];
}

// Scatter: one wave per kColBlock-point block, 64 points per step in point
// order.  off[] holds the (tile, block) start slots and is advanced in place
// (each column belongs to one wave), so that afterwards off[t][w] is the end of
// segment (t, w).
__global__ __launch_bounds__(256) void bin_scatter_kernel(BinGeom g, const float2 *__restrict__ pts,
                                                          unsigned *__restrict__ off, float2 *__restrict__ bins) {
    const int lane = threadIdx.x & 63;
    const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (w >= g.wblocks) return;  // whole wave
    const uint64_t below = (1ull << lane) - 1ull;
    for (int step = 0; step < kColBlock / 64; ++step) {
        const int64_t p = w * kColBlock + step * 64 + lane;
        if (w * kColBlock + step * 64 >= g.n) break;  // whole wave
        const bool valid = p < g.n;
        const float2 v = valid ? pts[p] : make_float2(0.0f, 0.0f);
        int tx0 = 1, tx1 = 0, ty0 = 1, ty1 = 0;
        if (valid) reach(g, v, tx0, tx1, ty0, ty1);
        const int ncols = tx1 >= tx0 ? tx1 - tx0 + 1 : 0;
        const int ntl = ncols > 0 && ty1 >= ty0 ? ncols * (ty1 - ty0 + 1) : 0;
        int most = ntl;
        for (int o = 32; o > 0; o >>= 1) most = max(most, __shfl_xor(most, o));
        for (int j = 0; j < most; ++j) {  // j-th tile of every lane, raster order within its rectangle
            int key = -1;
            if (j < ntl) key = (ty0 + j / ncols) * g.tiles_x + tx0 + j % ncols;
            uint64_t pending = __ballot(key >= 0);
            while (pending) {
                const int leader = __ffsll((unsigned long long)pending) - 1;
                const int lkey = __shfl(key, leader);
                const uint64_t same = __ballot(key == lkey);
                // Only this wave touches column w, so the atomic just returns the
                // current cursor and advances it, in this wave's program order.
                unsigned base = 0;
                if (lane == leader) base = atomicAdd(&off[(int64_t)lkey * g.wblocks + w], (unsigned)__popcll(same));
                base = __shfl(base, leader);
                if (key == lkey) bins[base + (unsigned)__popcll(same & below)] = v;
                pending &= ~same;
            }
        }
    }
}


// Items: item_off[t] (exclusive prefix over tiles, item_off[tiles] = all items)
// is the first item of tile t; tile t's bin is cut into item_off[t+1] -
// item_off[t] = max(1, ceil(bin length / per_item)) equal parts.  One
// workgroup, from the scanned (tile, column) table, whose last column of tile t
// ends t's bin after the scatter.
constexpr int kItemScan = 1024;

__global__ __launch_bounds__(kItemScan) void item_scan_kernel(const unsigned *__restrict__ end, int64_t wblocks,
                                                              int tiles, int64_t per_item,
                                                              unsigned *__restrict__ item_off) {
    __shared__ unsigned si[kItemScan];
    const int tid = threadIdx.x;
    unsigned carry = 0u;
    for (int base = 0; base < tiles; base += kItemScan) {
        const int t = base + tid;
        unsigned it = 0u;
        if (t < tiles) {
            const int64_t e = end[(int64_t)t * wblocks + wblocks - 1];
            const int64_t b = t > 0 ? (int64_t)end[(int64_t)t * wblocks - 1] : 0;
            const int64_t need = (e - b + per_item - 1) / per_item;
            it = (unsigned)(need > 1 ? need : 1);
        }
        si[tid] = it;
        __syncthreads();
        for (int off = 1; off < kItemScan; off <<= 1) {  // inclusive Hillis-Steele
            const unsigned a = tid >= off ? si[tid - off] : 0u;
            __syncthreads();
            si[tid] += a;
            __syncthreads();
        }
        if (t < tiles) item_off[t] = carry + si[tid] - it;
        carry += si[kItemScan - 1];
        __syncthreads();  // every thread has read the total before the next chunk
    }
    if (tid == 0) item_off[tiles] = carry;
}

// Order-free scatter, for the fixed-point accumulation (whose sums do not
// depend on the order of a tile's points): one thread per point takes slots
// from the scanned (tile, column) table with atomics, the lanes of a wave that
// register in one tile sharing one.  Only the waves of one 1024-point column
// touch its entries, and the table ends as the ordered scatter leaves it.
__global__ __launch_bounds__(256) void bin_scatter_free_kernel(BinGeom g, const float2 *__restrict__ pts,
                                                               unsigned *__restrict__ off,
                                                               float2 *__restrict__ bins) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    if (p - lane >= g.n) return;  // whole wave past the end
    const int64_t w = p / kColBlock;  // the wave's column (kColBlock is a multiple of 64)
    const uint64_t below = (1ull << lane) - 1ull;
    const bool valid = p < g.n;
    const float2 v = valid ? pts[p] : make_float2(0.0f, 0.0f);
    int tx0 = 1, tx1 = 0, ty0 = 1, ty1 = 0;
    if (valid) reach(g, v, tx0, tx1, ty0, ty1);
    const int ncols = tx1 >= tx0 ? tx1 - tx0 + 1 : 0;
    const int ntl = ncols > 0 && ty1 >= ty0 ? ncols * (ty1 - ty0 + 1) : 0;
    int most = ntl;
    for (int o = 32; o > 0; o >>= 1) most = max(most, __shfl_xor(most, o));
    for (int j = 0; j < most; ++j) {
        const int key = j < ntl ? (ty0 + j / ncols) * g.tiles_x + tx0 + j % ncols : -1;
        uint64_t pending = __ballot(key >= 0);
        while (pending) {
            const int leader = __ffsll((unsigned long long)pending) - 1;
            const int lkey = __shfl(key, leader);
            const uint64_t same = __ballot(key == lkey);
            unsigned slot = 0;
            if (lane == leader) slot = atomicAdd(&off[(int64_t)lkey * g.wblocks + w], (unsigned)__popcll(same));
            slot = __shfl(slot, leader);
            if (key == lkey) bins[slot + (unsigned)__popcll(same & below)] = v;
            pending &= ~same;
        }
    }
}

struct GatherLaunch {
    const float2 *bins;
    const unsigned *end;       // after the scatter, end[t * wblocks + wblocks - 1] is the end of tile t's bin
    const unsigned *item_off;  // [tiles + 1]
    int64_t wblocks;
    float Hx, Hy, ax, ay;
    int nx, ny, tiles_x, tiles;
    float *out;                // the map
    float *part;               // [items][TH][TW] partial tiles of tiles with several items
    unsigned long long *part_fixed;  // the same memory, as fixed-point partial tiles (bin_accum_kernel)
    float scale;
};

template <int K, int RC, bool kRuns>
__global__ __launch_bounds__(tile::kThreads) void bin_gather_kernel(GatherLaunch p) {
    using S = tile::Shape<K, RC>;
    __shared__ float2 sp[tile::kPointTile];
    __shared__ int swave[tile::kThreads / 64];
    const int64_t item = blockIdx.x;
    if (item >= (int64_t)p.item_off[p.tiles]) return;  // whole workgroup: beyond the items of this map
    int lo_t = 0, hi_t = p.tiles - 1;  // tile of this item: the last t with item_off[t] <= item
    while (lo_t < hi_t) {
        const int mid = (lo_t + hi_t + 1) / 2;
        if ((int64_t)p.item_off[mid] <= item) lo_t = mid;
        else hi_t = mid - 1;
    }
    const int t = lo_t, tid = threadIdx.x;
    const int64_t k = item - p.item_off[t], parts = (int64_t)p.item_off[t + 1] - p.item_off[t];
    const int64_t e = p.end[(int64_t)t * p.wblocks + p.wblocks - 1];
    const int64_t b = t > 0 ? (int64_t)p.end[(int64_t)t * p.wblocks - 1] : 0;
    const int64_t len = e - b;
    const int64_t lo = b + len * k / parts, hi = b + len * (k + 1) / parts;
    const int x0 = (t % p.tiles_x) * S::TW, y0 = (t / p.tiles_x) * S::TH;
    const int ib = x0 + (tid & 15) * S::C, jb = y0 + (tid >> 4) * S::R;
    float tot[S::R][S::C];
    tile::tile_sums<K, S::R, S::C, false, kRuns>(p.bins, lo, hi, p.Hx, p.Hy, p.ax, p.ay, ib, jb, 0.0f, 0.0f, 0.0f,
                                                 0.0f, sp, swave, tot);
    if constexpr (kRuns) tile::apply_run_q<S::R, S::C>(tot, p.ax, p.ay);
    if (parts == 1)
        tile::store_block<S::R, S::C>(tot, p.out, p.nx, p.ny, ib, jb, p.scale);
    else
        tile::store_block<S::R, S::C>(tot, p.part + item * (S::TW * S::TH), S::TW, S::TH, ib - x0, jb - y0, 1.0f);
}

// Compact kernels with small supports (tile::accum_applies): each binned point
// adds its own terms to the tile in LDS (tile::accum_point), instead of every
// thread of the tile testing every point (the gather above spends hundreds of
// lane operations per in-support pair when the support covers a few percent of
// the tile).  Each thread takes a contiguous run of the item's points, so that
// the lanes of a wave work on distant stretches of the tracks and seldom hit one
// node at once.  A tile with one item writes scale * acc / 2^32 (one rounding),
// otherwise its fixed-point partial tile for item_reduce_fixed_kernel, so that
// the map does not depend on how a tile's points are cut into items.
template <int K, int RC>
__global__ __launch_bounds__(tile::kThreads) void bin_accum_kernel(GatherLaunch p) {
    constexpr int TW = 16 * RC, TH = 16 * RC;
    __shared__ unsigned long long acc[TW * TH];
    const int64_t item = blockIdx.x;
    if (item >= (int64_t)p.item_off[p.tiles]) return;  // whole workgroup: beyond the items of this map
    int lo_t = 0, hi_t = p.tiles - 1;  // tile of this item: the last t with item_off[t] <= item
    while (lo_t < hi_t) {
        const int mid = (lo_t + hi_t + 1) / 2;
        if ((int64_t)p.item_off[mid] <= item) lo_t = mid;
        else hi_t = mid - 1;
    }
    const int t = lo_t, tid = threadIdx.x;
    const int64_t k = item - p.item_off[t], parts = (int64_t)p.item_off[t + 1] - p.item_off[t];
    const int64_t e = p.end[(int64_t)t * p.wblocks + p.wblocks - 1];
    const int64_t b = t > 0 ? (int64_t)p.end[(int64_t)t * p.wblocks - 1] : 0;
    const int64_t len = e - b;
    const int64_t lo = b + len * k / parts, hi = b + len * (k + 1) / parts;
    const int x0 = (t % p.tiles_x) * TW, y0 = (t / p.tiles_x) * TH;
    for (int i = tid; i < TW * TH; i += tile::kThreads) acc[i] = 0ull;
    __syncthreads();
    const int64_t per = (hi - lo + tile::kThreads - 1) / tile::kThreads;
    const int64_t q0 = lo + per * tid, q1 = min(hi, q0 + per);
    for (int64_t q = q0; q < q1; ++q)  // binned in this tile: the support reaches it
        tile::accum_point<K, TW, TH>(p.bins[q], x0, y0, p.nx, p.ny, p.Hx, p.Hy, p.ax, p.ay, acc);
    __syncthreads();
    const double raw = 1.0 / (double)tile::kFixedOne;
    for (int i = tid; i < TW * TH; i += tile::kThreads) {
        const int gi = x0 + i % TW, gj = y0 + i / TW;
        if (parts == 1) {
            if (gi < p.nx && gj < p.ny) p.out[(int64_t)gj * p.nx + gi] = (float)((double)acc[i] * (raw * p.scale));
        } else {
            p.part_fixed[item * (TW * TH) + i] = acc[i];
        }
    }
}

// Tiles with several items: the partial tiles added in item order, scaled.
__global__ __launch_bounds__(256) void item_reduce_kernel(const float *__restrict__ part,
                                                          const unsigned *__restrict__ item_off, int tw, int th,
                                                          int tiles_x, int nx, int ny, float scale,
                                                          float *__restrict__ out) {
    const int t = blockIdx.x;
    const int64_t i0 = item_off[t], i1 = item_off[t + 1];
    if (i1 - i0 <= 1) return;
    const int x0 = (t % tiles_x) * tw, y0 = (t / tiles_x) * th;
    for (int e = threadIdx.x; e < tw * th; e += blockDim.x) {
        const int i = x0 + e % tw, j = y0 + e / tw;
        float s = 0.0f;
        for (int64_t it = i0; it < i1; ++it) s += part[it * (tw * th) + e];
        if (i < nx && j < ny) out[(int64_t)j * nx + i] = s * scale;
    }
}

// The same for fixed-point partial tiles: integer sums, then one rounding.
__global__ __launch_bounds__(256) void item_reduce_fixed_kernel(const unsigned long long *__restrict__ part,
                                                                const unsigned *__restrict__ item_off, int tw, int th,
                                                                int tiles_x, int nx, int ny, float scale,
                                                                float *__restrict__ out) {
    const int t = blockIdx.x;
    const int64_t i0 = item_off[t], i1 = item_off[t + 1];
    if (i1 - i0 <= 1) return;
    const int x0 = (t % tiles_x) * tw, y0 = (t / tiles_x) * th;
    const double raw = 1.0 / (double)tile::kFixedOne;
    for (int e = threadIdx.x; e < tw * th; e += blockDim.x) {
        const int i = x0 + e % tw, j = y0 + e / tw;
        unsigned long long s = 0ull;
        for (int64_t it = i0; it < i1; ++it) s += part[it * (tw * th) + e];
        if (i < nx && j < ny) out[(int64_t)j * nx + i] = (float)((double)s * (raw * scale));
    }
}

struct BinPlan {
    BinGeom g;
    int64_t cnt_len, scan_blocks, max_entries;
    int64_t per_item, max_items;
    size_t off_bytes, totals_bytes, bins_bytes, item_bytes, part_bytes;
};

BinPlan bin_plan(const MapArgs &a, int T) {
    BinPlan pl;
    pl.g.nx = a.nx;
    pl.g.ny = a.ny;
    pl.g.tile = T;
    pl.g.tiles_x = (a.nx + T - 1) / T;
    pl.g.tiles_y = (a.ny + T - 1) / T;
    pl.g.Hx = a.Hx;
    pl.g.Hy = a.Hy;
    pl.g.n = a.n;
    pl.g.wblocks = (a.n + kColBlock - 1) / kColBlock;
    pl.cnt_len = (int64_t)pl.g.tiles_x * pl.g.tiles_y * pl.g.wblocks;
    pl.scan_blocks = (pl.cnt_len + kScanBlock - 1) / kScanBlock;
    // Tiles a point can reach per axis: its support spans at most 2H + 1 nodes.
    const int64_t rx = std::min<int64_t>(pl.g.tiles_x, (int64_t)(2.0f * a.Hx) / T + 2);
    const int64_t ry = std::min<int64_t>(pl.g.tiles_y, (int64_t)(2.0f * a.Hy) / T + 2);
    pl.max_entries = a.n * rx * ry;
    const int64_t tiles = (int64_t)pl.g.tiles_x * pl.g.tiles_y;
    // Items of at most per_item entries: each tile has max(1, ceil(len / per_item))
    // <= 1 + len / per_item of them, so at most tiles + max_entries / per_item.
    pl.per_item = std::max<int64_t>(1024, (pl.max_entries / kTargetItems + 255) / 256 * 256);
    pl.max_items = tiles + pl.max_entries / pl.per_item;
    pl.off_bytes = (size_t)pl.cnt_len * sizeof(unsigned);
    pl.totals_bytes = (size_t)(pl.scan_blocks + 1) * sizeof(unsigned);
    pl.bins_bytes = (size_t)pl.max_entries * sizeof(float2);
    pl.item_bytes = (size_t)(tiles + 1) * sizeof(unsigned);
    const bool fixed = T == 16 * a.rc && tile::accum_applies(a.kernel_id, a.rc, a.Hx, a.Hy);
    pl.part_bytes = (size_t)pl.max_items * T * T * (fixed ? sizeof(unsigned long long) : sizeof(float));
    return pl;
}

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

template <int K, int RC>
hipError_t launch_gather_r(const GatherLaunch &p, int64_t items, hipStream_t s) {
    main_kernel_begin(s);
    if constexpr (K != kGaussian && K != kGaussTrunc && RC <= 4) {
        if (tile::accum_applies(K, RC, p.Hx, p.Hy)) {
            hipLaunchKernelGGL((bin_accum_kernel<K, RC>), dim3((unsigned)items), dim3(tile::kThreads), 0, s, p);
            main_kernel_end(s);
            return hipGetLastError();
        }
    }
    // the truncated Gaussian takes the runs of the Gaussian (two exp2 per run, then the support mask)
    if (K == kGaussTrunc && p.ax <= kMaxRunScale && p.ay <= kMaxRunScale)
        hipLaunchKernelGGL((bin_gather_kernel<K, RC, K == kGaussTrunc>), dim3((unsigned)items), dim3(tile::kThreads),
                           0, s, p);
    else
        hipLaunchKernelGGL((bin_gather_kernel<K, RC, false>), dim3((unsigned)items), dim3(tile::kThreads), 0, s, p);
    main_kernel_end(s);
    return hipGetLastError();
}

template <int K>
hipError_t launch_gather(const GatherLaunch &p, int rc, int64_t items, hipStream_t s) {
    switch (rc) {
    case 2: return launch_gather_r<K, 2>(p, items, s);
    case 4: return launch_gather_r<K, 4>(p, items, s);
    case 8: return launch_gather_r<K, 8>(p, items, s);
    default: return hipErrorInvalidValue;
    }
}

// Count, scan and scatter into workspace ws (layout: counts/ends, scan totals,
// bins); the bins then hold each tile's points contiguously, in tile order.
hipError_t scatter_bins(const MapArgs &a, const BinPlan &pl, char *w, unsigned **off_out, float2 **bins_out,
                        hipStream_t s, bool ordered = true) {
    unsigned *off = reinterpret_cast<unsigned *>(w);
    unsigned *totals = reinterpret_cast<unsigned *>(w + align256(pl.off_bytes));
    float2 *bins = reinterpret_cast<float2 *>(w + align256(pl.off_bytes) + align256(pl.totals_bytes));
    hipError_t e = launch_fill_zero(reinterpret_cast<float *>(off), pl.cnt_len, s);  // 0.0f is all-zero bits
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(bin_count_kernel, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, s, pl.g, a.pts, off);
    hipLaunchKernelGGL(scan_blocks_kernel, dim3((unsigned)pl.scan_blocks), dim3(256), 0, s, off, pl.cnt_len, totals);
    hipLaunchKernelGGL(scan_totals_kernel, dim3(1), dim3(256), 0, s, totals, pl.scan_blocks);
    hipLaunchKernelGGL(scan_add_kernel, dim3((unsigned)((pl.cnt_len + 255) / 256)), dim3(256), 0, s, off,
                       pl.cnt_len, static_cast<const unsigned *>(totals));
    if (ordered)
        hipLaunchKernelGGL(bin_scatter_kernel, dim3((unsigned)((pl.g.wblocks + 3) / 4)), dim3(256), 0, s, pl.g,
                           a.pts, off, bins);
    else
        hipLaunchKernelGGL(bin_scatter_free_kernel, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, s, pl.g,
                           a.pts, off, bins);
    *off_out = off;
    *bins_out = bins;
    return hipGetLastError();
}

size_t scatter_bytes(const BinPlan &pl) {
    return align256(pl.off_bytes) + align256(pl.totals_bytes) + align256(pl.bins_bytes);
}

}  // namespace

size_t scan_u32_totals_bytes(int64_t len) { return (size_t)((len + kScanBlock - 1) / kScanBlock + 1) * sizeof(unsigned); }

hipError_t launch_scan_u32(unsigned *a, int64_t len, unsigned *totals, hipStream_t s) {
    const int64_t blocks = (len + kScanBlock - 1) / kScanBlock;
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(scan_blocks_kernel, dim3((unsigned)blocks), dim3(256), 0, s, a, len, totals);
    hipLaunchKernelGGL(scan_totals_kernel, dim3(1), dim3(256), 0, s, totals, blocks);
    hipLaunchKernelGGL(scan_add_kernel, dim3((unsigned)((len + 255) / 256)), dim3(256), 0, s, a, len,
                       static_cast<const unsigned *>(totals));
    return hipGetLastError();
}

bool binning_applies(const MapArgs &a) {
    if (a.kernel_id == kGaussian || a.n < 4096 || !valid_rc(a.rc)) return false;
    const float T = (float)(16 * a.rc);
    if (a.Hx > T || a.Hy > T) return false;  // at most 3 x 3 tiles per point
    const BinPlan pl = bin_plan(a, 16 * a.rc);
    return pl.cnt_len <= (int64_t(1) << 26) && pl.max_entries <= (int64_t(1) << 30);
}

size_t binned_workspace_bytes(const MapArgs &a) {
    const BinPlan pl = bin_plan(a, 16 * a.rc);
    return scatter_bytes(pl) + align256(pl.item_bytes) + pl.part_bytes;
}

bool tile_bins_fit(const MapArgs &a, int tile) {
    if (a.n < 1 || a.Hx > (float)tile || a.Hy > (float)tile) return false;
    const BinPlan pl = bin_plan(a, tile);
    return pl.cnt_len <= (int64_t(1) << 26) && pl.max_entries <= (int64_t(1) << 30);
}

size_t tile_bins_bytes(const MapArgs &a, int tile) { return scatter_bytes(bin_plan(a, tile)); }

hipError_t launch_tile_bins(const MapArgs &a, int tile, void *ws, hipStream_t s, TileBins *out) {
    const BinPlan pl = bin_plan(a, tile);
    unsigned *off = nullptr;
    float2 *bins = nullptr;
    hipError_t e = scatter_bins(a, pl, static_cast<char *>(ws), &off, &bins, s);
    out->bins = bins;
    out->end = off;
    out->wblocks = pl.g.wblocks;
    out->tiles_x = pl.g.tiles_x;
    out->tiles_y = pl.g.tiles_y;
    out->max_entries = pl.max_entries;
    return e;
}

hipError_t launch_binned(const MapArgs &a, void *ws, hipStream_t s) {
    const BinPlan pl = bin_plan(a, 16 * a.rc);
    const int T = 16 * a.rc;
    char *w = static_cast<char *>(ws);
    unsigned *item_off = reinterpret_cast<unsigned *>(w + scatter_bytes(pl));
    float *part = reinterpret_cast<float *>(w + scatter_bytes(pl) + align256(pl.item_bytes));
    unsigned *off = nullptr;
    float2 *bins = nullptr;
    // The fixed-point accumulation does not need a tile's points in order.
    const bool fixed = tile::accum_applies(a.kernel_id, a.rc, a.Hx, a.Hy);
    hipError_t e = scatter_bins(a, pl, w, &off, &bins, s, !fixed);
    if (e != hipSuccess) return e;
    const int tiles = pl.g.tiles_x * pl.g.tiles_y;
    hipLaunchKernelGGL(item_scan_kernel, dim3(1), dim3(kItemScan), 0, s, static_cast<const unsigned *>(off),
                       pl.g.wblocks, tiles, pl.per_item, item_off);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    GatherLaunch p;
    p.bins = bins;
    p.end = off;
    p.item_off = item_off;
    p.wblocks = pl.g.wblocks;
    p.Hx = a.Hx;
    p.Hy = a.Hy;
    p.ax = a.ax;
    p.ay = a.ay;
    p.nx = a.nx;
    p.ny = a.ny;
    p.tiles_x = pl.g.tiles_x;
    p.tiles = tiles;
    p.out = a.out;
    p.part = part;
    p.part_fixed = reinterpret_cast<unsigned long long *>(part);
    p.scale = a.scale;
    switch (a.kernel_id) {
    case kUniform: e = launch_gather<kUniform>(p, a.rc, pl.max_items, s); break;
    case kTriangular: e = launch_gather<kTriangular>(p, a.rc, pl.max_items, s); break;
    case kEpanechnikov: e = launch_gather<kEpanechnikov>(p, a.rc, pl.max_items, s); break;
    case kQuartic: e = launch_gather<kQuartic>(p, a.rc, pl.max_items, s); break;
    case kTriweight: e = launch_gather<kTriweight>(p, a.rc, pl.max_items, s); break;
    case kTricube: e = launch_gather<kTricube>(p, a.rc, pl.max_items, s); break;
    case kCosine: e = launch_gather<kCosine>(p, a.rc, pl.max_items, s); break;
    case kGaussTrunc: e = launch_gather<kGaussTrunc>(p, a.rc, pl.max_items, s); break;
    default: return hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
    if (fixed)  // the same test as launch_gather_r
        hipLaunchKernelGGL(item_reduce_fixed_kernel, dim3((unsigned)tiles), dim3(256), 0, s,
                           static_cast<const unsigned long long *>(p.part_fixed),
                           static_cast<const unsigned *>(item_off), T, T, pl.g.tiles_x, a.nx, a.ny, a.scale, a.out);
    else
        hipLaunchKernelGGL(item_reduce_kernel, dim3((unsigned)tiles), dim3(256), 0, s, part,
                           static_cast<const unsigned *>(item_off), T, T, pl.g.tiles_x, a.nx, a.ny, a.scale, a.out);
    return hipGetLastError();
}

}  // namespace kde
