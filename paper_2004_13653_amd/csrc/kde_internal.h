// Internal declarations shared by the HIP translation units of libkde.
// Nothing here is part of the C ABI (include/kde.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <utility>
#include <vector>

namespace kde {

// Evaluation paths (the precision argument of kde_eval).
enum Precision : int {
    kPrecFp32Direct = 0,
    kPrecFp16 = 1,
    kPrecBf16 = 2,
    kPrecFp16x3 = 3,
    kPrecBf16x3 = 4,
};

enum KernelId : int {
    kUniform = 0,
    kTriangular = 1,
    kEpanechnikov = 2,
    kQuartic = 3,
    kTriweight = 4,
    kTricube = 5,
    kGaussian = 6,
    kCosine = 7,
    kGaussTrunc = 8,  // internal: the Gaussian truncated at |u| <= kTruncSigmas (KDE_TRUNCATE)
};

// KDE_TRUNCATE: support half-width of the truncated Gaussian in bandwidths.  The
// map arguments then carry H = kTruncSigmas * (h / spacing) as the support and
// a = arg_scale(kGaussian, h / spacing) as the argument scale.
constexpr float kTruncSigmas = 8.0f;

// Normalising constant c of the 1-D factor k(u) = c g(u) (Table I); the kernels
// accumulate products of g and the epilogue multiplies by c^2.
double kernel_norm(int kernel_id);

// Scale that turns a grid-unit difference d = node - point into the argument of
// g: the Gaussian evaluates g = exp2(-(d a)^2) with a = sqrt(log2(e)/2)/H, the
// compact kernels evaluate g(|d|/H) with a = 1/H.
float arg_scale(int kernel_id, float H);

struct MapArgs {
    const float2 *pts;  // [n] grid units
    int64_t n;
    int kernel_id;
    float Hx, Hy;       // bandwidths in grid units
    float ax, ay;       // argument scales (arg_scale)
    int nx, ny;
    float scale;        // c^2 / (n hx hy), or c^2 for raw sums
    float *out;         // [ny][nx]
    int rc = 0;         // FP32 direct: register block side (2, 4 or 8; tile side 16 rc)
};

// Gaussian runs (consecutive nodes' factors as P_0 B^r times a per-position
// constant, see kde_tile.h and kde_sep.hip) are used when the argument scale
// a = sqrt(log2(e) / 2) / H is at most this (H >= 1.05 grid units), which keeps
// the run's intermediate values within a factor 2^8 of the factors.
constexpr float kMaxRunScale = 0.8f;

// Register-block sides the FP32 direct kernels are built for.
constexpr int kTileShapes[3] = {2, 4, 8};
inline bool valid_rc(int rc) { return rc == 2 || rc == 4 || rc == 8; }

// FP32 direct path: enqueues the map on `stream`; ws holds
// direct_workspace_bytes(a) bytes of device scratch.  Returns the launch status.
hipError_t launch_direct(const MapArgs &a, void *ws, hipStream_t stream);

// Bytes of workspace launch_direct needs for these arguments.
size_t direct_workspace_bytes(const MapArgs &a);

// Support binning for the compact kernels (FP32 direct path): used when the
// support reaches at most 3 x 3 tiles (of side 16 a.rc) per point and the count
// table stays small.
bool binning_applies(const MapArgs &a);
size_t binned_workspace_bytes(const MapArgs &a);
hipError_t launch_binned(const MapArgs &a, void *ws, hipStream_t stream);

// Points binned by square tiles of side `tile` (each point registered in every
// tile its support rectangle [X +- Hx] x [Y +- Hy] reaches; needs Hx, Hy <= tile):
// bins holds each tile's points contiguously in tile order, point order kept;
// tile t's points are bins[end[t*wblocks - 1] .. end[t*wblocks + wblocks - 1])
// (begin 0 for t = 0).  max_entries bounds the number of registrations.
struct TileBins {
    const float2 *bins;
    const unsigned *end;
    int64_t wblocks;
    int tiles_x, tiles_y;
    int64_t max_entries;
};
bool tile_bins_fit(const MapArgs &a, int tile);
size_t tile_bins_bytes(const MapArgs &a, int tile);
hipError_t launch_tile_bins(const MapArgs &a, int tile, void *ws, hipStream_t s, TileBins *out);

// In-place exclusive scan of a[len] (uint32, sums below 2^32); totals holds
// scan_u32_totals_bytes(len) bytes and receives the grand total at
// totals[ceil(len / 1024)].
size_t scan_u32_totals_bytes(int64_t len);
hipError_t launch_scan_u32(unsigned *a, int64_t len, unsigned *totals, hipStream_t s);

// Douglas-Peucker compression of merged tracks (kde_dp.hip).
struct DpArgs {
    const double2 *xy;      // [n] metres
    int64_t n;
    const int64_t *start;   // [n_tracks + 1] track offsets (device)
    int64_t n_tracks;
    double eps;
    uint8_t *keep;          // [n] output
    double2 *out_xy;        // [n] compacted kept points, or nullptr
    int64_t *out_lengths;   // [n_tracks] kept points per track, or nullptr
    int64_t *out_start;     // [n_tracks + 1] offsets of the compressed tracks, or nullptr
};
size_t dp_workspace_bytes(int64_t n);
// Runs the level loop (synchronising `stream` once per group of levels) and
// returns the number of kept points in *n_kept.
hipError_t run_dp(const DpArgs &a, void *ws, hipStream_t stream, int64_t *n_kept);

// Compression-quality measures (kde_metrics.hip): per track |T|, |T'| and the
// DTW distance; totals over the set.  Same layout as the C ABI's
// kde_track_metrics.
struct MetricsTotals {
    int64_t n_original, n_compressed;
    double cr_percent, length_original, length_compressed, rll, dtw_mean, dtw_std;
};
constexpr int64_t kMaxTrackPoints = (int64_t)1 << 30;  // per track, either set
struct MetricsArgs {
    const double2 *xo;   // [n_o] original points
    int64_t n_o;
    const int64_t *so;   // [n_tracks + 1] original offsets (device)
    const double2 *xc;   // [n_c] compressed points
    int64_t n_c;
    const int64_t *sc;   // [n_tracks + 1] compressed offsets (device)
    int64_t n_tracks;
    double *len_o, *len_c, *dtw;  // [n_tracks] each, or nullptr (then workspace)
};
size_t metrics_workspace_bytes(int64_t n_o, int64_t n_c, int64_t n_tracks, bool per_track_given);
// Checks the offsets on the device (the compute kernels skip all work when they
// do not rise from 0 to n_o and n_c with tracks under kMaxTrackPoints), computes,
// and synchronises once: hipErrorInvalidValue for bad offsets, else the totals
// in *host_out (if given).
hipError_t run_metrics(const MetricsArgs &a, void *ws, hipStream_t stream, MetricsTotals *host_out);

// Matrix-core separable path (precision kPrecFp16 .. kPrecBf16x3).  Compact
// kernels (and the truncated Gaussian) whose support fits a 256-node tile run
// banded: only the (tile, point) pairs the support reaches are multiplied.
hipError_t launch_sep(const MapArgs &a, int precision, void *ws, hipStream_t stream);
size_t sep_workspace_bytes(const MapArgs &a, int precision);

// Dense Gaussian maps of one matrix-core precision in one launch of the 8-wave
// kernel (runs true: sep_dense_batchable 1, the multiplicative runs apply) or
// of the kernel that evaluates every factor (runs false: 2, narrower
// bandwidths), plus one padding and one split-reduction launch for all of
// them.  A map's points are split only as far as its share of the batch's work
// asks for, never further than launch_sep splits them, so a result equals
// launch_sep's up to the FP32 order of the split sums.  ws holds
// sep_dense_batch_bytes; the map table goes up from a library-owned pinned
// buffer (release_dense_stage).  sep_dense_batchable is 0 for other maps.
int sep_dense_batchable(const MapArgs &a);
size_t sep_dense_batch_bytes(const MapArgs *maps, int n, int precision);
hipError_t launch_sep_dense_batch(const MapArgs *maps, int n, int precision, bool runs, void *ws,
                                  hipStream_t stream);
void release_dense_stage();

// A compact map that the persistent launch sums by fixed-point accumulation
// (supports spanning few nodes) rather than by the gather.
bool batch_accumulates(const MapArgs &a);

// Batched maps (FP32 direct path) in one persistent launch; use_graph captures
// the launch sequence once per batch shape and replays it (ws unused then).
hipError_t run_batched(const MapArgs *args, int n_maps, bool use_graph, void *ws_eager, size_t ws_bytes,
                       hipStream_t stream);
size_t batched_workspace_bytes(const MapArgs *args, int n_maps);
void release_batched_graphs();

// Adjoints.  launch_vjp writes grad[n][2] = (fx Tx_p, fy Ty_p) (if grad is not
// null) and per-workgroup FP64 sums (Ux, Uy, Q) into part[vjp_blocks(n)][3];
// launch_lscv writes per-workgroup FP64 sums (SA, SAX, SAY, SB, SBX, SBY) into
// part[lscv_blocks(n, kernel_id)][6].  See kde_adjoint.hip for the definitions.
int64_t vjp_blocks(int64_t n);
hipError_t launch_vjp(const float2 *pts, int64_t n, int kernel_id, float Hx, float Hy, const float *gbar, int nx,
                      int ny, float fx, float fy, float *grad, double *part, hipStream_t stream);
// Gaussian VJP on matrix cores (kde_vjp_mfma.hip): the same outputs as
// launch_vjp (grad, and the per-workgroup sums at the start of ws in the
// vjp_blocks(n) x 3 layout), from BF16 hi/lo contractions; ws holds
// vjp_mfma_workspace_bytes.
size_t vjp_mfma_workspace_bytes(int64_t n, int nx, int ny);
hipError_t launch_vjp_mfma(const float2 *pts, int64_t n, float Hx, float Hy, const float *gbar, int nx, int ny,
                           float fx, float fy, float *grad, void *ws, hipStream_t stream);
// launch_lscv needs lscv_workspace_bytes of workspace and leaves the
// lscv_blocks partial rows at its start.  Compact kernels visit only the tiles
// of spatially sorted points whose pairs can be in support (nx, ny fix the
// sort's cell grid, a locality heuristic with no effect on the sums).
int64_t lscv_blocks(int64_t n, int kernel_id);
size_t lscv_workspace_bytes(int64_t n, int kernel_id);
hipError_t launch_lscv(const float2 *pts, int64_t n, int kernel_id, float Hx, float Hy, int nx, int ny, void *ws,
                       hipStream_t stream);

// Spatial sort (kde_sort.hip): out[n] = the points ordered by the Z-order code
// of their cell (square cells of side `cell` grid units, 1024 per axis from the
// origin, outside points clamped to the border cells), stable, deterministic.
size_t spatial_sort_bytes(int64_t n);
hipError_t launch_spatial_sort(const float2 *pts, int64_t n, float cell, void *ws, float2 *out, hipStream_t s);
// Cell side for bandwidths Hx, Hy on an nx x ny grid: max(Hx, Hy), at least 1/1024 of the grid.
float spatial_sort_cell(float Hx, float Hy, int nx, int ny);

// out[i] = scale * sum_{s < splits} part[s * plane + i], summed in split order.
hipError_t launch_reduce_splits(const float *part, int splits, int64_t plane, float scale, float *out,
                                hipStream_t stream);

// Zero-fill kernel (used for empty inputs; no memset nodes in captured graphs).
hipError_t launch_fill_zero(float *out, int64_t count, hipStream_t stream);

// The paper's binned visualisation (kde_binned.hip): count matrix with gap
// filling, then the separable convolution of the counts.
constexpr int kMaxTapRadius = 128;  // taps |s| <= a, |t| <= b with a, b <= this
struct BinnedConvArgs {
    const uint32_t *counts;               // [ny][nx]
    int nx, ny, kernel_id;
    float Hx, Hy;                         // bandwidths in cells
    int a, b;                             // tap radii in cells
    double c2_over_hxhy;                  // c^2 / (hx hy), or c^2 for raw sums
    bool raw;                             // true: no division by the number of counted cells
    const unsigned long long *total;      // device: number of counted cells (density only)
    float *out;                           // [ny][nx]
};
hipError_t launch_bin_counts(const float2 *pts, int64_t n, const int32_t *labels, int nx, int ny, uint32_t *counts,
                             unsigned long long *total, hipStream_t s);
size_t conv_workspace_bytes(int nx, int ny);
hipError_t launch_conv_counts(const BinnedConvArgs &c, void *ws, hipStream_t s);

// Tile-shape autotuner cache (kde_autotune.cpp).  Keys and choices are
// described there; the timing runs live in kde_api.cpp.
namespace tune {
struct Entry {
    std::string choice;
    std::vector<std::pair<std::string, double>> ms;  // candidate -> measured ms
};
bool valid_choice(const std::string &key, const std::string &choice);
bool enabled();
void set_enabled(bool on);
int forced();  // 0, or the register-block side every FP32 direct map uses
void set_forced(int rc);
bool lookup(const std::string &key, std::string *choice);
void store(const std::string &key, const Entry &e);
bool load(const char *path, std::string *err);
bool save(const char *path, std::string *err);
std::string dump();
void clear();
}  // namespace tune

// Measurement hook: the launchers call these right before and after the launch of
// their main kernel; they record the events a caller armed with
// kde_time_next_main_kernel on this thread (and do nothing otherwise).
void main_kernel_begin(hipStream_t stream);
void main_kernel_end(hipStream_t stream);

}  // namespace kde
