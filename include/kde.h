/*
 * kde.h -- C ABI of libkde, an MI355X (gfx950) implementation of the kernel
 * density estimation (KDE) heat map of Huang, Li, Zhang and Liu, "GPU-Accelerated
 * Compression and Visualization of Large-Scale Vessel Trajectories in Maritime
 * IoT Industries" (arXiv 2004.13653), Sec. III-C and IV-B.
 *
 * The map.  For points (x_p, y_p), p = 0..n-1, bandwidths hx, hy > 0 and one of
 * the eight product kernels f(s,t) = k(s) k(t) of Table I, every grid node
 * (gx_i, gy_j) receives
 *
 *     S[j][i] = sum_p k((gx_i - x_p)/hx) * k((gy_j - y_p)/hy)
 *     out[j*nx + i] = S[j][i] / (n * hx * hy)          (or S with KDE_RAW_SUM)
 *
 * This is the convolution of Eq. (7) written as a direct sum over the points
 * instead of over a binned count matrix.  The indicator I(.) of Eq. (8) is read
 * as |u| <= 1 (inclusive) on the scaled argument u = (node - point)/h, the
 * support on which every Table I constant normalises k to unit mass; the
 * Gaussian has no indicator.
 *
 * Grid.  nx x ny nodes, gx_i = xmin + i*dx with dx = (xmax - xmin)/(nx - 1), both
 * box edges on nodes (the node spacing of Eq. (5)-(6)); rows j follow y.  Output
 * is row-major, x fastest (the density-matrix index order of Algorithm 3).
 *
 * Points on the device are FP32 "grid units": X_p = fl32((x_p - xmin)/dx), Y_p =
 * fl32((y_p - ymin)/dy), interleaved [n][2].  kde_to_grid_units produces them on
 * the host in FP64 with a single rounding.  Bandwidths are passed in world units
 * and converted to Hx = fl32(hx/dx), Hy = fl32(hy/dy) inside the library.
 *
 * Conventions for every call:
 *  - Return value: KDE_OK (0) or a negative kde_status.  On any failure
 *    kde_last_error() returns a message; it is thread-local and valid until the
 *    next call on the same thread.  No C++ exception crosses this interface.
 *  - Arguments are validated before anything is launched: a KDE_EINVAL return
 *    has written nothing and launched nothing.
 *  - Device buffers belong to the caller; the library never frees them.  The
 *    library owns grid handles and a workspace per (device, stream) that is
 *    reused across calls and released by kde_shutdown().
 *  - Device work is enqueued on `stream` (a hipStream_t; NULL = the null
 *    stream) and returns before it completes, except where a call writes a
 *    host scalar, which synchronises `stream` first.
 *  - Non-finite point coordinates are not checked (that would need a device
 *    pass); they yield NaN (Gaussian) or no contribution (compact kernels).
 */
#ifndef KDE_H
#define KDE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum kde_status {
    KDE_OK = 0,
    KDE_EINVAL = -1,       /* bad argument; nothing written or launched */
    KDE_ENOMEM = -2,       /* workspace allocation failed */
    KDE_EHIP = -3,         /* HIP runtime error (message in kde_last_error) */
    KDE_EUNSUPPORTED = -4  /* valid request this library does not implement */
} kde_status;

/* Kernel ids in Table I order. */
enum {
    KDE_UNIFORM = 0,      /* k(u) = 1/2                  I(u) */
    KDE_TRIANGULAR = 1,   /* k(u) = 1 - |u|              I(u) */
    KDE_EPANECHNIKOV = 2, /* k(u) = 3/4 (1 - u^2)        I(u) */
    KDE_QUARTIC = 3,      /* k(u) = 15/16 (1 - u^2)^2    I(u) */
    KDE_TRIWEIGHT = 4,    /* k(u) = 35/32 (1 - u^2)^3    I(u) */
    KDE_TRICUBE = 5,      /* k(u) = 70/81 (1 - |u|^3)^3  I(u) */
    KDE_GAUSSIAN = 6,     /* k(u) = exp(-u^2/2)/sqrt(2 pi)    */
    KDE_COSINE = 7,       /* k(u) = pi/4 cos(pi u/2)     I(u) */
    KDE_NUM_KERNELS = 8
};

/* Evaluation paths ("precision" argument of kde_eval). */
enum {
    KDE_FP32_DIRECT = 0, /* FP32 direct sum over all pairs (compact kernels skip
                            pairs outside the support); FP32 accumulation */
    KDE_FP16_SEP = 1,    /* separable form S = Gy Gx^T on matrix cores: 1-D
                            factors rounded to FP16, FP32 accumulation */
    KDE_BF16_SEP = 2,    /* the same with BF16 factors */
    KDE_FP16X3_SEP = 3,  /* FP16 hi/lo split: Gy_hi Gx_hi^T + Gy_hi Gx_lo^T +
                            Gy_lo Gx_hi^T, FP32 accumulation */
    KDE_BF16X3_SEP = 4   /* the same split with BF16 */
};

/* Flags. */
#define KDE_RAW_SUM 1u          /* the map is S instead of S/(n hx hy) */
#define KDE_GRID_UNIT_GRADS 2u  /* kde_backward: grad_points as dL/dX_p, dL/dY_p in grid units */
#define KDE_BATCH_EAGER 4u      /* kde_eval_batched: launch directly instead of replaying a graph */
#define KDE_TRUNCATE 8u         /* kde_eval, Gaussian, KDE_FP32_DIRECT: drop pairs beyond 8 bandwidths */
#define KDE_VJP_FP32 16u        /* kde_backward, Gaussian: per-pair FP32 sums instead of matrix cores */

typedef struct kde_grid kde_grid; /* opaque, immutable, library-owned */

/* Creates a grid of nx x ny nodes spanning [xmin, xmax] x [ymin, ymax] (world
 * units, both edges on nodes): the node spacing dx = (xmax - xmin)/(nx - 1),
 * dy = (ymax - ymin)/(ny - 1) of Eq. (5)-(6), on which every map is evaluated.  Requires finite bounds with xmin < xmax,
 * ymin < ymax, and 2 <= nx, ny <= 65536 (the node spacing divides by nx - 1).
 * *out receives the handle; release it with kde_destroy_grid. */
int kde_create_grid(double xmin, double xmax, double ymin, double ymax, int32_t nx, int32_t ny,
                    kde_grid **out);

/* Releases a grid handle (NULL is ignored). */
void kde_destroy_grid(kde_grid *g);

/* Reports the node counts and spacings of a grid; any output may be NULL. */
int kde_grid_shape(const kde_grid *g, int32_t *nx, int32_t *ny, double *dx, double *dy);

/* Host-side input conditioning: world points xy[n][2] (FP64, host) to grid units
 * out[n][2] (FP32, host), X = fl32((x - xmin)/dx), Y = fl32((y - ymin)/dy).
 * Points outside the box are allowed (they still contribute to nearby nodes). */
int kde_to_grid_units(const kde_grid *g, const double *xy, int64_t n, float *out);

/* Bandwidths in grid units: Hx = fl32(hx/dx), Hy = fl32(hy/dy).  hx, hy must be
 * finite and > 0 and give Hx, Hy in [2^-20, 2^20]. */
int kde_bandwidth_units(const kde_grid *g, double hx, double hy, float *Hx, float *Hy);

/* The heat map (Sec. III-C, Eq. (7)-(8), Table I).
 *   points    device, FP32 [n][2] grid units (may be NULL when n == 0)
 *   n         number of points, 0 <= n < 2^31; n == 0 writes a zero map
 *   kernel_id KDE_UNIFORM .. KDE_COSINE
 *   hx, hy    bandwidths in world units (see kde_bandwidth_units)
 *   g         grid handle
 *   out       device, FP32 [ny][nx], fully overwritten
 *   precision KDE_FP32_DIRECT or one of the *_SEP matrix-core paths
 *   flags     0, KDE_RAW_SUM, KDE_TRUNCATE (or both)
 *   stream    hipStream_t or NULL
 * KDE_TRUNCATE (not in the paper; Gaussian only, else KDE_EINVAL): pairs with
 * |i - X| > 8 Hx or |j - Y| > 8 Hy are dropped, so the Gaussian gets the compact
 * kernels' treatment: support binning on the FP32 path, banded (block-sparse)
 * products on the matrix-core paths.  Each dropped pair is below
 * e^-32 = 1.3e-14 of the largest pair value, so the map is below the full one by
 * at most n * 1.3e-14 of the peak pair value.
 * Matrix-core paths with a compact kernel (or KDE_TRUNCATE) whose support is at
 * most 256 grid units run banded: points are binned by 256 x 256 tile and only
 * the tiles a point reaches multiply it. */
int kde_eval(const float *points, int64_t n, int32_t kernel_id, double hx, double hy, const kde_grid *g,
             float *out, int32_t precision, uint32_t flags, void *stream);

/* Allocation-free kde_eval, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, validation, paths and results as kde_eval; the
 * workspace is a fixed device array of KDE_NOALLOC_SCRATCH_BYTES that every GPU
 * the library runs on holds until the process ends, and the call makes no
 * hipMalloc, hipFree or other allocating call.  Differences from kde_eval:
 *  - a map whose workspace would exceed KDE_NOALLOC_SCRATCH_BYTES is rejected
 *    with KDE_EINVAL before any launch (dense matrix-core maps need 64 MiB of
 *    split partial planes plus 8 bytes per point, e.g. 4*10^6 points on 2048^2
 *    fit; FP32 direct and banded maps need less);
 *  - the FP32 direct path uses the cached, forced or default tile shape and
 *    never runs tuning launches.
 * All calls on one GPU share that GPU's array and leave it holding the last
 * call's contents (every launch sequence clears what it needs zeroed with its
 * own fill kernel): calls on one GPU that overlap in time (different streams or
 * host threads, not ordered by the caller) race on it and give undefined maps.
 * Calls ordered on one stream are safe. */
#define KDE_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)
int kde_eval_noalloc(const float *points, int64_t n, int32_t kernel_id, double hx, double hy, const kde_grid *g,
                     float *out, int32_t precision, uint32_t flags, void *stream);

/* One map of a batch: the arguments of kde_eval except stream. */
typedef struct kde_map {
    const float *points; /* device [n][2] grid units of `grid` */
    int64_t n;
    int32_t kernel_id;
    int32_t precision; /* KDE_FP32_DIRECT or one of the *_SEP matrix-core paths */
    double hx, hy;     /* world units */
    const kde_grid *grid;
    float *out;        /* device [ny][nx] */
    uint32_t flags;    /* 0 or KDE_TRUNCATE (Gaussian only) */
    uint32_t reserved; /* must be 0 */
} kde_map;

/* Evaluates n_maps maps (host array of descriptors; not in the paper, which maps
 * one data set at a time).  The FP32 direct maps without KDE_TRUNCATE run in
 * one persistent launch: the batch is cut into (map, pixel tile, point range)
 * items, longest first, pulled by persistent workgroups from an atomic counter;
 * each such map's output equals what kde_eval(..., KDE_FP32_DIRECT, ...)
 * computes up to FP32 rounding order, and bit for bit for compact kernels whose
 * supports span at most 225 tried nodes, (floor(2Hx)+3)(floor(2Hy)+3) <= 225
 * (441 for the cosine), with n >= 4096 and kde_eval on tiles of side 32 or 64
 * (its default): both paths sum those in 64-bit fixed point, exactly.  The other maps follow on the
 * same stream: the Gaussian maps of each matrix-core precision (n > 0) as one
 * launch of the contraction kernel over all their tiles and point splits
 * (bandwidths of at least 1.05 node spacings, with multiplicative runs) and one
 * of the kernel that evaluates every factor (narrower bandwidths), the
 * truncated Gaussians as individual launches of the kde_eval path.  The batched
 * Gaussian maps fill the GPU together, so a map's points are split only as far
 * as its share of the batch's work asks for (never further than kde_eval splits
 * them): its output equals kde_eval's up to the FP32 order of the split sums;
 * the individual launches equal kde_eval's bit for bit.  A small table of the
 * Gaussian maps goes up from one of a few pinned buffers the library keeps per
 * device until kde_shutdown().  Every descriptor is validated before anything
 * is launched; output buffers must not overlap each other or any point buffer.
 * By default the persistent part is captured into a hipGraph the first time a
 * batch shape (per map: kernel, tile side, grid size, point count) is seen: its
 * item list goes up once, and the graph copies the map descriptors (pointers,
 * bandwidths) from a pinned staging buffer, then launches the kernels; later
 * calls of the shape write the descriptors and replay it.  The library keeps
 * one device buffer and pinned staging buffer per captured shape until
 * kde_shutdown().  A call on a shape that is still running waits for that run
 * to finish before reusing its staging buffer.  flags: KDE_RAW_SUM,
 * KDE_BATCH_EAGER (no graph; the call synchronises `stream`). */
int kde_eval_batched(const kde_map *maps, int32_t n_maps, uint32_t flags, void *stream);

/* Adjoint of kde_eval (vector-Jacobian product; not in the paper).  Given
 * grad_out = dL/d(out) (device FP32 [ny][nx]) for the map kde_eval produces with
 * the same points, kernel, bandwidths, grid and KDE_RAW_SUM flag, writes
 *   grad_points  device FP32 [n][2]: dL/dx_p, dL/dy_p in world units (dL/dX_p,
 *                dL/dY_p in grid units with KDE_GRID_UNIT_GRADS), or NULL
 *   grad_h       host FP64 [2]: dL/dhx, dL/dhy in world units, or NULL; when
 *                non-NULL the call synchronises `stream`
 * Per pair FP32; bandwidth sums reduced in FP64 in a fixed order.  The
 * derivative of k is taken from its formula inside the support (at the kink
 * u = 0 of the triangular kernel, 0).  The Gaussian uses its separability
 * (Sec. III-C): the sums become the contractions Gbar^T Gy and Gbar Gx on
 * matrix cores with BF16 hi/lo operands (three products, FP32 accumulation;
 * relative errors of a few 1e-6), unless KDE_VJP_FP32 asks for the per-pair
 * FP32 evaluation or the matrix-core workspace would exceed 4 GiB.
 * flags: KDE_RAW_SUM | KDE_GRID_UNIT_GRADS | KDE_VJP_FP32. */
int kde_backward(const float *points, int64_t n, int32_t kernel_id, double hx, double hy, const kde_grid *g,
                 const float *grad_out, float *grad_points, double *grad_h, uint32_t flags, void *stream);

/* Least-squares cross-validation score of the bandwidth (Rudemo 1982, Bowman
 * 1984; not in the paper), in world units:
 *   LSCV = 1/(n^2 hx hy) sum_{p,q} kbar(dx_pq/hx) kbar(dy_pq/hy)
 *        - 2/(n(n-1) hx hy) sum_{p!=q} k(dx_pq/hx) k(dy_pq/hy),   kbar = k * k,
 * and its gradient with respect to (hx, hy).  points as for kde_eval (the grid
 * only fixes the units), n >= 2, any Table I kernel (kbar: the Gaussian's is the
 * N(0, 2) density, the others' piecewise polynomials on |u| < 2, the cosine's
 * a closed form).  The derivative of k is taken from its formula inside the
 * support (the uniform kernel's jumps at the support edge contribute nothing).
 * Per pair FP32; sums in FP64.
 * value (host, FP64) and grad_h (host FP64 [2], or NULL); synchronises stream. */
int kde_lscv(const float *points, int64_t n, int32_t kernel_id, double hx, double hy, const kde_grid *g,
             double *value, double *grad_h, void *stream);

/* The paper's own binned visualisation (Sec. III-C and IV-B): a count matrix
 * of the points, optionally with the gaps between consecutive points of one
 * trajectory filled, then the convolution of Eq. (7) with a table of Table I
 * kernel values.  It approximates the kde_eval map (each point moved to the
 * cell above it, taps truncated at the radii) at a cost independent of the
 * bandwidth's reach over points.
 *
 * kde_bin_counts: counts[j*nx + i] = number of points with ceil(X) = i and
 * ceil(Y) = j (Eq. (5)-(6) with 0-based cells; points outside the grid are
 * dropped), plus, when labels is not NULL, the cells of Eq. (12)-(13) between
 * consecutive points p, p+1 with labels[p] == labels[p+1] whose cells are both
 * in the grid and more than one cell apart: c = 1 .. cmax-1,
 * cmax = max(|di|, |dj|), at the 1-based coordinate rounded half up.
 *   points  device FP32 [n][2] grid units (as kde_eval); n >= 0
 *   labels  device int32 [n] trajectory labels, or NULL (no gap filling)
 *   counts  device uint32 [ny][nx], overwritten
 *   total   device uint64 [1] receiving the number of counted cells, or NULL
 * Integer atomics: the result does not depend on thread order.  Asynchronous. */
int kde_bin_counts(const float *points, int64_t n, const int32_t *labels, const kde_grid *g, uint32_t *counts,
                   uint64_t *total, void *stream);

/* Eq. (7): out[j*nx + i] = scale * sum_{t=-b..b} sum_{s=-a..a} k(s/Hx) k(t/Hy)
 * counts[(j-t)*nx + (i-s)], cells outside the grid counting zero, Hx = hx/dx,
 * Hy = hy/dy, compact kernels 0 for |s| > Hx.  scale = 1/(N hx hy) with
 * N = *total (device uint64, the number of counted cells), or 1 with
 * KDE_RAW_SUM (total may then be NULL); N = 0 gives a zero map.  a, b in
 * [0, 128] (the paper's odd table size is 2a + 1).  FP32 taps and sums, a row
 * pass then a column pass.  Asynchronous. */
int kde_conv_counts(const uint32_t *counts, const uint64_t *total, const kde_grid *g, int32_t kernel_id, double hx,
                    double hy, int32_t a, int32_t b, float *out, uint32_t flags, void *stream);

/* kde_bin_counts then kde_conv_counts, the counts kept in library workspace. */
int kde_eval_binned(const float *points, int64_t n, const int32_t *labels, int32_t kernel_id, double hx, double hy,
                    int32_t a, int32_t b, const kde_grid *g, float *out, uint32_t flags, void *stream);

/* Douglas-Peucker compression of many trajectories at once (Sec. III-B; the
 * GPU framework of Sec. IV-A: every chord of every track handled in the same
 * level-synchronous pass).  Each track keeps its end points; within a chord
 * between kept points, the interior point farthest from the chord's line
 * (Eq. (9)) is kept when that distance is larger than eps, splitting the chord;
 * until no chord splits.  The farthest point is the lowest index among equal
 * distances; a chord with coinciding end points uses the distance to that
 * point; the test is cross^2 > eps^2 |chord|^2 in FP64 (no square root, no
 * fused multiply-add), so the mask is exact and order-independent.
 *   xy           device FP64 [n][2], planar coordinates (e.g. Mercator metres), finite
 *   track_start  device int64 [n_tracks + 1]: track t is [track_start[t], track_start[t+1]),
 *                rising from 0 to n (else KDE_EINVAL)
 *   eps          finite, >= 0, in the units of xy
 *   keep         device uint8 [n]: 1 for kept points
 *   out_xy       device FP64 [n][2] receiving the kept points in order, or NULL
 *   out_lengths  device int64 [n_tracks] receiving kept points per track, or NULL
 *   out_start    device int64 [n_tracks + 1] receiving the offsets of the compressed
 *                tracks in out_xy (0, ..., n_kept), or NULL
 *   n_kept       host, number of kept points, or NULL
 * Synchronises `stream` (once per few levels of the recursion and at the end). */
int kde_dp_compress(const double *xy, int64_t n, const int64_t *track_start, int64_t n_tracks, double eps,
                    uint8_t *keep, double *out_xy, int64_t *out_lengths, int64_t *out_start, int64_t *n_kept,
                    void *stream);

/* Compression quality of a track set against its compressed version
 * (Sec. V-B), over M tracks given by offsets: original track m is
 * xy_o[start_o[m] .. start_o[m+1]), its compressed version xy_c[start_c[m] ..
 * start_c[m+1]) (e.g. out_xy and out_start of kde_dp_compress; any series
 * works, a subsequence is not required).
 *   per track   len_o[m] = |T_m|, len_c[m] = |T'_m| (sum of Euclidean distances
 *               between consecutive points); dtw[m] = DTW(T_m, T'_m) of
 *               Eq. (16)-(18): sqrt of the last entry of the accumulated cost
 *               matrix D[i][j] = d(P_i, P'_j) + min(D[i-1][j-1], D[i-1][j],
 *               D[i][j-1]), d the squared Euclidean distance.  Two empty
 *               series are at distance 0, an empty and a non-empty one at +inf.
 *   totals      N_o, N_c, CR = (1 - N_c/N_o) * 100 (Eq. (14)), the summed
 *               lengths, RLL = (sum |T| - sum |T'|) / sum |T| (Eq. (15), a
 *               fraction), mu and delta = the mean and population standard
 *               deviation of the M DTW distances (Eq. (19)-(20)).  NaN where a
 *               denominator is 0.
 * FP64 throughout.  Each D entry is exact to the plain row-by-row recurrence
 * (no fused multiply-add); lengths and totals are fixed-order tree sums, so
 * results are bitwise reproducible.
 *   xy_o, xy_c        device FP64 [n][2] planar points (e.g. Mercator metres)
 *   start_o, start_c  device int64 [n_tracks + 1], rising from 0 to n_o (n_c);
 *                     tracks under 2^30 points (else KDE_EINVAL)
 *   len_o, len_c, dtw device FP64 [n_tracks] each, or NULL (not returned)
 *   out               host, the totals, or NULL
 * The offsets are checked on the device before any point is read; the call
 * synchronises `stream` once, at the end (KDE_EINVAL for bad offsets, with the
 * per-track outputs then unwritten). */
typedef struct kde_track_metrics {
    int64_t n_original, n_compressed;
    double cr_percent;
    double length_original, length_compressed;
    double rll;
    double dtw_mean, dtw_std;
} kde_track_metrics;

int kde_compression_metrics(const double *xy_o, int64_t n_o, const int64_t *start_o, const double *xy_c, int64_t n_c,
                            const int64_t *start_c, int64_t n_tracks, double *len_o, double *len_c, double *dtw,
                            kde_track_metrics *out, void *stream);

/* Tile-shape autotuner (FP32 direct path, kde_eval and kde_eval_batched).
 * The direct kernels exist for register blocks of 2 x 2, 4 x 4 and 8 x 8 pixels
 * per thread (pixel tiles of 32, 64 and 128 nodes per side).  The first call in
 * a shape bucket (single maps: kernel class, bandwidth in pixels, point count
 * and pixel count in log2 buckets; batches: every map's kernel class, point
 * count and grid) times the candidates on the caller's own data and stream
 * (each candidate computes the whole map or batch, so outputs stay valid) and
 * caches the fastest per device architecture; later calls reuse it.  No tuning
 * runs while `stream` is being captured (the cached or default shape is used).
 * Untuned defaults: 8 x 8 for the Gaussian, 2 x 2 for compact single maps,
 * 4 x 4 for compact maps in a batch.  Results of different shapes agree to
 * FP32 rounding (the split count over points follows the tile count).
 * Environment, read at first use: KDE_AUTOTUNE=0 disables tuning, KDE_TILE=2|4|8
 * forces a shape, KDE_AUTOTUNE_CACHE=<path> loads that JSON cache and rewrites
 * it after each new entry.  The cache is process-wide and thread-safe. */

/* on = 1 (default) tunes on a cache miss; on = 0 uses cached or default
 * shapes only.  KDE_EINVAL for other values. */
int kde_autotune_enable(int32_t on);
/* rc = 2, 4 or 8 makes every FP32 direct map use that register block; 0 ends
 * the forcing.  KDE_EINVAL for other values. */
int kde_autotune_force(int32_t rc);
/* Merges the entries of a JSON cache file ({"format": "kde-autotune-1",
 * "entries": {key: {"choice": ..., "ms": {...}}}}).  A file that cannot be read,
 * does not parse or holds an invalid choice is rejected as a whole with
 * KDE_EINVAL, leaving the cache unchanged. */
int kde_autotune_load(const char *path);
/* Writes the cache as JSON to path (via a temporary file and a rename). */
int kde_autotune_save(const char *path);
/* Copies the cache's JSON text (NUL-terminated) into buf and sets *needed to
 * its size including the NUL; with buf NULL only *needed is set.  KDE_EINVAL
 * if cap is too small (nothing written). */
int kde_autotune_dump(char *buf, size_t cap, size_t *needed);
/* Empties the in-memory cache. */
int kde_autotune_clear(void);

/* Measurement hook.  The next kde_eval, kde_eval_noalloc, kde_backward,
 * kde_conv_counts, kde_eval_binned or kde_compression_metrics call made by this
 * thread records start_event on its stream right before it launches its main
 * kernel (the separable contraction, the FP32 direct evaluation, the
 * support-binned gather, the VJP kernel, the two convolution passes, or the
 * per-track length and DTW pass) and stop_event right after, so that the
 * elapsed time between the two events is that work alone, without the point
 * padding, split reduction, support-binning or counting passes.  Both are
 * hipEvent_t handles owned by the caller, created on the device of that call
 * with timing enabled; the request is consumed by that call (also by one that
 * fails or has n = 0, which records nothing).  NULL, NULL cancels a pending
 * request, and so does kde_eval_batched.  Returns KDE_OK, or KDE_EINVAL if
 * exactly one event is NULL. */
int kde_time_next_main_kernel(void *start_event, void *stop_event);

/* Thread-local text of the last failure on this thread ("" if none). */
const char *kde_last_error(void);

/* Frees every cached workspace on every device.  No call may be in flight. */
void kde_shutdown(void);

#ifdef __cplusplus
}
#endif

#endif /* KDE_H */
