// Compression quality of a track set against its compressed version (Sec. V-B)
// on gfx950: per track the lengths |T| and |T'| (RLL, Eq. (15)) and the DTW
// distance of Eq. (16)-(18); over the set CR (Eq. (14)), RLL, and the mean and
// population standard deviation of the DTW distances (Eq. (19)-(20)).
//
// One wave per track.  DTW fills the accumulated cost matrix as an
// anti-diagonal wavefront inside the wave: one series is "owned" (lane l holds
// R consecutive entries of it, a strip of 64 R), the other is swept; at step s
// lane l updates its R cells of swept column j = s - l, so every cell's left
// neighbours are in the lane's own registers and its upper neighbours come
// from lane l - 1's last row of the step before (one DPP lane shift per
// step).  Which series is owned, and R (1 to 8), are chosen per track to
// minimise lane-steps.  Swept points are staged 64 at a time into an LDS ring
// of two chunks, each chunk loaded a whole chunk ahead.  Series longer than
// one strip run several strips; the last row of each is handed to the next
// through a per-track global buffer (two of them, by strip parity).
//
// The recurrence is symmetric under transposing the matrix (d is symmetric and
// min is exact), so owning either series gives the same cells.  Squared
// distances and sums are FP64 without fused multiply-add, so every D entry, and
// the DTW distance before its square root, is bit-identical to a plain row-by-row
// fill.  Per-track lengths are wave tree sums; set totals a fixed-order block
// reduction: both deterministic.
#include "kde_internal.h"

#include <cmath>

namespace kde {

namespace {

constexpr int kWave = 64;
constexpr int kReduceThreads = 1024;
constexpr int kMaxBlock = 8;     // register block (owned entries per lane) at most
constexpr double kStepCost = 2.0; // per-step shifts, loads and bookkeeping, in cells (measured)

__device__ __forceinline__ double kInfD() { return __builtin_huge_val(); }

// Butterfly sum over the wave; every lane ends with the same bits (each
// pairwise add is commutative).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

__device__ __forceinline__ double sq_dist(double ax, double ay, double2 b) {
#pragma clang fp contract(off)
    const double dx = ax - b.x, dy = ay - b.y;
    return dx * dx + dy * dy;
}

// Sum of |P_i P_{i+1}|: lane l takes i = l, l + 64, ... in order, then a wave sum.
__device__ double polyline_length(const double2 *__restrict__ p, int n, int lane) {
#pragma clang fp contract(off)
    double s = 0.0;
    for (int i = lane; i + 1 < n; i += kWave) {
        const double2 a = p[i], b = p[i + 1];
        const double dx = b.x - a.x, dy = b.y - a.y;
        s += sqrt(dx * dx + dy * dy);
    }
    return wave_sum(s);
}

// min of two FP64 values known to be non-NaN.  (The compiler's fmin quiets
// signalling NaNs first, one extra v_max_f64 per operand it cannot prove
// canonical; accumulated costs are sums of squares or +inf.)
__device__ __forceinline__ double dmin(double a, double b) {
    double r;
    asm("v_min_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

// Lane l receives lane l - 1's v, lane 0 receives fill (a DPP whole-wave shift
// right by one lane: two 32-bit moves, no LDS traffic).
__device__ __forceinline__ double shift_up_or(double v, double fill) {
    const int lo = __builtin_amdgcn_update_dpp(__double2loint(fill), __double2loint(v), 0x138, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(__double2hiint(fill), __double2hiint(v), 0x138, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}

// D[na-1][nb-1] of the accumulated cost matrix between A (owned, na entries)
// and B (swept, nb entries), both non-empty.  bound: 2 * nb doubles.  Returns
// the value on every lane.
//
// No lane is masked inside the sweep: before its first column a lane reads the
// swept point (+inf, +inf) (the LDS slot of chunk -1), so every cell it
// computes is +inf, the border value; past its last column it computes cells no
// valid cell depends on.  The sweep of the last strip ends on the step where
// the lane holding row na - 1 finishes column nb - 1, so that lane's register
// then holds the result.
template <int R>
__device__ double dtw_wave(const double2 *__restrict__ A, int na, const double2 *__restrict__ B, int nb,
                           double *__restrict__ bound, double2 *ring_b, double *ring_t, int lane) {
#pragma clang fp contract(off)
    constexpr int kStrip = kWave * R;
    const double inf = kInfD();
    const int strips = (na + kStrip - 1) / kStrip;
    double result = 0.0;
    for (int k = 0; k < strips; ++k) {
        const int base = k * kStrip;
        double ax[R], ay[R], left[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int idx = base + lane * R + r;
            const double2 a = idx < na ? A[idx] : make_double2(0.0, 0.0);  // rows past na feed no valid cell
            ax[r] = a.x;
            ay[r] = a.y;
            left[r] = inf;  // column -1
        }
        const bool last = k + 1 == strips;
        const double *tin = k > 0 ? bound + ((k - 1) & 1) * (size_t)nb : nullptr;  // row base - 1
        double *tout = last ? nullptr : bound + (k & 1) * (size_t)nb;             // row base + kStrip - 1
        const int lanes_used = last ? (na - base + R - 1) / R : kWave;
        const int steps = nb + lanes_used - 1;
        double bottom = inf;                                // last row of the previous step (inf before the start)
        double diag = (k == 0 && lane == 0) ? 0.0 : inf;   // D[row0 - 1][j - 1]; D[-1][-1] = 0
        __syncthreads();  // the previous strip no longer reads the ring
        ring_b[kWave + lane] = make_double2(inf, inf);  // chunk -1: columns before the first
        // chunk c of the swept series (and of the row above the strip), one a lane
        double2 nxt_b = lane < nb ? B[lane] : make_double2(0.0, 0.0);
        double nxt_t = (tin != nullptr && lane < nb) ? tin[lane] : inf;
        for (int c = 0; c * kWave < steps; ++c) {  // chunk c: steps 64 c .. 64 c + 63
            __syncthreads();  // the slot's previous chunk (c - 2) is no longer read
            ring_b[(c & 1) * kWave + lane] = nxt_b;
            ring_t[(c & 1) * kWave + lane] = nxt_t;
            __syncthreads();
            const int jn = (c + 1) * kWave + lane;
            nxt_b = jn < nb ? B[jn] : make_double2(0.0, 0.0);
            nxt_t = (tin != nullptr && jn < nb) ? tin[jn] : inf;
            const int s_end = min(steps, (c + 1) * kWave);
            for (int s = c * kWave; s < s_end; ++s) {
                // D[row0 - 1][j]: lane l - 1's last row of the previous step; for
                // lane 0 (column s) the row above the strip
                const double up_in = shift_up_or(bottom, ring_t[s & (2 * kWave - 1)]);
                const int j = s - lane;
                const double2 b = ring_b[j & (2 * kWave - 1)];
                // cell r takes min(D[r-1][j-1], D[r][j-1]) (old registers, off the
                // dependency chain), then min with D[r-1][j] and the distance;
                // each new value overwrites its row's register once the next
                // row's first min has read the old one.
                double t = dmin(diag, left[0]), up = up_in;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const double t_next = r + 1 < R ? dmin(left[r], left[r + 1]) : 0.0;
                    left[r] = sq_dist(ax[r], ay[r], b) + dmin(t, up);
                    up = left[r];
                    t = t_next;
                }
                bottom = up;
                if (tout != nullptr && lane == kWave - 1 && j >= 0) tout[j] = bottom;  // j < nb: s < nb + 63
                diag = up_in;
            }
        }
        if (last) {
            const int owner_r = (na - 1 - base) - (lanes_used - 1) * R;
#pragma unroll
            for (int r = 0; r < R; ++r)
                if (r == owner_r) result = left[r];
        }
        __syncthreads();  // the strip's last row is visible to the next strip's loads
    }
    return __shfl(result, (na - 1 - (strips - 1) * kStrip) / R);
}

// Lane-steps of a sweep owning na entries with register block R, swept over
// nb; each step costs R cells plus about kStepCost cells' worth of shifts,
// loads and bookkeeping.
__device__ __forceinline__ double sweep_cost(int na, int nb, int R) {
    const int strip = kWave * R, strips = (na + strip - 1) / strip;
    const int last_lanes = (na - (strips - 1) * strip + R - 1) / R;
    const double steps = (double)(strips - 1) * (nb + kWave - 1) + (nb + last_lanes - 1);
    return steps * (R + kStepCost);
}

// Cheapest orientation and register block for a pair of series of lengths
// no and nc: returns R, and own_c = whether the compressed series is owned.
__device__ __forceinline__ int pick_block(int no, int nc, bool *own_c) {
    int best = 0;
    double best_cost = 0.0;
    for (int o = 0; o < 2; ++o) {
        const int na = o ? nc : no, nb = o ? no : nc;
        for (int R = 1; R <= kMaxBlock; ++R) {
            const double cost = sweep_cost(na, nb, R);
            if (best == 0 || cost < best_cost) {
                best = R;
                best_cost = cost;
                *own_c = o != 0;
            }
        }
    }
    return best;
}

__global__ __launch_bounds__(kWave) void track_metrics_kernel(const double2 *__restrict__ xo,
                                                              const int64_t *__restrict__ so,
                                                              const double2 *__restrict__ xc,
                                                              const int64_t *__restrict__ sc,
                                                              double *__restrict__ bound, double *__restrict__ len_o,
                                                              double *__restrict__ len_c, double *__restrict__ dtw,
                                                              const unsigned *__restrict__ bad) {
    __shared__ double2 ring_b[2 * kWave];
    __shared__ double ring_t[2 * kWave];
    if (*bad != 0u) return;  // offsets rejected by the check: touch no point
    const int64_t m = blockIdx.x;
    const int lane = threadIdx.x;
    const int64_t o0 = so[m], c0 = sc[m];
    const int no = (int)(so[m + 1] - o0), nc = (int)(sc[m + 1] - c0);
    const double2 *O = xo + o0, *C = xc + c0;
    const double lo = polyline_length(O, no, lane);
    const double lc = polyline_length(C, nc, lane);
    double d;
    if (no == 0 || nc == 0) {
        d = (no == 0 && nc == 0) ? 0.0 : kInfD();  // no warping path joins an empty series to a non-empty one
    } else {
        bool own_c = false;
        const int R = pick_block(no, nc, &own_c);
        const double2 *A = own_c ? C : O, *B = own_c ? O : C;
        const int na = own_c ? nc : no, nb = own_c ? no : nc;
        double *bd = bound + 2 * (o0 + c0);  // 2 (no + nc) >= 2 nb doubles of this track
        double D;
        switch (R) {
        case 1: D = dtw_wave<1>(A, na, B, nb, bd, ring_b, ring_t, lane); break;
        case 2: D = dtw_wave<2>(A, na, B, nb, bd, ring_b, ring_t, lane); break;
        case 3: D = dtw_wave<3>(A, na, B, nb, bd, ring_b, ring_t, lane); break;
        case 4: D = dtw_wave<4>(A, na, B, nb, bd, ring_b, ring_t, lane); break;
        case 5: D = dtw_wave<5>(A, na, B, nb, bd, ring_b, ring_t, lane); break;
        case 6: D = dtw_wave<6>(A, na, B, nb, bd, ring_b, ring_t, lane); break;
        case 7: D = dtw_wave<7>(A, na, B, nb, bd, ring_b, ring_t, lane); break;
        default: D = dtw_wave<8>(A, na, B, nb, bd, ring_b, ring_t, lane); break;
        }
        d = sqrt(D);
    }
    if (lane == 0) {
        len_o[m] = lo;
        len_c[m] = lc;
        dtw[m] = d;
    }
}

// Fixed-order block sum: strided per-thread partials, wave sums, then the 16
// wave results added in wave order.  Every thread returns the total.
__device__ double block_sum(double v, double *red) {
    v = wave_sum(v);
    const int w = threadIdx.x / kWave;
    __syncthreads();  // red free from any previous use
    if ((threadIdx.x & (kWave - 1)) == 0) red[w] = v;
    __syncthreads();
    double t = 0.0;
    for (int i = 0; i < kReduceThreads / kWave; ++i) t += red[i];
    return t;
}

__global__ __launch_bounds__(kReduceThreads) void metrics_reduce_kernel(const double *__restrict__ len_o,
                                                                        const double *__restrict__ len_c,
                                                                        const double *__restrict__ dtw, int64_t m,
                                                                        const int64_t *__restrict__ so,
                                                                        const int64_t *__restrict__ sc,
                                                                        const unsigned *__restrict__ bad,
                                                                        MetricsTotals *__restrict__ out) {
#pragma clang fp contract(off)
    __shared__ double red[kReduceThreads / kWave];
    if (*bad != 0u) return;
    double a = 0.0, b = 0.0, c = 0.0;
    for (int64_t i = threadIdx.x; i < m; i += kReduceThreads) {
        a += len_o[i];
        b += len_c[i];
        c += dtw[i];
    }
    const double lo = block_sum(a, red), lc = block_sum(b, red), sd = block_sum(c, red);
    const double nan = __builtin_nan("");
    const double mu = m > 0 ? sd / (double)m : nan;
    double q = 0.0;
    for (int64_t i = threadIdx.x; i < m; i += kReduceThreads) {
        const double e = dtw[i] - mu;
        q += e * e;
    }
    const double sq = block_sum(q, red);
    if (threadIdx.x == 0) {
        const int64_t no = so[m], nc = sc[m];
        out->n_original = no;
        out->n_compressed = nc;
        out->cr_percent = no > 0 ? (1.0 - (double)nc / (double)no) * 100.0 : nan;
        out->length_original = lo;
        out->length_compressed = lc;
        out->rll = lo != 0.0 ? (lo - lc) / lo : nan;
        out->dtw_mean = mu;
        out->dtw_std = m > 0 ? sqrt(sq / (double)m) : nan;
    }
}

// bad = 1 unless both offset arrays rise from 0 to their point counts.
__global__ __launch_bounds__(256) void metrics_check_kernel(const int64_t *__restrict__ so, int64_t n_o,
                                                            const int64_t *__restrict__ sc, int64_t n_c, int64_t m,
                                                            unsigned *__restrict__ bad) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t > m) return;
    bool ok = true;
    if (t == 0) ok = so[0] == 0 && sc[0] == 0;
    if (t == m) ok = ok && so[m] == n_o && sc[m] == n_c;
    if (t < m) ok = ok && so[t] <= so[t + 1] && sc[t] <= sc[t + 1] && so[t + 1] - so[t] < kMaxTrackPoints &&
                    sc[t + 1] - sc[t] < kMaxTrackPoints;
    if (!ok) atomicOr(bad, 1u);
}

__global__ void zero_flag_kernel(unsigned *flag) {
    if (threadIdx.x == 0) *flag = 0u;
}

size_t al256(size_t x) { return (x + 255) / 256 * 256; }

}  // namespace

// Totals and the offsets check's flag, next to each other so that one copy
// brings both back.
struct MetricsResult {
    MetricsTotals totals;
    unsigned bad;
    unsigned pad_;
};

size_t metrics_workspace_bytes(int64_t n_o, int64_t n_c, int64_t n_tracks, bool per_track_given) {
    size_t b = al256(sizeof(MetricsResult)) + al256((size_t)2 * (n_o + n_c) * sizeof(double));
    if (!per_track_given) b += 3 * al256((size_t)n_tracks * sizeof(double));
    return b;
}

hipError_t run_metrics(const MetricsArgs &a, void *ws, hipStream_t s, MetricsTotals *host_out) {
    char *w = static_cast<char *>(ws);
    MetricsResult *res = reinterpret_cast<MetricsResult *>(w);
    w += al256(sizeof(MetricsResult));
    double *bound = reinterpret_cast<double *>(w);
    w += al256((size_t)2 * (a.n_o + a.n_c) * sizeof(double));
    double *lo = a.len_o, *lc = a.len_c, *dt = a.dtw;
    const size_t per = al256((size_t)a.n_tracks * sizeof(double));
    if (lo == nullptr) { lo = reinterpret_cast<double *>(w); w += per; }
    if (lc == nullptr) { lc = reinterpret_cast<double *>(w); w += per; }
    if (dt == nullptr) { dt = reinterpret_cast<double *>(w); w += per; }
    unsigned *bad = &res->bad;
    // The check runs first on the stream; the kernels after it read its flag
    // and do nothing when it is set, so bad offsets never index the points.
    hipLaunchKernelGGL(zero_flag_kernel, dim3(1), dim3(64), 0, s, bad);
    hipLaunchKernelGGL(metrics_check_kernel, dim3((unsigned)((a.n_tracks + 1 + 255) / 256)), dim3(256), 0, s, a.so,
                       a.n_o, a.sc, a.n_c, a.n_tracks, bad);
    if (a.n_tracks > 0) {
        main_kernel_begin(s);
        hipLaunchKernelGGL(track_metrics_kernel, dim3((unsigned)a.n_tracks), dim3(kWave), 0, s, a.xo, a.so, a.xc,
                           a.sc, bound, lo, lc, dt, static_cast<const unsigned *>(bad));
        main_kernel_end(s);
    }
    hipLaunchKernelGGL(metrics_reduce_kernel, dim3(1), dim3(kReduceThreads), 0, s, static_cast<const double *>(lo),
                       static_cast<const double *>(lc), static_cast<const double *>(dt), a.n_tracks, a.so, a.sc,
                       static_cast<const unsigned *>(bad), &res->totals);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    MetricsResult host;
    e = hipMemcpyAsync(&host, res, sizeof host, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    if (host.bad) return hipErrorInvalidValue;
    if (host_out != nullptr) *host_out = host.totals;
    return hipSuccess;
}

}  // namespace kde
