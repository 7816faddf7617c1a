// Douglas-Peucker compression of many trajectories at once (Sec. III-B, its
// GPU form in Sec. IV-A), level-synchronous: every chord of every track is
// processed in the same pass, as the paper's label sets do.
//
// State per point i: the kept points lo[i] < i < hi[i] that enclose it (its
// chord), and whether it is still undecided (active).  One level:
//   1. score: |cross| of Eq. (9)'s numerator (squared distance to P_s for a
//      chord of zero length), integer atomic max of its bits into the chord's
//      slot (slots are indexed by the chord's first point, unique among the
//      chords of one level, and double-buffered by level parity);
//   2. argmax: points whose score equals the slot's maximum take an integer
//      atomic min of their index (the lowest index wins ties);
//   3. decide: the chord's argmax keeps itself when cross^2 > eps^2 |chord|^2
//      (or dist^2 > eps^2), marking the chord split or final, and resets the
//      next level's slots of both halves;
//   4. update: points of final chords are dropped, the others move to the half
//      chord on their side of the new kept point, and are scored right away for
//      the next level (the same kernel: a point's update needs only its own
//      chord's decision).
// Scores are FP64 with no fused multiply-add (the decision is taken exactly as
// the reference does), and all cross-thread combination is integer atomics:
// the keep mask does not depend on thread order.
//
// Tracks are independent, so each track of at most kTrackMax points runs all
// its levels inside one workgroup (dp_track_kernel): the track's points in
// LDS, the chord slots as LDS atomics, the four steps separated by workgroup
// barriers, until a level splits no chord.  Only longer tracks take the
// level-synchronous kernels below, three launches per level over the points of
// those tracks, the host checking after each group of levels whether any chord
// still split (the paper synchronises with the host every level).
#include "kde_internal.h"

#include <algorithm>
#include <climits>

namespace kde {

namespace {

constexpr unsigned long long kNoIndex = ULLONG_MAX;
constexpr int kLevelsPerCheck = 8;

__device__ __forceinline__ double dp_score(const double2 *__restrict__ xy, int64_t s, int64_t e, int64_t i,
                                           bool &zero) {
#pragma clang fp contract(off)
    const double2 ps = xy[s], pe = xy[e], pi = xy[i];
    const double cx = pe.x - ps.x, cy = pe.y - ps.y;
    const double px = pi.x - ps.x, py = pi.y - ps.y;
    const double c2 = cx * cx + cy * cy;
    zero = c2 == 0.0;
    if (zero) return px * px + py * py;
    const double a = px * cy, b = py * cx;
    return fabs(a - b);
}

__device__ __forceinline__ bool dp_split(const double2 *__restrict__ xy, int64_t s, int64_t e, double score,
                                         bool zero, double eps2) {
#pragma clang fp contract(off)
    if (zero) return score > eps2;
    const double2 ps = xy[s], pe = xy[e];
    const double cx = pe.x - ps.x, cy = pe.y - ps.y;
    const double c2 = cx * cx + cy * cy;
    return score * score > eps2 * c2;
}

constexpr int kTrackThreads = 256;
constexpr int kTrackMax = 1024;                       // longest track one workgroup takes
constexpr int kTrackPer = kTrackMax / kTrackThreads;  // points per thread

// counters[0] = 1 unless start[0] = 0, start[n_tracks] = n and the offsets
// never decrease; counters[1] = number of tracks longer than kTrackMax;
// counters[2] = the longest of the other tracks.
__global__ __launch_bounds__(256) void dp_check_kernel(const int64_t *__restrict__ start, int64_t n_tracks, int64_t n,
                                                       unsigned *__restrict__ counters) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t > n_tracks) return;
    bool ok = true;
    if (t == 0) ok = start[0] == 0;
    if (t == n_tracks) ok = ok && start[n_tracks] == n;
    if (t < n_tracks) {
        ok = ok && start[t] <= start[t + 1];
        const int64_t len = start[t + 1] - start[t];
        if (len > kTrackMax) atomicAdd(counters + 1, 1u);
        else if (len > 0) atomicMax(counters + 2, (unsigned)len);
    }
    if (!ok) atomicOr(counters, 1u);
}

// One track of at most kTrackMax points per workgroup, every level in LDS.
// Point i of the track (local index) belongs to thread i % 256, which keeps its
// chord (lo, hi), score and activity in registers; the slots of level L (chord
// maximum and argmax, indexed by the chord's first point) are buffer L % 2, as
// in the level-synchronous form.  Per level: [scores into the slots] barrier,
// argmax, barrier, decide, barrier, stop if no chord split, else update and
// score the next level.  Longer tracks are left to the level-synchronous path.
// The LDS arrays are sized at launch for `cap` points (the call's longest short
// track, dp_track_lds_bytes), so that short tracks leave room for more
// workgroups per CU.
constexpr size_t dp_track_lds_bytes(int cap) { return (size_t)41 * cap + 16; }

__global__ __launch_bounds__(kTrackThreads) void dp_track_kernel(const double2 *__restrict__ xy,
                                                                 const int64_t *__restrict__ start, double eps2,
                                                                 int cap, uint8_t *__restrict__ keep) {
    extern __shared__ __align__(16) unsigned char dp_lds[];
    unsigned long long *smax0 = reinterpret_cast<unsigned long long *>(dp_lds);  // [2][cap]
    double2 *pxy = reinterpret_cast<double2 *>(dp_lds + 16 * (size_t)cap);      // [cap]
    unsigned *sarg0 = reinterpret_cast<unsigned *>(dp_lds + 32 * (size_t)cap);   // [2][cap]
    uint8_t *sdec = dp_lds + 40 * (size_t)cap;                                    // [cap]
    int *sflag = reinterpret_cast<int *>(dp_lds + ((41 * (size_t)cap + 3) & ~(size_t)3));  // [2]
    auto SMAX = [&](int b, int i) -> unsigned long long & { return smax0[b * cap + i]; };
    auto SARG = [&](int b, int i) -> unsigned & { return sarg0[b * cap + i]; };
    const int64_t s0 = start[blockIdx.x], len64 = start[blockIdx.x + 1] - s0;
    if (len64 <= 0 || len64 > cap) return;  // uniform over the workgroup; longer tracks: level loop
    const int len = (int)len64, tid = threadIdx.x;
    for (int i = tid; i < len; i += kTrackThreads) {
        pxy[i] = xy[s0 + i];
        keep[s0 + i] = (i == 0 || i == len - 1) ? 1 : 0;
    }
    if (len <= 2) return;
    int lo[kTrackPer], hi[kTrackPer];
    double sc[kTrackPer];
    bool act[kTrackPer];
#pragma unroll
    for (int q = 0; q < kTrackPer; ++q) {
        const int i = tid + q * kTrackThreads;
        act[q] = i > 0 && i < len - 1;
        lo[q] = 0;
        hi[q] = len - 1;
    }
    if (tid == 0) {
        SMAX(0, 0) = 0ull;
        SARG(0, 0) = UINT_MAX;
        sflag[0] = sflag[1] = 0;
    }
    __syncthreads();
    auto score_into = [&](int buf) {
#pragma unroll
        for (int q = 0; q < kTrackPer; ++q) {
            if (!act[q]) continue;
            bool zero;
            sc[q] = dp_score(pxy, lo[q], hi[q], tid + q * kTrackThreads, zero);
            atomicMax(&SMAX(buf, lo[q]), (unsigned long long)__double_as_longlong(sc[q]));
        }
    };
    score_into(0);
    for (int level = 0;; ++level) {
        const int cur = level & 1, nxt = cur ^ 1;
        __syncthreads();  // this level's chord maxima are complete
        if (tid == 0) sflag[nxt] = 0;  // read by every thread before the barrier above
#pragma unroll
        for (int q = 0; q < kTrackPer; ++q)
            if (act[q] && (unsigned long long)__double_as_longlong(sc[q]) == SMAX(cur, lo[q]))
                atomicMin(&SARG(cur, lo[q]), (unsigned)(tid + q * kTrackThreads));
        __syncthreads();  // argmax complete
#pragma unroll
        for (int q = 0; q < kTrackPer; ++q) {
            const int i = tid + q * kTrackThreads;
            if (!act[q] || SARG(cur, lo[q]) != (unsigned)i) continue;
            bool zero;
            (void)dp_score(pxy, lo[q], hi[q], i, zero);  // the zero-chord case, decided as the score was
            const bool split = dp_split(pxy, lo[q], hi[q], sc[q], zero, eps2);
            sdec[lo[q]] = split ? 1 : 2;
            if (split) {
                keep[s0 + i] = 1;
                SMAX(nxt, lo[q]) = 0ull;
                SARG(nxt, lo[q]) = UINT_MAX;
                SMAX(nxt, i) = 0ull;
                SARG(nxt, i) = UINT_MAX;
                sflag[cur] = 1;
            }
        }
        __syncthreads();  // decisions and the next level's slot resets complete
        if (sflag[cur] == 0) break;  // no chord split: every chord is final
#pragma unroll
        for (int q = 0; q < kTrackPer; ++q) {
            if (!act[q]) continue;
            const int i = tid + q * kTrackThreads;
            if (sdec[lo[q]] == 2) {
                act[q] = false;  // within eps of its final chord: dropped
                continue;
            }
            const int k = (int)SARG(cur, lo[q]);
            if (k == i) act[q] = false;  // kept
            else if (i < k) hi[q] = k;
            else lo[q] = k;
        }
        score_into(nxt);
    }
}

// Track of point i (binary search in the offsets), its end points kept; the
// slots of the first chords (at the track starts) are reset for level 0.
// Points of tracks of at most kTrackMax points (done by dp_track_kernel) are
// left inactive and their keep entries untouched.
__global__ __launch_bounds__(256) void dp_init_kernel(const int64_t *__restrict__ start, int64_t n_tracks, int64_t n,
                                                      int *__restrict__ lo, int *__restrict__ hi,
                                                      uint8_t *__restrict__ keep, uint8_t *__restrict__ active,
                                                      unsigned long long *__restrict__ segmax,
                                                      unsigned long long *__restrict__ segarg) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int64_t a = 0, b = n_tracks;  // find t with start[t] <= i < start[t + 1]
    while (b - a > 1) {
        const int64_t m = (a + b) / 2;
        if (start[m] <= i) a = m;
        else b = m;
    }
    const int64_t s = start[a], e = start[a + 1] - 1;
    if (e - s + 1 <= kTrackMax) {
        active[i] = 0;
        return;
    }
    lo[i] = (int)s;
    hi[i] = (int)e;
    const bool end_point = i == s || i == e;
    keep[i] = end_point ? 1 : 0;
    active[i] = end_point ? 0 : 1;
    if (i == s) {
        segmax[i] = 0ull;
        segarg[i] = kNoIndex;
    }
}

// Slots of level L live in buffer L % 2: the kept point of a split chord resets
// the next level's slots of both halves while this level's are still read.
// Scores an active point against its chord (s, e) and folds the chord maxima
// of the wave into the chord slots.  Chords are index ranges, so the active
// lanes of a wave fall into a few runs of equal chord: a segmented max-scan
// over the wave (a lane takes the running max of lanes off = 1, 2, 4, ... below
// it while they hold its chord) leaves each run's maximum in its last lane,
// which alone issues the atomic.  Runs cut by inactive lanes (chord -1) give
// one atomic per piece; integer max is order-free, so the slot ends the same.
__device__ __forceinline__ void score_point(const double2 *__restrict__ xy, int64_t i, bool act, int s, int e,
                                            double *__restrict__ score, unsigned long long *__restrict__ segmax) {
    unsigned long long bits = 0ull;
    if (act) {
        bool zero;
        const double sc = dp_score(xy, s, e, i, zero);
        score[i] = sc;
        bits = (unsigned long long)__double_as_longlong(sc);  // non-negative doubles order like their bits
    } else {
        s = -1;
    }
    if (__ballot(act) == 0ull) return;
    const int lane = (int)(threadIdx.x & 63);
    unsigned long long m = bits;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const unsigned long long o = __shfl_up(m, off);
        const int so = __shfl_up(s, off);
        if (lane >= off && so == s && o > m) m = o;
    }
    const int s_next = __shfl_down(s, 1);
    if (act && (lane == 63 || s_next != s)) atomicMax(segmax + s, m);
}

// Level 0: every active point against its track's end-point chord.
__global__ __launch_bounds__(256) void dp_score_kernel(const double2 *__restrict__ xy, int64_t n,
                                                       const int *__restrict__ lo, const int *__restrict__ hi,
                                                       const uint8_t *__restrict__ active,
                                                       double *__restrict__ score,
                                                       unsigned long long *__restrict__ segmax) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool act = i < n && active[i];
    score_point(xy, i, act, act ? lo[i] : -1, act ? hi[i] : -1, score, segmax);
}

__global__ __launch_bounds__(256) void dp_argmax_kernel(int64_t n, const int *__restrict__ lo,
                                                        const uint8_t *__restrict__ active,
                                                        const double *__restrict__ score,
                                                        const unsigned long long *__restrict__ segmax,
                                                        unsigned long long *__restrict__ segarg) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || !active[i]) return;
    if ((unsigned long long)__double_as_longlong(score[i]) == segmax[lo[i]])
        atomicMin(segarg + lo[i], (unsigned long long)i);
}

// The chord's argmax decides: 1 = split at it (kept), 2 = final.
__global__ __launch_bounds__(256) void dp_decide_kernel(const double2 *__restrict__ xy, int64_t n, double eps2,
                                                        const int *__restrict__ lo, const int *__restrict__ hi,
                                                        const uint8_t *__restrict__ active,
                                                        const double *__restrict__ score,
                                                        const unsigned long long *__restrict__ segarg,
                                                        uint8_t *__restrict__ segdec, uint8_t *__restrict__ keep,
                                                        unsigned long long *__restrict__ next_max,
                                                        unsigned long long *__restrict__ next_arg,
                                                        unsigned *__restrict__ splits) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool split = false;
    if (i < n && active[i] && segarg[lo[i]] == (unsigned long long)i) {
        const int s = lo[i];
        bool zero;
        (void)dp_score(xy, s, hi[i], i, zero);  // the zero-chord case, decided as the score was
        split = dp_split(xy, s, hi[i], score[i], zero, eps2);
        segdec[s] = split ? 1 : 2;
        if (split) {
            keep[i] = 1;
            next_max[s] = 0ull;
            next_arg[s] = kNoIndex;
            next_max[i] = 0ull;
            next_arg[i] = kNoIndex;
        }
    }
    // Only "some chord split" is needed: one lane per wave that saw a split
    // sets the flag, and skips the store once it reads the flag already set
    // (many concurrent stores to one line would serialise in the cache).
    const uint64_t any = __ballot(split);
    if (any != 0ull && (int)(threadIdx.x & 63) == __ffsll((unsigned long long)any) - 1 &&
        __atomic_load_n(splits, __ATOMIC_RELAXED) == 0u)
        *splits = 1u;
}

// End of a level and start of the next, per point: a point of a final chord is
// dropped, the splitting point itself is kept (and leaves), every other point
// moves to the half chord on its side of it; then it is scored against that
// chord into the next level's slots.  (The update needs only the point's own
// chord's decision, so no level-wide barrier separates the two.)
__global__ __launch_bounds__(256) void dp_update_score_kernel(const double2 *__restrict__ xy, int64_t n,
                                                              int *__restrict__ lo, int *__restrict__ hi,
                                                              uint8_t *__restrict__ active,
                                                              const unsigned long long *__restrict__ segarg,
                                                              const uint8_t *__restrict__ segdec,
                                                              double *__restrict__ score,
                                                              unsigned long long *__restrict__ next_max) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool act = i < n && active[i];
    int l = -1, h = -1;
    if (act) {
        l = lo[i];
        h = hi[i];
        if (segdec[l] == 2) {
            act = false;  // within eps of its final chord: dropped
        } else {
            const int k = (int)segarg[l];
            if (k == i) {
                act = false;  // kept
            } else if (i < k) {
                h = k;
                hi[i] = k;
            } else {
                l = k;
                lo[i] = k;
            }
        }
        if (!act) active[i] = 0;
    }
    score_point(xy, i, act, l, h, score, next_max);
}

__global__ __launch_bounds__(256) void zero_u32_kernel(unsigned *p, int64_t count) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0u;
}

__global__ __launch_bounds__(256) void keep_to_u32_kernel(const uint8_t *__restrict__ keep, int64_t n,
                                                          unsigned *__restrict__ pos) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) pos[i] = keep[i];
}

// Compaction (pos = exclusive scan of keep) and kept points per track.
__global__ __launch_bounds__(256) void dp_compact_kernel(const double2 *__restrict__ xy, int64_t n,
                                                         const uint8_t *__restrict__ keep,
                                                         const unsigned *__restrict__ pos, double2 *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && keep[i]) out[pos[i]] = xy[i];
}

// Kept points per track and the compressed tracks' offsets (pos of each track's
// first point; the last offset is the total).
__global__ __launch_bounds__(256) void dp_lengths_kernel(const int64_t *__restrict__ start, int64_t n_tracks,
                                                         const unsigned *__restrict__ pos, unsigned total,
                                                         int64_t n, int64_t *__restrict__ lengths,
                                                         int64_t *__restrict__ out_start) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t > n_tracks) return;
    if (t == n_tracks) {
        if (out_start != nullptr) out_start[t] = total;
        return;
    }
    const int64_t a = start[t], b = start[t + 1];
    const unsigned pa = a < n ? pos[a] : total, pb = b < n ? pos[b] : total;
    if (lengths != nullptr) lengths[t] = (int64_t)pb - (int64_t)pa;
    if (out_start != nullptr) out_start[t] = pa;
}

struct DpLayout {
    size_t lo, hi, active, score, segmax, segarg, segdec, counters, pos, totals, total;
};

size_t al(size_t x) { return (x + 255) / 256 * 256; }

DpLayout dp_layout(int64_t n) {
    DpLayout L;
    size_t o = 0;
    L.lo = o; o += al((size_t)n * 4);
    L.hi = o; o += al((size_t)n * 4);
    L.active = o; o += al((size_t)n);
    L.score = o; o += al((size_t)n * 8);
    L.segmax = o; o += al((size_t)n * 16);  // two parity buffers
    L.segarg = o; o += al((size_t)n * 16);
    L.segdec = o; o += al((size_t)n);
    L.counters = o; o += 256;
    L.pos = o; o += al((size_t)n * 4);
    L.totals = o; o += al(scan_u32_totals_bytes(n));
    L.total = o;
    return L;
}

}  // namespace

size_t dp_workspace_bytes(int64_t n) { return dp_layout(n).total; }

hipError_t run_dp(const DpArgs &a, void *ws, hipStream_t s, int64_t *n_kept) {
    const DpLayout L = dp_layout(a.n);
    char *w = static_cast<char *>(ws);
    int *lo = reinterpret_cast<int *>(w + L.lo);
    int *hi = reinterpret_cast<int *>(w + L.hi);
    uint8_t *active = reinterpret_cast<uint8_t *>(w + L.active);
    double *score = reinterpret_cast<double *>(w + L.score);
    unsigned long long *segmax = reinterpret_cast<unsigned long long *>(w + L.segmax);
    unsigned long long *segarg = reinterpret_cast<unsigned long long *>(w + L.segarg);
    uint8_t *segdec = reinterpret_cast<uint8_t *>(w + L.segdec);
    unsigned *splits = reinterpret_cast<unsigned *>(w + L.counters);
    unsigned *pos = reinterpret_cast<unsigned *>(w + L.pos);
    unsigned *totals = reinterpret_cast<unsigned *>(w + L.totals);
    const dim3 grid((unsigned)((a.n + 255) / 256)), block(256);
    const double eps2 = a.eps * a.eps;
    *n_kept = -1;
    hipLaunchKernelGGL(zero_u32_kernel, dim3(1), block, 0, s, splits, (int64_t)3);
    hipLaunchKernelGGL(dp_check_kernel, dim3((unsigned)((a.n_tracks + 1 + 255) / 256)), block, 0, s, a.start,
                       a.n_tracks, a.n, splits);
    unsigned chk[3] = {0u, 0u, 0u};  // invalid offsets, tracks longer than kTrackMax, longest other track
    hipError_t e = hipMemcpyAsync(chk, splits, sizeof chk, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    if (chk[0]) return hipErrorInvalidValue;  // *n_kept stays -1: invalid offsets
    if (a.n_tracks > 0 && chk[2] > 0) {
        const int cap = (int)((chk[2] + 63) / 64 * 64);
        hipLaunchKernelGGL(dp_track_kernel, dim3((unsigned)a.n_tracks), dim3(kTrackThreads),
                           (unsigned)dp_track_lds_bytes(cap), s, a.xy, a.start, eps2, cap, a.keep);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int64_t long_groups = chk[1] > 0 ? a.n / kLevelsPerCheck + 1 : -1;  // no long track: no level loop
    if (chk[1] > 0) {
        hipLaunchKernelGGL(dp_init_kernel, grid, block, 0, s, a.start, a.n_tracks, a.n, lo, hi, a.keep, active,
                           segmax, segarg);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        hipLaunchKernelGGL(dp_score_kernel, grid, block, 0, s, a.xy, a.n, static_cast<const int *>(lo),
                           static_cast<const int *>(hi), static_cast<const uint8_t *>(active), score, segmax);
    }
    // Every level either splits a chord or leaves all remaining ones final, so
    // no track needs more levels than it has points.
    int64_t level = 0;
    for (int64_t group = 0; group <= long_groups; ++group) {
        hipLaunchKernelGGL(zero_u32_kernel, dim3(1), block, 0, s, splits, (int64_t)1);
        for (int l = 0; l < kLevelsPerCheck; ++l, ++level) {
            // level's scores are in segmax + cur; the update of its chords also
            // scores the next level into segmax + nxt
            const int64_t cur = (level & 1) * a.n, nxt = ((level + 1) & 1) * a.n;
            hipLaunchKernelGGL(dp_argmax_kernel, grid, block, 0, s, a.n, static_cast<const int *>(lo),
                               static_cast<const uint8_t *>(active), static_cast<const double *>(score),
                               static_cast<const unsigned long long *>(segmax + cur), segarg + cur);
            hipLaunchKernelGGL(dp_decide_kernel, grid, block, 0, s, a.xy, a.n, eps2, static_cast<const int *>(lo),
                               static_cast<const int *>(hi), static_cast<const uint8_t *>(active),
                               static_cast<const double *>(score),
                               static_cast<const unsigned long long *>(segarg + cur), segdec, a.keep, segmax + nxt,
                               segarg + nxt, splits);
            hipLaunchKernelGGL(dp_update_score_kernel, grid, block, 0, s, a.xy, a.n, lo, hi, active,
                               static_cast<const unsigned long long *>(segarg + cur),
                               static_cast<const uint8_t *>(segdec), score, segmax + nxt);
        }
        if ((e = hipGetLastError()) != hipSuccess) return e;
        unsigned got = 0;
        if ((e = hipMemcpyAsync(&got, splits, sizeof got, hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
        if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
        if (got == 0) break;  // no chord split in the whole group: every chord is final
    }
    // Kept count (and compaction) from the exclusive scan of the mask.
    hipLaunchKernelGGL(keep_to_u32_kernel, grid, block, 0, s, static_cast<const uint8_t *>(a.keep), a.n, pos);
    if ((e = launch_scan_u32(pos, a.n, totals, s)) != hipSuccess) return e;
    const int64_t blocks = (a.n + 1023) / 1024;
    unsigned total = 0;
    if ((e = hipMemcpyAsync(&total, totals + blocks, sizeof total, hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
    *n_kept = total;
    if (a.out_xy)
        hipLaunchKernelGGL(dp_compact_kernel, grid, block, 0, s, a.xy, a.n, static_cast<const uint8_t *>(a.keep),
                           static_cast<const unsigned *>(pos), a.out_xy);
    if (a.out_lengths || a.out_start)
        hipLaunchKernelGGL(dp_lengths_kernel, dim3((unsigned)((a.n_tracks + 1 + 255) / 256)), block, 0, s, a.start,
                           a.n_tracks, static_cast<const unsigned *>(pos), total, a.n, a.out_lengths, a.out_start);
    return hipGetLastError();
}

}  // namespace kde
