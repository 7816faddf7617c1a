// C ABI of libkde: argument validation, grid handles, workspace cache and
// dispatch to the HIP kernels.  Every entry point validates all arguments
// before it touches the GPU and never lets a C++ exception escape.
#include "kde.h"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "kde_internal.h"

// Workspace of kde_eval_noalloc: one copy per GPU, held until the process ends.
static __device__ __align__(256) unsigned char scratch[KDE_NOALLOC_SCRATCH_BYTES];

struct kde_grid {
    uint64_t magic;
    double xmin, xmax, ymin, ymax;
    int32_t nx, ny;
    double dx, dy;
};

namespace {

constexpr uint64_t kGridMagic = 0x6b64655f67726964ull;  // "kde_grid"
constexpr int32_t kMaxSide = 65536;
constexpr double kMinH = 1.0 / 1048576.0, kMaxH = 1048576.0;
constexpr int64_t kMaxPoints = (int64_t)1 << 31;

thread_local std::string g_err;

// Events armed by kde_time_next_main_kernel for this thread's next map call.
struct MainTimer {
    hipEvent_t start = nullptr, stop = nullptr;
};
thread_local MainTimer g_timer;

// Disarms the events when a map call returns (whether or not it launched).
struct ConsumeTimer {
    ~ConsumeTimer() { g_timer = MainTimer{}; }
};

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int hip_fail(hipError_t e, const char *where) {
    return fail(KDE_EHIP, "%s: HIP error %d (%s)", where, (int)e, hipGetErrorString(e));
}

bool grid_ok(const kde_grid *g) { return g != nullptr && g->magic == kGridMagic; }

// Library-owned device scratch, one buffer per (device, stream), grown on demand.
std::mutex g_ws_mu;
std::map<std::pair<int, hipStream_t>, std::pair<void *, size_t>> g_ws;

int get_workspace(hipStream_t stream, size_t bytes, void **out) {
    *out = nullptr;
    if (bytes == 0) return KDE_OK;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> lock(g_ws_mu);
    auto &slot = g_ws[{dev, stream}];
    if (slot.second >= bytes) {
        *out = slot.first;
        return KDE_OK;
    }
    if (slot.first != nullptr) {
        // Work already enqueued on this stream may still read the old buffer.
        e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
        e = hipFree(slot.first);
        slot = {nullptr, 0};
        if (e != hipSuccess) return hip_fail(e, "hipFree");
    }
    size_t want = bytes + bytes / 4;
    void *p = nullptr;
    e = hipMalloc(&p, want);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(KDE_ENOMEM, "workspace allocation of %zu bytes failed (%s)", want, hipGetErrorString(e));
    }
    slot = {p, want};
    *out = p;
    return KDE_OK;
}

// Shared validation of (points, n, kernel, hx, hy, grid).
int check_map(const float *points, int64_t n, int32_t kernel_id, double hx, double hy, const kde_grid *g,
              const char *who) {
    if (!grid_ok(g)) return fail(KDE_EINVAL, "%s: invalid grid handle", who);
    if (n < 0 || n >= kMaxPoints) return fail(KDE_EINVAL, "%s: n = %lld out of range [0, 2^31)", who, (long long)n);
    if (n > 0 && points == nullptr) return fail(KDE_EINVAL, "%s: points is NULL with n = %lld", who, (long long)n);
    if (kernel_id < 0 || kernel_id >= KDE_NUM_KERNELS)
        return fail(KDE_EINVAL, "%s: unknown kernel id %d", who, (int)kernel_id);
    if (!(std::isfinite(hx) && std::isfinite(hy) && hx > 0.0 && hy > 0.0))
        return fail(KDE_EINVAL, "%s: bandwidths must be finite and > 0 (hx = %g, hy = %g)", who, hx, hy);
    const double Hx = hx / g->dx, Hy = hy / g->dy;
    if (!(Hx >= kMinH && Hx <= kMaxH && Hy >= kMinH && Hy <= kMaxH))
        return fail(KDE_EINVAL, "%s: bandwidth in grid units (%g, %g) outside [2^-20, 2^20]", who, Hx, Hy);
    return KDE_OK;
}

kde::MapArgs make_args(const float *points, int64_t n, int32_t kernel_id, double hx, double hy, const kde_grid *g,
                       float *out, uint32_t flags) {
    kde::MapArgs a;
    a.pts = reinterpret_cast<const float2 *>(points);
    a.n = n;
    a.kernel_id = kernel_id;
    a.Hx = (float)(hx / g->dx);
    a.Hy = (float)(hy / g->dy);
    a.ax = kde::arg_scale(kernel_id, a.Hx);
    a.ay = kde::arg_scale(kernel_id, a.Hy);
    a.nx = g->nx;
    a.ny = g->ny;
    const double c = kde::kernel_norm(kernel_id);
    a.scale = (flags & KDE_RAW_SUM) ? (float)(c * c) : (float)(c * c / ((double)n * hx * hy));
    a.out = out;
    return a;
}

// ------------------------------------------------------------ tile-shape tuning
// The FP32 direct kernels exist for register blocks of 2, 4 and 8 (tiles of 32,
// 64 and 128 nodes).  The first call in a shape bucket times the candidates on
// the caller's data and stream (each candidate computes the full map, so the
// output is valid whichever runs last) and caches the fastest; see
// kde_autotune.cpp for the buckets.  No tuning while the stream is capturing.

constexpr int kRcGauss = 8;          // defaults: Gaussian maps amortise exp over 8 x 8 blocks,
constexpr int kRcCompact = 2;        // single compact maps gain most from small tiles,
constexpr int kRcCompactBatch = 4;   // batched compact tiles each scan all of the map's points
constexpr float kTuneStopMs = 25.0f; // a default run this long is not tuned further

std::string device_arch() {
    static std::mutex mu;
    static std::map<int, std::string> names;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return "unknown";
    std::lock_guard<std::mutex> lock(mu);
    auto it = names.find(dev);
    if (it != names.end()) return it->second;
    hipDeviceProp_t prop;
    std::string a = "unknown";
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) {
        a = prop.gcnArchName;
        const size_t c = a.find(':');
        if (c != std::string::npos) a.resize(c);
    }
    names[dev] = a;
    return a;
}

int log2_floor(double v) { return v > 0.0 ? (int)std::floor(std::log2(v)) : -1; }

std::string eval_key(const kde::MapArgs &a) {
    char buf[192];
    const double H = std::max(a.Hx, a.Hy);
    std::snprintf(buf, sizeof buf, "eval/%s/%s/H%d/n%d/px%d", device_arch().c_str(),
                  a.kernel_id == KDE_GAUSSIAN ? "gauss" : a.kernel_id == kde::kGaussTrunc ? "gtrunc" : "compact",
                  (int)std::floor(2.0 * std::log2(H)),
                  log2_floor((double)a.n), log2_floor((double)a.nx * a.ny));
    return buf;
}

std::string batch_key(const std::vector<kde::MapArgs> &args) {
    uint64_t h = 1469598103934665603ull;  // FNV-1a
    auto mix = [&](int64_t v) {
        for (int k = 0; k < 8; ++k) {
            h ^= (uint64_t)((v >> (8 * k)) & 0xff);
            h *= 1099511628211ull;
        }
    };
    for (const kde::MapArgs &a : args) {
        mix(a.kernel_id == KDE_GAUSSIAN);
        mix(a.n);
        mix(a.nx);
        mix(a.ny);
    }
    char buf[128];
    std::snprintf(buf, sizeof buf, "batch/%s/%016llx", device_arch().c_str(), (unsigned long long)h);
    return buf;
}

bool capturing(hipStream_t s) {
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    return hipStreamIsCapturing(s, &st) != hipSuccess || st != hipStreamCaptureStatusNone;
}

struct EventPair {
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t init() {
        hipError_t e = hipEventCreate(&a);
        return e == hipSuccess ? hipEventCreate(&b) : e;
    }
    ~EventPair() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

// Runs f() twice (the first run warms up) and times the second on stream s.
template <class F>
hipError_t time_twice(F f, hipStream_t s, const EventPair &ev, float *ms) {
    hipError_t e = f();
    if (e == hipSuccess) e = hipEventRecord(ev.a, s);
    if (e == hipSuccess) e = f();
    if (e == hipSuccess) e = hipEventRecord(ev.b, s);
    if (e == hipSuccess) e = hipEventSynchronize(ev.b);
    if (e == hipSuccess) e = hipEventElapsedTime(ms, ev.a, ev.b);
    return e;
}

// Register-block side for one FP32 direct map: forced, cached, tuned now or default.
int pick_rc(kde::MapArgs a, hipStream_t s, int *rc_out) {
    const int forced = kde::tune::forced();
    int def = a.kernel_id == KDE_GAUSSIAN ? kRcGauss : kRcCompact;
    if (a.kernel_id == kde::kGaussTrunc) {  // the smallest tile that still bins the support
        const float reach = std::max(a.Hx, a.Hy);
        def = reach <= 32.0f ? 2 : reach <= 64.0f ? 4 : 8;
    }
    *rc_out = forced ? forced : def;
    if (forced || !kde::tune::enabled()) return KDE_OK;
    const std::string key = eval_key(a);
    std::string choice;
    if (kde::tune::lookup(key, &choice)) {
        *rc_out = choice[0] - '0';
        return KDE_OK;
    }
    if (capturing(s)) return KDE_OK;
    EventPair ev;
    hipError_t e = ev.init();
    if (e != hipSuccess) return hip_fail(e, "kde_eval (tile-shape tuning)");
    kde::tune::Entry entry;
    float best = INFINITY;
    int best_rc = def;
    std::vector<int> order{def};
    for (int rc : kde::kTileShapes)
        if (rc != def) order.push_back(rc);
    for (int rc : order) {
        a.rc = rc;
        void *ws = nullptr;
        int st = get_workspace(s, kde::direct_workspace_bytes(a), &ws);
        if (st != KDE_OK) return st;
        float ms = 0.0f;
        e = time_twice([&] { return kde::launch_direct(a, ws, s); }, s, ev, &ms);
        if (e != hipSuccess) return hip_fail(e, "kde_eval (tile-shape tuning)");
        entry.ms.emplace_back(std::to_string(rc), (double)ms);
        if (ms < best) {
            best = ms;
            best_rc = rc;
        }
        if (rc == def && ms > kTuneStopMs) break;
    }
    entry.choice = std::to_string(best_rc);
    kde::tune::store(key, entry);
    *rc_out = best_rc;
    return KDE_OK;
}

// Compact maps that a batch sums by fixed-point accumulation take tiles of side
// 64 (one accumulation pass per item) unless a shape is pinned; the tuned side
// applies to the other compact maps.
constexpr int kRcAccumBatch = 4;

void set_batch_rc(std::vector<kde::MapArgs> &args, int rc_gauss, int rc_compact, bool pinned = false) {
    for (kde::MapArgs &a : args)
        a.rc = a.kernel_id == KDE_GAUSSIAN                        ? rc_gauss
               : !pinned && kde::batch_accumulates(a) ? kRcAccumBatch
                                                      : rc_compact;
}

// Register-block sides for a batch (one for its Gaussian maps, one for its
// compact maps): forced, cached, tuned now (runs of the whole batch, in the mode
// of the call: graph replays, whose host part is a copy of the descriptors, or
// eager runs, which rebuild the item list each time) or default.
int pick_batch_rc(std::vector<kde::MapArgs> &args, bool eager, hipStream_t s) {
    const int forced = kde::tune::forced();
    if (forced) {
        set_batch_rc(args, forced, forced, true);
        return KDE_OK;
    }
    set_batch_rc(args, kRcGauss, kRcCompactBatch);
    if (!kde::tune::enabled()) return KDE_OK;
    const std::string key = batch_key(args);
    std::string choice;
    if (kde::tune::lookup(key, &choice)) {
        set_batch_rc(args, choice[0] - '0', choice[2] - '0');
        return KDE_OK;
    }
    if (capturing(s)) return KDE_OK;
    bool has_g = false, has_c = false;
    for (const kde::MapArgs &a : args) (a.kernel_id == KDE_GAUSSIAN ? has_g : has_c) = true;
    std::vector<int> gs{kRcGauss}, cs{kRcCompactBatch};
    if (has_g) gs.push_back(4);
    if (has_c) {
        cs.push_back(2);
        cs.push_back(8);
    }
    EventPair ev;
    hipError_t e = ev.init();
    if (e != hipSuccess) return hip_fail(e, "kde_eval_batched (tile-shape tuning)");
    kde::tune::Entry entry;
    float best = INFINITY;
    int bg = kRcGauss, bc = kRcCompactBatch;
    bool stop = false;
    for (int g : gs) {
        for (int c : cs) {
            set_batch_rc(args, g, c);
            size_t bytes = 0;
            void *ws = nullptr;
            if (eager) {
                bytes = kde::batched_workspace_bytes(args.data(), (int)args.size());
                int st = get_workspace(s, bytes, &ws);
                if (st != KDE_OK) return st;
            }
            float ms = 0.0f;
            e = time_twice([&] { return kde::run_batched(args.data(), (int)args.size(), !eager, ws, bytes, s); }, s,
                           ev, &ms);
            if (e != hipSuccess) return hip_fail(e, "kde_eval_batched (tile-shape tuning)");
            char name[8];
            std::snprintf(name, sizeof name, "%d,%d", g, c);
            entry.ms.emplace_back(name, (double)ms);
            if (ms < best) {
                best = ms;
                bg = g;
                bc = c;
            }
            if (g == kRcGauss && c == kRcCompactBatch && ms > 4.0f * kTuneStopMs) stop = true;
            if (stop) break;
        }
        if (stop) break;
    }
    char name[8];
    std::snprintf(name, sizeof name, "%d,%d", bg, bc);
    entry.choice = name;
    kde::tune::store(key, entry);
    set_batch_rc(args, bg, bc);
    return KDE_OK;
}

// ------------------------------------------------------------ allocation-free maps
// kde_eval_noalloc runs the same launches as kde_eval with a fixed device array
// as its workspace instead of the (device, stream) cache, so it never allocates.
// In host code the array's name stands for a host-side shadow: its device
// address, one per GPU, comes from hipGetSymbolAddress on that GPU and is the
// only form in which it reaches a kernel or a HIP call.

std::mutex g_scratch_mu;
std::map<int, void *> g_scratch_dev;  // device ordinal -> address of `scratch` there

int noalloc_scratch(void **out) {
    *out = nullptr;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    auto it = g_scratch_dev.find(dev);
    if (it != g_scratch_dev.end()) {
        *out = it->second;
        return KDE_OK;
    }
    void *ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || ptr == nullptr)
        return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
    g_scratch_dev[dev] = ptr;
    *out = ptr;
    return KDE_OK;
}

// Register-block side without tuning runs: forced, cached or default.
int untuned_rc(const kde::MapArgs &a) {
    if (const int forced = kde::tune::forced()) return forced;
    int rc = a.kernel_id == KDE_GAUSSIAN ? kRcGauss : kRcCompact;
    if (a.kernel_id == kde::kGaussTrunc) {
        const float reach = std::max(a.Hx, a.Hy);
        rc = reach <= 32.0f ? 2 : reach <= 64.0f ? 4 : 8;
    }
    std::string choice;
    if (kde::tune::enabled() && kde::tune::lookup(eval_key(a), &choice)) rc = choice[0] - '0';
    return rc;
}

// The body of kde_eval and kde_eval_noalloc.
int eval_map(const float *points, int64_t n, int32_t kernel_id, double hx, double hy, const kde_grid *g, float *out,
             int32_t precision, uint32_t flags, void *stream, bool noalloc, const char *who) {
    int st = check_map(points, n, kernel_id, hx, hy, g, who);
    if (st != KDE_OK) return st;
    if (out == nullptr) return fail(KDE_EINVAL, "%s: out is NULL", who);
    if (flags & ~(KDE_RAW_SUM | KDE_TRUNCATE)) return fail(KDE_EINVAL, "%s: unknown flags 0x%x", who, flags);
    if (precision < KDE_FP32_DIRECT || precision > KDE_BF16X3_SEP)
        return fail(KDE_EINVAL, "%s: unknown precision %d", who, (int)precision);
    const bool truncate = (flags & KDE_TRUNCATE) != 0;
    if (truncate && kernel_id != KDE_GAUSSIAN)
        return fail(KDE_EINVAL, "%s: KDE_TRUNCATE applies to the Gaussian kernel only", who);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t plane = (int64_t)g->nx * g->ny;
    if (n == 0) {
        hipError_t e = kde::launch_fill_zero(out, plane, s);
        return e == hipSuccess ? KDE_OK : hip_fail(e, who);
    }
    kde::MapArgs a = make_args(points, n, kernel_id, hx, hy, g, out, flags);
    if (truncate) {  // support 8 bandwidths, Gaussian argument scale and constant
        a.kernel_id = kde::kGaussTrunc;
        a.Hx *= kde::kTruncSigmas;
        a.Hy *= kde::kTruncSigmas;
    }
    const bool direct = precision == KDE_FP32_DIRECT;
    if (direct) {
        if (noalloc) {
            a.rc = untuned_rc(a);
        } else {
            st = pick_rc(a, s, &a.rc);
            if (st != KDE_OK) return st;
        }
    }
    const size_t bytes = direct ? kde::direct_workspace_bytes(a) : kde::sep_workspace_bytes(a, precision);
    void *ws = nullptr;
    if (noalloc) {
        if (bytes > KDE_NOALLOC_SCRATCH_BYTES)
            return fail(KDE_EINVAL, "%s: this map needs %zu bytes of scratch, more than the %zu bytes the "
                        "allocation-free entry point holds (use kde_eval)", who, bytes,
                        (size_t)KDE_NOALLOC_SCRATCH_BYTES);
        if (bytes > 0) st = noalloc_scratch(&ws);
    } else {
        st = get_workspace(s, bytes, &ws);
    }
    if (st != KDE_OK) return st;
    hipError_t e = direct ? kde::launch_direct(a, ws, s) : kde::launch_sep(a, precision, ws, s);
    return e == hipSuccess ? KDE_OK : hip_fail(e, who);
}

}  // namespace

extern "C" {

int kde_create_grid(double xmin, double xmax, double ymin, double ymax, int32_t nx, int32_t ny, kde_grid **out) {
    if (out == nullptr) return fail(KDE_EINVAL, "kde_create_grid: out is NULL");
    *out = nullptr;
    if (!(std::isfinite(xmin) && std::isfinite(xmax) && std::isfinite(ymin) && std::isfinite(ymax)))
        return fail(KDE_EINVAL, "kde_create_grid: bounds must be finite");
    if (!(xmin < xmax && ymin < ymax)) return fail(KDE_EINVAL, "kde_create_grid: need xmin < xmax and ymin < ymax");
    if (nx < 2 || ny < 2 || nx > kMaxSide || ny > kMaxSide)
        return fail(KDE_EINVAL, "kde_create_grid: nx, ny = %d, %d outside [2, %d]", (int)nx, (int)ny, (int)kMaxSide);
    kde_grid *g = new (std::nothrow) kde_grid;
    if (g == nullptr) return fail(KDE_ENOMEM, "kde_create_grid: out of host memory");
    g->magic = kGridMagic;
    g->xmin = xmin;
    g->xmax = xmax;
    g->ymin = ymin;
    g->ymax = ymax;
    g->nx = nx;
    g->ny = ny;
    g->dx = (xmax - xmin) / (double)(nx - 1);
    g->dy = (ymax - ymin) / (double)(ny - 1);
    if (!(g->dx > 0.0 && g->dy > 0.0 && std::isfinite(g->dx) && std::isfinite(g->dy))) {
        delete g;
        return fail(KDE_EINVAL, "kde_create_grid: degenerate node spacing");
    }
    *out = g;
    return KDE_OK;
}

void kde_destroy_grid(kde_grid *g) {
    if (g != nullptr && g->magic == kGridMagic) {
        g->magic = 0;
        delete g;
    }
}

int kde_grid_shape(const kde_grid *g, int32_t *nx, int32_t *ny, double *dx, double *dy) {
    if (!grid_ok(g)) return fail(KDE_EINVAL, "kde_grid_shape: invalid grid handle");
    if (nx) *nx = g->nx;
    if (ny) *ny = g->ny;
    if (dx) *dx = g->dx;
    if (dy) *dy = g->dy;
    return KDE_OK;
}

int kde_to_grid_units(const kde_grid *g, const double *xy, int64_t n, float *out) {
    if (!grid_ok(g)) return fail(KDE_EINVAL, "kde_to_grid_units: invalid grid handle");
    if (n < 0) return fail(KDE_EINVAL, "kde_to_grid_units: n < 0");
    if (n > 0 && (xy == nullptr || out == nullptr)) return fail(KDE_EINVAL, "kde_to_grid_units: NULL buffer");
    for (int64_t p = 0; p < n; ++p) {
        out[2 * p] = (float)((xy[2 * p] - g->xmin) / g->dx);
        out[2 * p + 1] = (float)((xy[2 * p + 1] - g->ymin) / g->dy);
    }
    return KDE_OK;
}

int kde_bandwidth_units(const kde_grid *g, double hx, double hy, float *Hx, float *Hy) {
    int st = check_map(nullptr, 0, KDE_GAUSSIAN, hx, hy, g, "kde_bandwidth_units");
    if (st != KDE_OK) return st;
    if (Hx) *Hx = (float)(hx / g->dx);
    if (Hy) *Hy = (float)(hy / g->dy);
    return KDE_OK;
}

int kde_eval(const float *points, int64_t n, int32_t kernel_id, double hx, double hy, const kde_grid *g, float *out,
             int32_t precision, uint32_t flags, void *stream) {
    ConsumeTimer consume_timer;
    try {
        return eval_map(points, n, kernel_id, hx, hy, g, out, precision, flags, stream, false, "kde_eval");
    } catch (...) {
        return fail(KDE_EHIP, "kde_eval: internal error");
    }
}

int kde_eval_noalloc(const float *points, int64_t n, int32_t kernel_id, double hx, double hy, const kde_grid *g,
                     float *out, int32_t precision, uint32_t flags, void *stream) {
    ConsumeTimer consume_timer;
    try {
        return eval_map(points, n, kernel_id, hx, hy, g, out, precision, flags, stream, true, "kde_eval_noalloc");
    } catch (...) {
        return fail(KDE_EHIP, "kde_eval_noalloc: internal error");
    }
}

int kde_eval_batched(const kde_map *maps, int32_t n_maps, uint32_t flags, void *stream) {
    // A pending main-kernel timing request is cancelled, not served: the batch
    // has no single main kernel.
    g_timer = MainTimer{};
    try {
        if (n_maps < 0 || (n_maps > 0 && maps == nullptr)) return fail(KDE_EINVAL, "kde_eval_batched: bad map array");
        if (flags & ~(KDE_RAW_SUM | KDE_BATCH_EAGER))
            return fail(KDE_EINVAL, "kde_eval_batched: unknown flags 0x%x", flags);
        for (int32_t m = 0; m < n_maps; ++m) {
            const kde_map &d = maps[m];
            int st = check_map(d.points, d.n, d.kernel_id, d.hx, d.hy, d.grid, "kde_eval_batched");
            if (st != KDE_OK) return fail(st, "kde_eval_batched: map %d: %s", m, g_err.c_str());
            if (d.out == nullptr || d.reserved != 0)
                return fail(KDE_EINVAL, "kde_eval_batched: map %d: out is NULL or reserved != 0", m);
            if (d.precision < KDE_FP32_DIRECT || d.precision > KDE_BF16X3_SEP)
                return fail(KDE_EINVAL, "kde_eval_batched: map %d: unknown precision %d", m, (int)d.precision);
            if (d.flags & ~KDE_TRUNCATE)
                return fail(KDE_EINVAL, "kde_eval_batched: map %d: unknown map flags 0x%x", m, d.flags);
            if ((d.flags & KDE_TRUNCATE) && d.kernel_id != KDE_GAUSSIAN)
                return fail(KDE_EINVAL, "kde_eval_batched: map %d: KDE_TRUNCATE applies to the Gaussian only", m);
        }
        if (n_maps == 0) return KDE_OK;
        // FP32 direct maps share the persistent launch; the others run one by one.
        std::vector<kde::MapArgs> args;
        std::vector<int32_t> single;
        for (int32_t m = 0; m < n_maps; ++m) {
            const kde_map &d = maps[m];
            if (d.precision != KDE_FP32_DIRECT || (d.flags & KDE_TRUNCATE)) {
                single.push_back(m);
                continue;
            }
            args.push_back(make_args(d.points, d.n, d.kernel_id, d.hx, d.hy, d.grid, d.out, flags));
            if (d.n == 0) args.back().scale = 0.0f;  // zero map
        }
        hipStream_t s = static_cast<hipStream_t>(stream);
        const bool eager = (flags & KDE_BATCH_EAGER) != 0;
        if (!args.empty()) {
            int st = pick_batch_rc(args, eager, s);
            if (st != KDE_OK) return st;
            void *ws = nullptr;
            size_t bytes = 0;
            if (eager) {
                bytes = kde::batched_workspace_bytes(args.data(), (int)args.size());
                st = get_workspace(s, bytes, &ws);
                if (st != KDE_OK) return st;
            }
            hipError_t e = kde::run_batched(args.data(), (int)args.size(), !eager, ws, bytes, s);
            if (e != hipSuccess) return hip_fail(e, "kde_eval_batched");
        }
        // Dense Gaussian maps on the matrix cores: one launch per precision and
        // kernel (multiplicative runs, or every factor evaluated).
        std::vector<kde::MapArgs> dense[2][KDE_BF16X3_SEP + 1];
        std::vector<int32_t> rest;
        for (int32_t m : single) {
            const kde_map &d = maps[m];
            if (d.precision != KDE_FP32_DIRECT && !(d.flags & KDE_TRUNCATE) && d.n > 0) {
                kde::MapArgs a = make_args(d.points, d.n, d.kernel_id, d.hx, d.hy, d.grid, d.out, flags);
                if (const int kind = kde::sep_dense_batchable(a)) {
                    dense[kind - 1][d.precision].push_back(a);
                    continue;
                }
            }
            rest.push_back(m);
        }
        for (int kind = 0; kind < 2; ++kind) {
            for (int prec = KDE_FP16_SEP; prec <= KDE_BF16X3_SEP; ++prec) {
                const std::vector<kde::MapArgs> &v = dense[kind][prec];
                if (v.empty()) continue;
                void *ws = nullptr;
                int st = get_workspace(s, kde::sep_dense_batch_bytes(v.data(), (int)v.size(), prec), &ws);
                if (st != KDE_OK) return st;
                hipError_t e = kde::launch_sep_dense_batch(v.data(), (int)v.size(), prec, kind == 0, ws, s);
                if (e != hipSuccess) return hip_fail(e, "kde_eval_batched");
            }
        }
        for (int32_t m : rest) {
            const kde_map &d = maps[m];
            int st = eval_map(d.points, d.n, d.kernel_id, d.hx, d.hy, d.grid, d.out, d.precision,
                              d.flags | (flags & KDE_RAW_SUM), stream, false, "kde_eval_batched");
            if (st != KDE_OK) return st;
        }
        if (eager && !single.empty()) {
            hipError_t e = hipStreamSynchronize(s);
            if (e != hipSuccess) return hip_fail(e, "kde_eval_batched");
        }
        return KDE_OK;
    } catch (const std::bad_alloc &) {
        return fail(KDE_ENOMEM, "kde_eval_batched: out of host memory");
    } catch (...) {
        return fail(KDE_EHIP, "kde_eval_batched: internal error");
    }
}

// ------------------------------------------------------------ binned visualisation

namespace {

int check_taps(int32_t kernel_id, double hx, double hy, int32_t a, int32_t b, const kde_grid *g, const char *who) {
    int st = check_map(nullptr, 0, kernel_id, hx, hy, g, who);
    if (st != KDE_OK) return st;
    if (a < 0 || b < 0 || a > kde::kMaxTapRadius || b > kde::kMaxTapRadius)
        return fail(KDE_EINVAL, "%s: tap radii (%d, %d) outside [0, %d]", who, (int)a, (int)b, kde::kMaxTapRadius);
    return KDE_OK;
}

kde::BinnedConvArgs conv_args(const uint32_t *counts, const uint64_t *total, const kde_grid *g, int32_t kernel_id,
                              double hx, double hy, int32_t a, int32_t b, float *out, uint32_t flags) {
    kde::BinnedConvArgs c;
    c.counts = counts;
    c.nx = g->nx;
    c.ny = g->ny;
    c.kernel_id = kernel_id;
    c.Hx = (float)(hx / g->dx);
    c.Hy = (float)(hy / g->dy);
    c.a = a;
    c.b = b;
    const double k0 = kde::kernel_norm(kernel_id);
    c.raw = (flags & KDE_RAW_SUM) != 0;
    c.c2_over_hxhy = c.raw ? k0 * k0 : k0 * k0 / (hx * hy);
    c.total = reinterpret_cast<const unsigned long long *>(total);
    c.out = out;
    return c;
}

size_t align_up(size_t x) { return (x + 255) / 256 * 256; }

}  // namespace

int kde_bin_counts(const float *points, int64_t n, const int32_t *labels, const kde_grid *g, uint32_t *counts,
                   uint64_t *total, void *stream) {
    try {
        if (!grid_ok(g)) return fail(KDE_EINVAL, "kde_bin_counts: invalid grid handle");
        if (n < 0 || n >= kMaxPoints) return fail(KDE_EINVAL, "kde_bin_counts: n = %lld out of range", (long long)n);
        if (n > 0 && points == nullptr) return fail(KDE_EINVAL, "kde_bin_counts: points is NULL with n > 0");
        if (counts == nullptr) return fail(KDE_EINVAL, "kde_bin_counts: counts is NULL");
        hipError_t e = kde::launch_bin_counts(reinterpret_cast<const float2 *>(points), n, labels, g->nx, g->ny,
                                              counts, reinterpret_cast<unsigned long long *>(total),
                                              static_cast<hipStream_t>(stream));
        return e == hipSuccess ? KDE_OK : hip_fail(e, "kde_bin_counts");
    } catch (...) {
        return fail(KDE_EHIP, "kde_bin_counts: internal error");
    }
}

int kde_conv_counts(const uint32_t *counts, const uint64_t *total, const kde_grid *g, int32_t kernel_id, double hx,
                    double hy, int32_t a, int32_t b, float *out, uint32_t flags, void *stream) {
    ConsumeTimer consume_timer;
    try {
        int st = check_taps(kernel_id, hx, hy, a, b, g, "kde_conv_counts");
        if (st != KDE_OK) return st;
        if (counts == nullptr || out == nullptr) return fail(KDE_EINVAL, "kde_conv_counts: counts or out is NULL");
        if (flags & ~KDE_RAW_SUM) return fail(KDE_EINVAL, "kde_conv_counts: unknown flags 0x%x", flags);
        if (!(flags & KDE_RAW_SUM) && total == nullptr)
            return fail(KDE_EINVAL, "kde_conv_counts: a density needs total (or KDE_RAW_SUM)");
        hipStream_t s = static_cast<hipStream_t>(stream);
        void *ws = nullptr;
        st = get_workspace(s, kde::conv_workspace_bytes(g->nx, g->ny), &ws);
        if (st != KDE_OK) return st;
        hipError_t e = kde::launch_conv_counts(conv_args(counts, total, g, kernel_id, hx, hy, a, b, out, flags), ws, s);
        return e == hipSuccess ? KDE_OK : hip_fail(e, "kde_conv_counts");
    } catch (...) {
        return fail(KDE_EHIP, "kde_conv_counts: internal error");
    }
}

int kde_eval_binned(const float *points, int64_t n, const int32_t *labels, int32_t kernel_id, double hx, double hy,
                    int32_t a, int32_t b, const kde_grid *g, float *out, uint32_t flags, void *stream) {
    ConsumeTimer consume_timer;
    try {
        int st = check_taps(kernel_id, hx, hy, a, b, g, "kde_eval_binned");
        if (st != KDE_OK) return st;
        if (n < 0 || n >= kMaxPoints) return fail(KDE_EINVAL, "kde_eval_binned: n = %lld out of range", (long long)n);
        if (n > 0 && points == nullptr) return fail(KDE_EINVAL, "kde_eval_binned: points is NULL with n > 0");
        if (out == nullptr) return fail(KDE_EINVAL, "kde_eval_binned: out is NULL");
        if (flags & ~KDE_RAW_SUM) return fail(KDE_EINVAL, "kde_eval_binned: unknown flags 0x%x", flags);
        hipStream_t s = static_cast<hipStream_t>(stream);
        const size_t cells = (size_t)g->nx * g->ny;
        const size_t counts_bytes = align_up(cells * sizeof(uint32_t)), total_bytes = 256;
        void *ws = nullptr;
        st = get_workspace(s, counts_bytes + total_bytes + kde::conv_workspace_bytes(g->nx, g->ny), &ws);
        if (st != KDE_OK) return st;
        char *w = static_cast<char *>(ws);
        uint32_t *counts = reinterpret_cast<uint32_t *>(w);
        uint64_t *total = reinterpret_cast<uint64_t *>(w + counts_bytes);
        hipError_t e = kde::launch_bin_counts(reinterpret_cast<const float2 *>(points), n, labels, g->nx, g->ny,
                                              counts, reinterpret_cast<unsigned long long *>(total), s);
        if (e == hipSuccess)
            e = kde::launch_conv_counts(conv_args(counts, total, g, kernel_id, hx, hy, a, b, out, flags),
                                        w + counts_bytes + total_bytes, s);
        return e == hipSuccess ? KDE_OK : hip_fail(e, "kde_eval_binned");
    } catch (...) {
        return fail(KDE_EHIP, "kde_eval_binned: internal error");
    }
}

int kde_dp_compress(const double *xy, int64_t n, const int64_t *track_start, int64_t n_tracks, double eps,
                    uint8_t *keep, double *out_xy, int64_t *out_lengths, int64_t *out_start, int64_t *n_kept,
                    void *stream) {
    try {
        if (n < 0 || n >= kMaxPoints) return fail(KDE_EINVAL, "kde_dp_compress: n = %lld out of range", (long long)n);
        if (n_tracks < 0 || (n_tracks == 0 && n > 0) || n_tracks > n)
            return fail(KDE_EINVAL, "kde_dp_compress: n_tracks = %lld invalid for n = %lld", (long long)n_tracks,
                        (long long)n);
        if (!(std::isfinite(eps) && eps >= 0.0)) return fail(KDE_EINVAL, "kde_dp_compress: eps must be finite and >= 0");
        if (n > 0 && (xy == nullptr || track_start == nullptr || keep == nullptr))
            return fail(KDE_EINVAL, "kde_dp_compress: xy, track_start and keep are required");
        hipStream_t s = static_cast<hipStream_t>(stream);
        if (n == 0) {  // no tracks either
            if (out_start != nullptr) {
                hipError_t e = hipMemsetAsync(out_start, 0, sizeof(int64_t), s);
                if (e == hipSuccess) e = hipStreamSynchronize(s);
                if (e != hipSuccess) return hip_fail(e, "kde_dp_compress");
            }
            if (n_kept) *n_kept = 0;
            return KDE_OK;
        }
        void *ws = nullptr;
        int st = get_workspace(s, kde::dp_workspace_bytes(n), &ws);
        if (st != KDE_OK) return st;
        kde::DpArgs a{reinterpret_cast<const double2 *>(xy), n, track_start, n_tracks, eps, keep,
                      reinterpret_cast<double2 *>(out_xy), out_lengths, out_start};
        int64_t kept = 0;
        hipError_t e = kde::run_dp(a, ws, s, &kept);
        if (e == hipErrorInvalidValue && kept < 0)
            return fail(KDE_EINVAL, "kde_dp_compress: track offsets must rise from 0 to n without decreasing");
        if (e != hipSuccess) return hip_fail(e, "kde_dp_compress");
        if (n_kept) *n_kept = kept;
        return KDE_OK;
    } catch (...) {
        return fail(KDE_EHIP, "kde_dp_compress: internal error");
    }
}

static_assert(sizeof(kde_track_metrics) == sizeof(kde::MetricsTotals), "kde_track_metrics layout");

int kde_compression_metrics(const double *xy_o, int64_t n_o, const int64_t *start_o, const double *xy_c, int64_t n_c,
                            const int64_t *start_c, int64_t n_tracks, double *len_o, double *len_c, double *dtw,
                            kde_track_metrics *out, void *stream) {
    ConsumeTimer consume_timer;
    try {
        if (n_o < 0 || n_o >= kMaxPoints || n_c < 0 || n_c >= kMaxPoints)
            return fail(KDE_EINVAL, "kde_compression_metrics: n_o = %lld, n_c = %lld out of range", (long long)n_o,
                        (long long)n_c);
        if (n_tracks < 0 || n_tracks >= kMaxPoints)
            return fail(KDE_EINVAL, "kde_compression_metrics: n_tracks = %lld out of range", (long long)n_tracks);
        if (start_o == nullptr || start_c == nullptr)
            return fail(KDE_EINVAL, "kde_compression_metrics: start_o and start_c are required");
        if ((n_o > 0 && xy_o == nullptr) || (n_c > 0 && xy_c == nullptr))
            return fail(KDE_EINVAL, "kde_compression_metrics: points are required");
        hipStream_t s = static_cast<hipStream_t>(stream);
        const bool given = len_o != nullptr && len_c != nullptr && dtw != nullptr;
        void *ws = nullptr;
        int st = get_workspace(s, kde::metrics_workspace_bytes(n_o, n_c, n_tracks, given), &ws);
        if (st != KDE_OK) return st;
        kde::MetricsArgs a{reinterpret_cast<const double2 *>(xy_o), n_o, start_o, reinterpret_cast<const double2 *>(xy_c),
                           n_c, start_c, n_tracks, len_o, len_c, dtw};
        kde::MetricsTotals t{};
        hipError_t e = kde::run_metrics(a, ws, s, out != nullptr ? &t : nullptr);
        if (e == hipErrorInvalidValue)
            return fail(KDE_EINVAL, "kde_compression_metrics: track offsets must rise from 0 to the point counts "
                                    "without decreasing, tracks under 2^30 points");
        if (e != hipSuccess) return hip_fail(e, "kde_compression_metrics");
        if (out != nullptr) {
            out->n_original = t.n_original;
            out->n_compressed = t.n_compressed;
            out->cr_percent = t.cr_percent;
            out->length_original = t.length_original;
            out->length_compressed = t.length_compressed;
            out->rll = t.rll;
            out->dtw_mean = t.dtw_mean;
            out->dtw_std = t.dtw_std;
        }
        return KDE_OK;
    } catch (...) {
        return fail(KDE_EHIP, "kde_compression_metrics: internal error");
    }
}

int kde_backward(const float *points, int64_t n, int32_t kernel_id, double hx, double hy, const kde_grid *g,
                 const float *grad_out, float *grad_points, double *grad_h, uint32_t flags, void *stream) {
    ConsumeTimer consume_timer;
    try {
        int st = check_map(points, n, kernel_id, hx, hy, g, "kde_backward");
        if (st != KDE_OK) return st;
        if (grad_out == nullptr) return fail(KDE_EINVAL, "kde_backward: grad_out is NULL");
        if (flags & ~(KDE_RAW_SUM | KDE_GRID_UNIT_GRADS | KDE_VJP_FP32))
            return fail(KDE_EINVAL, "kde_backward: unknown flags 0x%x", flags);
        if (grad_points == nullptr && grad_h == nullptr) return KDE_OK;
        if (n == 0) {
            if (grad_h) grad_h[0] = grad_h[1] = 0.0;
            return KDE_OK;
        }
        hipStream_t s = static_cast<hipStream_t>(stream);
        const bool raw = (flags & KDE_RAW_SUM) != 0;
        const float Hx = (float)(hx / g->dx), Hy = (float)(hy / g->dy);
        const double c = kde::kernel_norm(kernel_id);
        // out = sigma * S: sigma = c^2 (raw) or c^2 / (n hx hy) (density).
        const double sigma = raw ? c * c : c * c / ((double)n * hx * hy);
        // dL/dX_p = sigma * (-1/Hx) * Tx_p; world units divide by dx once more.
        const bool grid_units = (flags & KDE_GRID_UNIT_GRADS) != 0;
        const double fx = -sigma / (double)Hx / (grid_units ? 1.0 : g->dx);
        const double fy = -sigma / (double)Hy / (grid_units ? 1.0 : g->dy);
        const int64_t blocks = kde::vjp_blocks(n);
        const size_t mfma_bytes = kde::vjp_mfma_workspace_bytes(n, g->nx, g->ny);
        const bool mfma = kernel_id == KDE_GAUSSIAN && !(flags & KDE_VJP_FP32) && mfma_bytes <= (size_t(4) << 30);
        void *ws = nullptr;
        st = get_workspace(s, mfma ? mfma_bytes : (size_t)blocks * 3 * sizeof(double), &ws);
        if (st != KDE_OK) return st;
        const float2 *pts = reinterpret_cast<const float2 *>(points);
        hipError_t e = mfma ? kde::launch_vjp_mfma(pts, n, Hx, Hy, grad_out, g->nx, g->ny, (float)fx, (float)fy,
                                                   grad_points, ws, s)
                            : kde::launch_vjp(pts, n, kernel_id, Hx, Hy, grad_out, g->nx, g->ny, (float)fx,
                                              (float)fy, grad_points, static_cast<double *>(ws), s);
        if (e != hipSuccess) return hip_fail(e, "kde_backward");
        if (grad_h != nullptr) {
            std::vector<double> part((size_t)blocks * 3);
            e = hipMemcpyAsync(part.data(), ws, part.size() * sizeof(double), hipMemcpyDeviceToHost, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            if (e != hipSuccess) return hip_fail(e, "kde_backward");
            double ux = 0.0, uy = 0.0, q = 0.0;
            for (int64_t b = 0; b < blocks; ++b) {
                ux += part[3 * b];
                uy += part[3 * b + 1];
                q += part[3 * b + 2];
            }
            // d out/dhx = sigma/dx * dS/dHx (+ dsigma/dhx S for densities); with
            // Hx dS/dHx = -sum Gbar s g'(s) g(t) = -Ux and dsigma/dhx = -sigma/hx.
            grad_h[0] = -sigma * ux / ((double)Hx * g->dx) - (raw ? 0.0 : sigma * q / hx);
            grad_h[1] = -sigma * uy / ((double)Hy * g->dy) - (raw ? 0.0 : sigma * q / hy);
        }
        return KDE_OK;
    } catch (...) {
        return fail(KDE_EHIP, "kde_backward: internal error");
    }
}

int kde_lscv(const float *points, int64_t n, int32_t kernel_id, double hx, double hy, const kde_grid *g, double *value,
             double *grad_h, void *stream) {
    try {
        int st = check_map(points, n, kernel_id, hx, hy, g, "kde_lscv");
        if (st != KDE_OK) return st;
        if (n < 2) return fail(KDE_EINVAL, "kde_lscv: need n >= 2");
        if (value == nullptr) return fail(KDE_EINVAL, "kde_lscv: value is NULL");
        hipStream_t s = static_cast<hipStream_t>(stream);
        const float Hx = (float)(hx / g->dx), Hy = (float)(hy / g->dy);
        const int64_t blocks = kde::lscv_blocks(n, kernel_id);
        void *ws = nullptr;
        st = get_workspace(s, kde::lscv_workspace_bytes(n, kernel_id), &ws);
        if (st != KDE_OK) return st;
        hipError_t e = kde::launch_lscv(reinterpret_cast<const float2 *>(points), n, kernel_id, Hx, Hy, g->nx, g->ny,
                                        ws, s);
        if (e != hipSuccess) return hip_fail(e, "kde_lscv");
        std::vector<double> part((size_t)blocks * 6);
        e = hipMemcpyAsync(part.data(), ws, part.size() * sizeof(double), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(e, "kde_lscv");
        double S[6] = {0, 0, 0, 0, 0, 0};
        for (int64_t b = 0; b < blocks; ++b)
            for (int k = 0; k < 6; ++k) S[k] += part[6 * b + k];
        // Remove the p == q terms of the leave-one-out sums (each exactly 1).
        const double nn = (double)n;
        S[3] -= nn;
        S[4] -= nn;
        S[5] -= nn;
        const double pi = 3.14159265358979323846;
        const double c = kde::kernel_norm(kernel_id);  // k = c g
        // kbar = cb kb: the Gaussian's kb is exp(-u^2/4), the Epanechnikov's (2-a)^3 (a^2+6a+4),
        // the others' g * g with k = c g
        const double cb = kernel_id == KDE_GAUSSIAN ? 1.0 / (2.0 * std::sqrt(pi))
                          : kernel_id == KDE_EPANECHNIKOV ? 3.0 / 160.0
                                                          : c * c;
        const double ca = cb * cb / (nn * nn), cbb = 2.0 * c * c / (nn * (nn - 1.0));
        *value = (ca * S[0] - cbb * S[3]) / (hx * hy);
        if (grad_h != nullptr) {
            grad_h[0] = (-ca * S[1] + cbb * S[4]) / (hx * hx * hy);
            grad_h[1] = (-ca * S[2] + cbb * S[5]) / (hx * hy * hy);
        }
        return KDE_OK;
    } catch (...) {
        return fail(KDE_EHIP, "kde_lscv: internal error");
    }
}

int kde_autotune_enable(int32_t on) {
    if (on != 0 && on != 1) return fail(KDE_EINVAL, "kde_autotune_enable: on must be 0 or 1");
    kde::tune::set_enabled(on == 1);
    return KDE_OK;
}

int kde_autotune_force(int32_t rc) {
    if (rc != 0 && !kde::valid_rc(rc)) return fail(KDE_EINVAL, "kde_autotune_force: rc must be 0, 2, 4 or 8");
    kde::tune::set_forced(rc);
    return KDE_OK;
}

int kde_autotune_load(const char *path) {
    try {
        if (path == nullptr) return fail(KDE_EINVAL, "kde_autotune_load: path is NULL");
        std::string err;
        if (!kde::tune::load(path, &err)) return fail(KDE_EINVAL, "kde_autotune_load: %s", err.c_str());
        return KDE_OK;
    } catch (...) {
        return fail(KDE_ENOMEM, "kde_autotune_load: out of host memory");
    }
}

int kde_autotune_save(const char *path) {
    try {
        if (path == nullptr) return fail(KDE_EINVAL, "kde_autotune_save: path is NULL");
        std::string err;
        if (!kde::tune::save(path, &err)) return fail(KDE_EINVAL, "kde_autotune_save: %s", err.c_str());
        return KDE_OK;
    } catch (...) {
        return fail(KDE_ENOMEM, "kde_autotune_save: out of host memory");
    }
}

int kde_autotune_dump(char *buf, size_t cap, size_t *needed) {
    try {
        if (needed == nullptr) return fail(KDE_EINVAL, "kde_autotune_dump: needed is NULL");
        const std::string text = kde::tune::dump();
        *needed = text.size() + 1;
        if (buf == nullptr) return KDE_OK;
        if (cap < text.size() + 1) return fail(KDE_EINVAL, "kde_autotune_dump: buffer of %zu bytes, need %zu", cap,
                                                text.size() + 1);
        std::memcpy(buf, text.c_str(), text.size() + 1);
        return KDE_OK;
    } catch (...) {
        return fail(KDE_ENOMEM, "kde_autotune_dump: out of host memory");
    }
}

int kde_autotune_clear(void) {
    kde::tune::clear();
    return KDE_OK;
}

int kde_time_next_main_kernel(void *start_event, void *stop_event) {
    if ((start_event == nullptr) != (stop_event == nullptr))
        return fail(KDE_EINVAL, "kde_time_next_main_kernel: give both events or neither");
    g_timer.start = static_cast<hipEvent_t>(start_event);
    g_timer.stop = static_cast<hipEvent_t>(stop_event);
    return KDE_OK;
}

const char *kde_last_error(void) { return g_err.c_str(); }

void kde_shutdown(void) {
    std::lock_guard<std::mutex> lock(g_ws_mu);
    int cur = 0;
    bool have_cur = hipGetDevice(&cur) == hipSuccess;
    for (auto &kv : g_ws) {
        if (kv.second.first != nullptr) {
            (void)hipSetDevice(kv.first.first);
            (void)hipFree(kv.second.first);
        }
    }
    g_ws.clear();
    kde::release_batched_graphs();
    kde::release_dense_stage();
    if (have_cur) (void)hipSetDevice(cur);
}

}  // extern "C"

namespace kde {

void main_kernel_begin(hipStream_t stream) {
    if (g_timer.start) (void)hipEventRecord(g_timer.start, stream);
}

void main_kernel_end(hipStream_t stream) {
    if (g_timer.stop) (void)hipEventRecord(g_timer.stop, stream);
}

}  // namespace kde
