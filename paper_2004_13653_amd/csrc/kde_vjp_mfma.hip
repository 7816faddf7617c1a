// Vector-Jacobian product of the Gaussian map on gfx950 matrix cores.
//
// The VJP needs, for every point p, the five sums of kde_adjoint.hip (Tx, Ty,
// Ux, Uy, Q), all bilinear in the cotangent Gbar[j][i] and the point's factor
// vectors.  With s_ip = (i - X_p)/Hx, t_jp = (j - Y_p)/Hy, g(u) = exp(-u^2/2)
// and g'(u) = -u g(u), the Gaussian's separability (Sec. III-C) gives
//
//     C0 = Gbar^T Gy   ([nx x ny] by [ny x n], Gy[j][p] = g(t_jp))
//     C1 = Gbar Gx     ([ny x nx] by [nx x n], Gx[i][p] = g(s_ip))
//     Tx_p = sum_i C0[i][p] g'(s_ip)     Ux_p = sum_i C0[i][p] s_ip g'(s_ip)
//     Q_p  = sum_i C0[i][p] g(s_ip)
//     Ty_p = sum_j C1[j][p] g'(t_jp)     Uy_p = sum_j C1[j][p] t_jp g'(t_jp)
//
// so the work is two contractions over the grid ("halves" 0 and 1), each
// followed by a weighted sum over its rows per point.  Both operands are
// BF16 hi/lo pairs (three products hi.hi + hi.lo + lo.hi, FP32 accumulation):
// a single BF16 product would leave relative errors near 1e-3 in the point
// gradients, the split leaves a few 1e-6.
//
// Layout.  A workgroup (8 waves, two per SIMD) owns one half, a 256-row tile of
// that half's M axis (columns i for half 0, rows j for half 1) and 256 points;
// wave w holds the 128 x 64 accumulator block (w / 4, w % 4): 4 x 2 MFMA tiles.
// The contraction axis K (rows j for half 0, columns i for half 1) streams
// through in chunks of 32 nodes, double-buffered in LDS as in the separable map
// (row-major rows of 16-byte words, 8 values each, one pad word per row).
//   * Operand A (the cotangent) is rearranged once per call by vjp_pack_kernel
//     into images of those LDS slices, hi then lo, one contiguous 40 KB block
//     per (half, M tile, chunk); a workgroup copies each chunk's block into LDS
//     with the LDS DMA (global_load_lds) one chunk ahead.
//   * Operand B (the point factors g over the chunk's nodes) is generated in the
//     kernel, one exp2 per factor, half a chunk per MFMA phase.
// Epilogue: each lane weights its accumulators by g, g' and u g' of its rows
// for its two points and sums them; the two lane halves and the two waves that
// share the points are added in a fixed order, giving one partial sum per (half,
// M tile, point) in HBM.  vjp_finish_kernel adds the M tiles in order, writes
// the point gradients and the per-workgroup FP64 sums of Ux, Uy and Q in the
// layout of the vector-unit VJP.  Every order is fixed: results are bitwise
// reproducible.
#include "kde_internal.h"
#include "kde_mfma.h"

#include <algorithm>

namespace kde {

namespace {

constexpr int kVThreads = 512;             // 8 waves
constexpr int kVTile = 256;                // M rows and points per workgroup
constexpr int kVKC = 32;                   // contraction nodes per chunk
constexpr int kVKK = kVKC / 16;            // MFMA k-steps per chunk
constexpr int kVRowWords = kVKC / 8 + 1;   // 16-byte words per LDS row (one pad)
constexpr int kVW = kVTile * kVRowWords;   // words per operand slice
constexpr int kVImage = 2 * kVW;           // A image of one chunk: hi slice, lo slice
constexpr int kVFinish = 256;              // threads of the finishing kernel (one per point)
constexpr float kVFar = 1.0e30f;
constexpr float kHalfLog2e = 0.72134752044448170368f;  // log2(e) / 2

struct VjpMfmaLaunch {
    const float2 *pts;
    int64_t n;
    // Per half (0, 1); scalar fields, so that the kernel selects them without
    // indexing into its argument block.
    const uint4 *img0, *img1;  // A images: [mtiles][nch][kVImage] words
    int mt0, mt1;              // M tiles (ceil(M / 256))
    int nch0, nch1;            // chunks (even)
    float ga0, ga1;            // exp2 scale of the generated (K) axis: sqrt(log2(e)/2) / H
    float inv0, inv1;          // 1 / H of the M axis (epilogue)
    float *part2;         // partial planes, see plane_of
};

// Partial plane of (half, quantity, M tile): half 0 holds T, U, Q (q = 0, 1, 2)
// per M tile, half 1 holds T and U.
__device__ __host__ inline int64_t plane_of(int h, int q, int mt, int mt0, int mt1) {
    return h == 0 ? (int64_t)q * mt0 + mt : 3 * (int64_t)mt0 + (int64_t)q * mt1 + mt;
}

// A images.  Half 0: A[m = i][k = j] = Gbar[j][i]; half 1: A[m = j][k = i] =
// Gbar[j][i].  Word w of a slice: row w / 5, slot w % 5 (slot 4: pad); a slot
// holds the 8 values k = 32 c + 8 slot + 0..7 of row m = 256 mt + row, zero
// outside the grid.  One thread per word, writing hi and lo.
__global__ __launch_bounds__(256) void vjp_pack_kernel(const float *__restrict__ gbar, int nx, int ny,
                                                       uint4 *img0, int mt0, int nch0, uint4 *img1, int mt1,
                                                       int nch1) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t words0 = (int64_t)mt0 * nch0 * kVW, words1 = (int64_t)mt1 * nch1 * kVW;
    if (g >= words0 + words1) return;
    const int h = g < words0 ? 0 : 1;
    const int64_t e = h == 0 ? g : g - words0;
    const int nch = h == 0 ? nch0 : nch1;
    const int64_t blk = e / kVW;  // (mt, c)
    const int w = (int)(e - blk * kVW);
    const int mt = (int)(blk / nch), c = (int)(blk - (int64_t)mt * nch);
    const int row = w / kVRowWords, slot = w - row * kVRowWords;
    float v[8];
    const int m = kVTile * mt + row;
    const int k0 = kVKC * c + 8 * slot;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int k = k0 + q;
        float x = 0.0f;
        if (slot < kVRowWords - 1) {
            if (h == 0) {
                if (m < nx && k < ny) x = gbar[(int64_t)k * nx + m];
            } else {
                if (m < ny && k < nx) x = gbar[(int64_t)m * nx + k];
            }
        }
        v[q] = x;
    }
    const uint4 hi = pack8<true>(v);
    float lo[8];
    residual8<true>(v, hi, lo);
    uint4 *dst = (h == 0 ? img0 : img1) + blk * kVImage;
    dst[w] = hi;
    dst[kVW + w] = pack8<true>(lo);
}

__global__ __launch_bounds__(kVThreads, 1) void vjp_mfma_kernel(VjpMfmaLaunch p) {
    // Double buffers of A (hi slice, lo slice: the copied image) and B (hi, lo),
    // each its own array, so that the compiler can tell the DMA's destination
    // from the factor stores and the fragment reads of the other buffer and
    // need not wait for the DMA before them.
    __shared__ uint4 ldsA0[2 * kVW];
    __shared__ uint4 ldsA1[2 * kVW];
    __shared__ uint4 ldsB0[2 * kVW];
    __shared__ uint4 ldsB1[2 * kVW];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int per = p.mt0 + p.mt1;
    const int item = (int)(blockIdx.x % per);
    const int64_t p0 = (int64_t)(blockIdx.x / per) * kVTile;
    const int h = item < p.mt0 ? 0 : 1;
    const int mt = h == 0 ? item : item - p.mt0;
    const int nch = h == 0 ? p.nch0 : p.nch1;
    const uint4 *img = (h == 0 ? p.img0 : p.img1) + (int64_t)mt * nch * kVImage;
    const float ga = h == 0 ? p.ga0 : p.ga1;

    // Generation role: point t / 2 of the block, nodes 16 (t % 2) .. +16 of each
    // chunk (one 8-node word per phase); its K-axis coordinate (Y for half 0).
    const int gpt = tid >> 1, gw = 2 * (tid & 1);
    float ck = kVFar;
    {
        const int64_t q = p0 + gpt;
        if (q < p.n) {
            const float2 v = p.pts[q];
            ck = h == 0 ? v.y : v.x;
        }
    }
    auto gen_word = [&](int c, int wi, uint4 *buf) {
        float v[8];
        const float k0 = (float)(kVKC * c + 8 * (gw + wi));
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const float t = ((k0 + (float)q) - ck) * ga;
            v[q] = __builtin_amdgcn_exp2f(-t * t);
        }
        const uint4 hi = pack8<true>(v);
        float lo[8];
        residual8<true>(v, hi, lo);
        const int word = gpt * kVRowWords + gw + wi;
        buf[word] = hi;
        buf[kVW + word] = pack8<true>(lo);
    };

    f32x16 acc[4][2];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;

    const int ta0 = 4 * (wave >> 2), tb0 = 2 * (wave & 3);  // first M tile / point tile of this wave
    const int frag0 = (lane & 31) * kVRowWords + (lane >> 5);
    auto frag = [&](int t, int kk) { return frag0 + 32 * t * kVRowWords + 2 * kk; };

    // A chunk: the image block is copied by the waves' LDS DMA (global_load_lds,
    // 16 bytes per lane: wave w moves words 64 (5 w + q) .. +64, q < 5), so the
    // copy holds no registers while it is in flight; each wave waits for its own
    // copies (vmcnt) before the barrier that publishes the chunk.
    auto copy_a = [&](int c, uint4 *buf) {
        const uint4 *src = img + (int64_t)c * kVImage;
#pragma unroll
        for (int q = 0; q < kVImage / kVThreads; ++q) {
            const int base = 64 * ((kVImage / kVThreads) * wave + q);
            __builtin_amdgcn_global_load_lds(src + base + lane, buf + base, 16, 0, 0);
        }
    };
    auto publish = [&]() {
        __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): this wave's DMA writes have landed
        __syncthreads();
    };

    // Chunk 0.
    copy_a(0, ldsA0);
    gen_word(0, 0, ldsB0);
    gen_word(0, 1, ldsB0);
    publish();

    // Step c: MFMAs on chunk c (use) while chunk c + 1 is copied and generated
    // into gen.
    auto step = [&](int c, uint4 *genA, uint4 *genB, const uint4 *useA, const uint4 *useB) {
        const bool more = c + 1 < nch;
        if (more) copy_a(c + 1, genA);
        const uint4 *Ah = useA, *Al = useA + kVW, *Bh = useB, *Bl = useB + kVW;
#pragma unroll
        for (int kk = 0; kk < kVKK; ++kk) {
            uint4 fa[4], fb[2], la[4], lb[2];
#pragma unroll
            for (int i = 0; i < 4; ++i) fa[i] = Ah[frag(ta0 + i, kk)];
#pragma unroll
            for (int j = 0; j < 2; ++j) fb[j] = Bh[frag(tb0 + j, kk)];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) acc[i][j] = mfma<true>(fa[i], fb[j], acc[i][j]);
#pragma unroll
            for (int i = 0; i < 4; ++i) la[i] = Al[frag(ta0 + i, kk)];
#pragma unroll
            for (int j = 0; j < 2; ++j) lb[j] = Bl[frag(tb0 + j, kk)];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    acc[i][j] = mfma<true>(fa[i], lb[j], acc[i][j]);
                    acc[i][j] = mfma<true>(la[i], fb[j], acc[i][j]);
                }
            if (more) gen_word(c + 1, kk, genB);
            __builtin_amdgcn_sched_barrier(0);
        }
        publish();
    };
    for (int c = 0; c < nch; c += 2) {
        step(c, ldsA1, ldsB1, ldsA0, ldsB0);
        step(c + 1, ldsA0, ldsB0, ldsA1, ldsB1);
    }

    // Epilogue.  Register r of lane l in MFMA tile (i, j) holds M row
    // 256 mt + 32 (ta0 + i) + 8 (r / 4) + 4 (l / 32) + r % 4 and point
    // p0 + 32 (tb0 + j) + l % 32.  Rows past the grid hold exact zeros (zero A
    // rows), so they add nothing.
    const float inv = h == 0 ? p.inv0 : p.inv1;
    float T[2], U[2], Q[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int64_t q = p0 + 32 * (tb0 + j) + (lane & 31);
        float cm = kVFar;
        if (q < p.n) {
            const float2 v = p.pts[q];
            cm = h == 0 ? v.x : v.y;
        }
        float t = 0.0f, u = 0.0f, s = 0.0f;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int m = kVTile * mt + 32 * (ta0 + i) + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                const float x = ((float)m - cm) * inv;
                const float g = __builtin_amdgcn_exp2f(-kHalfLog2e * x * x);
                const float dg = -x * g;
                const float c = acc[i][j][r];
                t = fmaf(c, dg, t);
                u = fmaf(c, x * dg, u);
                s = fmaf(c, g, s);
            }
        }
        T[j] = t + __shfl_xor(t, 32);
        U[j] = u + __shfl_xor(u, 32);
        Q[j] = s + __shfl_xor(s, 32);
    }
    // The two waves of a point column (M blocks 0 and 1) meet in LDS.
    float *red = reinterpret_cast<float *>(ldsB0);  // [2 M blocks][3][256 points]
    if (lane < 32) {
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int pl = 32 * (tb0 + j) + lane;
            float *r = red + (wave >> 2) * 3 * kVTile;
            r[pl] = T[j];
            r[kVTile + pl] = U[j];
            r[2 * kVTile + pl] = Q[j];
        }
    }
    __syncthreads();
    if (tid < kVTile && p0 + tid < p.n) {
        const int64_t q = p0 + tid;
        const int mt0 = p.mt0, mt1 = p.mt1;
        const int nq = h == 0 ? 3 : 2;
        for (int k = 0; k < nq; ++k) {
            const float v = red[k * kVTile + tid] + red[3 * kVTile + k * kVTile + tid];
            p.part2[plane_of(h, k, mt, mt0, mt1) * p.n + q] = v;
        }
    }
}

// Adds the M tiles of each point in order, writes the point gradients and the
// per-workgroup FP64 sums (Ux, Uy, Q) of kVFinish points each.
__global__ __launch_bounds__(kVFinish) void vjp_finish_kernel(const float *__restrict__ part2, int64_t n, int mt0,
                                                              int mt1, float fx, float fy, float *grad,
                                                              double *part) {
    __shared__ double red[3][kVFinish];
    const int tid = threadIdx.x;
    const int64_t q = (int64_t)blockIdx.x * kVFinish + tid;
    const bool active = q < n;
    float Tx = 0.0f, Ux = 0.0f, Q = 0.0f, Ty = 0.0f, Uy = 0.0f;
    if (active) {
        for (int mt = 0; mt < mt0; ++mt) {
            Tx += part2[plane_of(0, 0, mt, mt0, mt1) * n + q];
            Ux += part2[plane_of(0, 1, mt, mt0, mt1) * n + q];
            Q += part2[plane_of(0, 2, mt, mt0, mt1) * n + q];
        }
        for (int mt = 0; mt < mt1; ++mt) {
            Ty += part2[plane_of(1, 0, mt, mt0, mt1) * n + q];
            Uy += part2[plane_of(1, 1, mt, mt0, mt1) * n + q];
        }
        if (grad != nullptr) {
            grad[2 * q] = fx * Tx;
            grad[2 * q + 1] = fy * Ty;
        }
    }
    red[0][tid] = active ? (double)Ux : 0.0;
    red[1][tid] = active ? (double)Uy : 0.0;
    red[2][tid] = active ? (double)Q : 0.0;
    __syncthreads();
    for (int w = kVFinish / 2; w > 0; w >>= 1) {
        if (tid < w) {
            red[0][tid] += red[0][tid + w];
            red[1][tid] += red[1][tid + w];
            red[2][tid] += red[2][tid + w];
        }
        __syncthreads();
    }
    if (tid == 0) {
        part[3 * blockIdx.x + 0] = red[0][0];
        part[3 * blockIdx.x + 1] = red[1][0];
        part[3 * blockIdx.x + 2] = red[2][0];
    }
}

struct VjpMfmaPlan {
    int mt[2], nch[2];
    size_t part_bytes, part2_bytes, img_bytes[2];
};

VjpMfmaPlan vjp_mfma_plan(int64_t n, int nx, int ny) {
    VjpMfmaPlan pl;
    const int mdim[2] = {nx, ny}, kdim[2] = {ny, nx};
    for (int h = 0; h < 2; ++h) {
        pl.mt[h] = (mdim[h] + kVTile - 1) / kVTile;
        pl.nch[h] = 2 * ((kdim[h] + 2 * kVKC - 1) / (2 * kVKC));  // even: the loop runs pairs of steps
        pl.img_bytes[h] = (size_t)pl.mt[h] * pl.nch[h] * kVImage * sizeof(uint4);
    }
    const int64_t blocks = (n + kVFinish - 1) / kVFinish;
    pl.part_bytes = ((size_t)blocks * 3 * sizeof(double) + 255) / 256 * 256;
    pl.part2_bytes = ((size_t)(3 * pl.mt[0] + 2 * pl.mt[1]) * n * sizeof(float) + 255) / 256 * 256;
    return pl;
}

}  // namespace

static_assert(kVFinish == 256, "the partial rows match vjp_blocks (256 points per workgroup)");

size_t vjp_mfma_workspace_bytes(int64_t n, int nx, int ny) {
    const VjpMfmaPlan pl = vjp_mfma_plan(n, nx, ny);
    return pl.part_bytes + pl.part2_bytes + pl.img_bytes[0] + pl.img_bytes[1];
}

hipError_t launch_vjp_mfma(const float2 *pts, int64_t n, float Hx, float Hy, const float *gbar, int nx, int ny,
                           float fx, float fy, float *grad, void *ws, hipStream_t stream) {
    const VjpMfmaPlan pl = vjp_mfma_plan(n, nx, ny);
    char *base = static_cast<char *>(ws);
    double *part = reinterpret_cast<double *>(base);
    float *part2 = reinterpret_cast<float *>(base + pl.part_bytes);
    uint4 *img0 = reinterpret_cast<uint4 *>(base + pl.part_bytes + pl.part2_bytes);
    uint4 *img1 = reinterpret_cast<uint4 *>(base + pl.part_bytes + pl.part2_bytes + pl.img_bytes[0]);

    const int64_t words = (int64_t)(pl.mt[0] * pl.nch[0] + pl.mt[1] * pl.nch[1]) * kVW;
    hipLaunchKernelGGL(vjp_pack_kernel, dim3((unsigned)((words + 255) / 256)), dim3(256), 0, stream, gbar, nx, ny,
                       img0, pl.mt[0], pl.nch[0], img1, pl.mt[1], pl.nch[1]);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;

    VjpMfmaLaunch p;
    p.pts = pts;
    p.n = n;
    p.img0 = img0;
    p.img1 = img1;
    p.mt0 = pl.mt[0];
    p.mt1 = pl.mt[1];
    p.nch0 = pl.nch[0];
    p.nch1 = pl.nch[1];
    // Half 0 generates along y (rows) and weights along x; half 1 the reverse.
    p.ga0 = arg_scale(kGaussian, Hy);
    p.ga1 = arg_scale(kGaussian, Hx);
    p.inv0 = (float)(1.0 / (double)Hx);
    p.inv1 = (float)(1.0 / (double)Hy);
    p.part2 = part2;
    const int64_t pblocks = (n + kVTile - 1) / kVTile;
    const int64_t groups = pblocks * (pl.mt[0] + pl.mt[1]);
    main_kernel_begin(stream);
    hipLaunchKernelGGL(vjp_mfma_kernel, dim3((unsigned)groups), dim3(kVThreads), 0, stream, p);
    main_kernel_end(stream);
    e = hipGetLastError();
    if (e != hipSuccess) return e;

    const int64_t blocks = (n + kVFinish - 1) / kVFinish;
    hipLaunchKernelGGL(vjp_finish_kernel, dim3((unsigned)blocks), dim3(kVFinish), 0, stream, part2, n, pl.mt[0],
                       pl.mt[1], fx, fy, grad, part);
    return hipGetLastError();
}

}  // namespace kde
