// Bfloat16 kernels of the learned-initialisation U-Net (NHWC activations, FP32
// master weights, FP32 accumulation on the matrix cores).
//
// Every convolution is an implicit GEMM  D[m][n] = sum_k A[m][k] W[n][k]:
//   rows m     pixels of a row grid (b, y, x), decoded with shifts (powers of two);
//   columns n  output channels, optionally grouped by output tap
//              (n = t * nout + co, used by the 2x2 stride-2 transposed convolution,
//              whose four taps land on the four sub-pixels of the output);
//   K          (tap, channel) pairs, tap-major, gathered on the fly from up to two
//              NHWC sources (the second one is the skip connection of a
//              concatenation, read in place).
// The same kernel computes data gradients: a 3x3 convolution's input gradient is
// a 3x3 convolution of the output gradient with the flipped, transposed weights,
// and a transposed convolution's input gradient is a 2x2 stride-2 convolution.
// Weight gradients are a second GEMM whose reduction runs over pixels; both of its
// operands are staged transposed through LDS so that each lane reads eight
// consecutive pixels.
//
// Matrix-core layout of v_mfma_f32_32x32x16_bf16 (lane l, 64 lanes):
//   A[row l % 32][k 8 (l / 32) .. + 7], B[k 8 (l / 32) .. + 7][col l % 32],
//   D[row 8 (e / 4) + 4 (l / 32) + e % 4][col l % 32] for accumulator e = 0..15.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace unet {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kThreads = 256;   // four wavefronts
constexpr int kBK = 32;         // K (or pixels, for weight gradients) per pipeline step
constexpr int kLDK = 40;        // LDS row stride in bf16: 80 B, so that 16-byte reads of
                                // consecutive rows by 8 lanes cover all banks once

// Round to nearest even (the hardware conversion, one v_cvt_pk_bf16_f32); NaN stays NaN.
__device__ __forceinline__ uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }

__device__ __forceinline__ float bf2f(uint32_t h) { return __uint_as_float(h << 16); }

__device__ __forceinline__ uint32_t bf_at(const uint4 &v, int e)
{
    const uint32_t w = (e < 2) ? v.x : (e < 4) ? v.y : (e < 6) ? v.z : v.w;
    return (e & 1) ? (w >> 16) : (w & 0xffffu);
}

// Where the K columns come from.
struct Gather {
    const uint16_t *src0, *src1;   // NHWC bf16
    int c0, c1;                    // channels of each source (multiples of 8); c1 = 0: one source
    int hs_log, ws_log;            // source image height / width (log2)
    int stride, kw, pad, taps;     // tap t = (u, v) = (t / kw, t % kw) reads (y stride + u - pad, x stride + v - pad)
};

// The GEMM rows: pixels (b, y, x) of an image of 2^ho_log x 2^wo_log.
struct RowGrid {
    int ho_log, wo_log;
    int m_total;
};

// Column n = t * nout + co goes to channel co of pixel (y ostride + t / okw, x ostride + t % okw)
// of a 2^hd_log x 2^wd_log destination image.
struct OutMap {
    int nout, n_total, ostride, okw, hd_log, wd_log;
};

struct GemmArgs {
    Gather g;
    RowGrid r;
    OutMap o;
    const uint16_t *w;        // [n_total][kpad] bf16
    int kpad;                 // multiple of kBK; columns past taps * (c0 + c1) are zero
    const float *bias;        // [nout] or null
    int relu;
    const uint16_t *mask;     // [dest pixels][d0c]: output *= (mask > 0), or null
    void *dst0;               // channels [0, d0c)
    int d0c;
    void *dst1;               // channels [d0c, nout)
    int d1c;
    int out_f32;              // dst0 is float (otherwise bf16)
};

struct KPos {
    int tap, u, v, ch;
};

__device__ __forceinline__ void kpos_init(KPos &s, int k, const Gather &g)
{
    const int C = g.c0 + g.c1;
    s.tap = k / C;
    s.ch = k - s.tap * C;
    s.u = s.tap / g.kw;
    s.v = s.tap - s.u * g.kw;
}

__device__ __forceinline__ void kpos_advance(KPos &s, const Gather &g, int step = kBK)
{
    const int C = g.c0 + g.c1;
    s.ch += step;
    while (s.ch >= C) {
        s.ch -= C;
        ++s.tap;
        if (++s.v == g.kw) { s.v = 0; ++s.u; }
    }
}

__device__ __forceinline__ void decode(int m, int h_log, int w_log, int &b, int &y, int &x)
{
    x = m & ((1 << w_log) - 1);
    y = (m >> w_log) & ((1 << h_log) - 1);
    b = m >> (w_log + h_log);
}

// Eight consecutive channels of one (pixel, tap): 16 bytes, or zeros outside the image / past K.
__device__ __forceinline__ uint4 gather8(const Gather &g, int b, int sy0, int sx0, bool ok, const KPos &s)
{
    uint4 z = make_uint4(0u, 0u, 0u, 0u);
    if (!ok || s.tap >= g.taps) return z;
    const int sy = sy0 + s.u, sx = sx0 + s.v;
    if (sy < 0 || sx < 0 || sy >= (1 << g.hs_log) || sx >= (1 << g.ws_log)) return z;
    const long long pix = ((long long)((b << g.hs_log) + sy) << g.ws_log) + sx;
    const uint16_t *p = (s.ch < g.c0) ? g.src0 + pix * g.c0 + s.ch : g.src1 + pix * g.c1 + (s.ch - g.c0);
    return *reinterpret_cast<const uint4 *>(p);
}

__device__ __forceinline__ long long dest_pixel(const OutMap &o, int b, int y, int x, int t)
{
    const int ty = t / o.okw, tx = t - ty * o.okw;
    return ((long long)((b << o.hd_log) + y * o.ostride + ty) << o.wd_log) + x * o.ostride + tx;
}

// One pipeline step of BK columns of K, in K order (16 at a time), from LDS rows of LDK bf16.
template <int FM, int FN, int BK = kBK, int LDK = kLDK>
__device__ __forceinline__ void mfma_step(f32x16 (&acc)[FM][FN], const uint16_t *sa, const uint16_t *sb, int lane)
{
#pragma unroll
    for (int kk = 0; kk < BK / 16; ++kk) {
        bf16x8 fa[FM], fb[FN];
        const int off = (lane & 31) * LDK + kk * 16 + (lane >> 5) * 8;
#pragma unroll
        for (int i = 0; i < FM; ++i) fa[i] = *reinterpret_cast<const bf16x8 *>(sa + i * 32 * LDK + off);
#pragma unroll
        for (int j = 0; j < FN; ++j) fb[j] = *reinterpret_cast<const bf16x8 *>(sb + j * 32 * LDK + off);
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[i], fb[j], acc[i][j], 0, 0, 0);
    }
}

// One BM x BN output tile per workgroup; WM x WN wavefronts, each a (BM/WM) x (BN/WN) sub-tile
// of 32 x 32 matrix-core blocks.  Two LDS stages: the global loads of step s+1 are in flight
// while step s runs on the matrix cores.  BK columns of K a step (kpad a multiple of BK): 64
// gives each barrier twice the matrix-core work of 32, with the same products in the same order.
template <int BM, int BN, int WM, int WN, int BK = kBK>
__global__ __launch_bounds__(kThreads) void gemm_kernel(const GemmArgs a)
{
    constexpr int TM = BM / WM, TN = BN / WN, FM = TM / 32, FN = TN / 32;
    constexpr int LDK = BK + 8;                           // LDS row stride (bf16): 16 B past a multiple of 64 B
    constexpr int KC = BK / 8;                            // 16-byte chunks of a row per step
    constexpr int RP = kThreads / KC;                     // rows the workgroup fills per pass
    constexpr int CA = BM / RP;                           // A chunks per thread
    constexpr int NB = BN * KC;                           // B chunks per tile
    constexpr int CB = (NB + kThreads - 1) / kThreads;
    static_assert(WM * WN == 4 && TM % 32 == 0 && TN % 32 == 0 && CA >= 1 && BM % RP == 0, "tile shape");
    __shared__ __attribute__((aligned(16))) uint16_t sA[2][BM * LDK];
    __shared__ __attribute__((aligned(16))) uint16_t sB[2][BN * LDK];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave / WN, wn = wave % WN;
    const int m0 = blockIdx.x * BM, n0 = blockIdx.y * BN;
    const int kc = tid % KC;

    int ab[CA], ay[CA], ax[CA];
    bool aok[CA];
#pragma unroll
    for (int i = 0; i < CA; ++i) {
        const int m = m0 + tid / KC + RP * i;
        int b, y, x;
        decode(m, a.r.ho_log, a.r.wo_log, b, y, x);
        aok[i] = m < a.r.m_total;
        ab[i] = b;
        ay[i] = y * a.g.stride - a.g.pad;
        ax[i] = x * a.g.stride - a.g.pad;
    }
    KPos kp;
    kpos_init(kp, kc * 8, a.g);

    uint4 ra[CA], rb[CB];
    auto load = [&](int step) {
#pragma unroll
        for (int i = 0; i < CA; ++i) ra[i] = gather8(a.g, ab[i], ay[i], ax[i], aok[i], kp);
#pragma unroll
        for (int i = 0; i < CB; ++i) {
            const int q = tid + kThreads * i;
            const int n = n0 + q / KC;
            rb[i] = make_uint4(0u, 0u, 0u, 0u);
            if (q < NB && n < a.o.n_total)
                rb[i] = *reinterpret_cast<const uint4 *>(a.w + (long long)n * a.kpad + step * BK + (q % KC) * 8);
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int i = 0; i < CA; ++i)
            *reinterpret_cast<uint4 *>(&sA[buf][(tid / KC + RP * i) * LDK + kc * 8]) = ra[i];
#pragma unroll
        for (int i = 0; i < CB; ++i) {
            const int q = tid + kThreads * i;
            if (q < NB) *reinterpret_cast<uint4 *>(&sB[buf][(q / KC) * LDK + (q % KC) * 8]) = rb[i];
        }
    };

    f32x16 acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
            for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.0f;

    const int nsteps = a.kpad / BK;
    load(0);
    store(0);
    __syncthreads();
    for (int s = 0; s < nsteps; ++s) {
        const int cur = s & 1;
        if (s + 1 < nsteps) {
            kpos_advance(kp, a.g, BK);
            load(s + 1);
        }
        mfma_step<FM, FN, BK, LDK>(acc, &sA[cur][wm * TM * LDK], &sB[cur][wn * TN * LDK], lane);
        if (s + 1 < nsteps) store(cur ^ 1);
        __syncthreads();
    }

    // Epilogue: bias, ReLU, mask, split over two destinations.
#pragma unroll
    for (int j = 0; j < FN; ++j) {
        const int n = n0 + wn * TN + j * 32 + (lane & 31);
        if (n >= a.o.n_total) continue;
        const int t = n / a.o.nout, co = n - t * a.o.nout;
        const float bias = a.bias ? a.bias[co] : 0.0f;
        if (a.out_f32) {
#pragma unroll
            for (int i = 0; i < FM; ++i) {
#pragma unroll
                for (int e = 0; e < 16; ++e) {
                    const int m = m0 + wm * TM + i * 32 + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
                    if (m >= a.r.m_total || co >= a.d0c) continue;
                    int b, y, x;
                    decode(m, a.r.ho_log, a.r.wo_log, b, y, x);
                    const long long d = dest_pixel(a.o, b, y, x, t);
                    float val = acc[i][j][e] + bias;
                    if (a.relu) val = fmaxf(val, 0.0f);
                    if (a.mask && !(bf2f(a.mask[d * a.d0c + co]) > 0.0f)) val = 0.0f;
                    static_cast<float *>(a.dst0)[d * a.d0c + co] = val;
                }
            }
            continue;
        }
        // bf16 outputs: elements e and e + 1 are consecutive rows (pixels) of column n; lanes n and
        // n ^ 1 (channels co and co ^ 1 of one tap: nout, d0c and d1c are even) swap one of them so
        // that each writes both channels of one pixel as a 32-bit word
        const bool odd = co & 1;
        uint16_t *dst = co < a.d0c ? static_cast<uint16_t *>(a.dst0) : static_cast<uint16_t *>(a.dst1);
        const int ldd = co < a.d0c ? a.d0c : a.d1c;
        const int cd = (co < a.d0c ? co : co - a.d0c) & ~1;
        const bool masked = a.mask && co < a.d0c;
#pragma unroll
        for (int i = 0; i < FM; ++i) {
#pragma unroll
            for (int e = 0; e < 16; e += 2) {
                float v0 = acc[i][j][e] + bias, v1 = acc[i][j][e + 1] + bias;
                if (a.relu) {
                    v0 = fmaxf(v0, 0.0f);
                    v1 = fmaxf(v1, 0.0f);
                }
                const float got = __shfl_xor(odd ? v0 : v1, 1, 64);
                float lo = odd ? got : v0, hi = odd ? v1 : got;
                const int ee = odd ? e + 1 : e;
                const int m = m0 + wm * TM + i * 32 + 8 * (ee >> 2) + 4 * (lane >> 5) + (ee & 3);
                if (m >= a.r.m_total) continue;
                int b, y, x;
                decode(m, a.r.ho_log, a.r.wo_log, b, y, x);
                const long long d = dest_pixel(a.o, b, y, x, t) * ldd + cd;
                if (masked) {
                    const uint32_t mk = *reinterpret_cast<const uint32_t *>(a.mask + d);
                    if (!(bf2f(mk & 0xffffu) > 0.0f)) lo = 0.0f;
                    if (!(bf2f(mk >> 16) > 0.0f)) hi = 0.0f;
                }
                *reinterpret_cast<uint32_t *>(dst + d) = (uint32_t)f2bf(lo) | ((uint32_t)f2bf(hi) << 16);
            }
        }
    }
}

// Weight gradient partials  P[z][n][k] = sum over pixels m of split z of dY(m, n) A[m][k],
// where A is the forward gather and dY(m, n) is channel co of the output gradient at the
// destination pixel of (m, t), n = t * nout + co.
struct WgradArgs {
    Gather g;
    RowGrid r;
    OutMap o;
    const uint16_t *gy;       // output gradient [dest pixels][gyc] bf16
    int gyc;
    int n_rows;               // rows of the weight matrix (n < n_rows written)
    int kpad;
    int m_chunk;              // pixels per split, multiple of kBK
    float *part;              // [splits][n_rows][kpad]
};

__device__ __forceinline__ uint32_t pack2(uint32_t lo, uint32_t hi) { return lo | (hi << 16); }

template <int BM, int BN, int WM, int WN>
__global__ __launch_bounds__(kThreads) void wgrad_kernel(const WgradArgs a)
{
    constexpr int TM = BM / WM, TN = BN / WN, FM = TM / 32, FN = TN / 32;
    constexpr int PG = 2 * BM, PX = 2 * BN;               // pixel-pair chunks per step
    constexpr int CG = (PG + kThreads - 1) / kThreads, CX = (PX + kThreads - 1) / kThreads;
    static_assert(WM * WN == 4 && TM % 32 == 0 && TN % 32 == 0, "tile shape");
    __shared__ __attribute__((aligned(16))) uint16_t sG[2][BM * kLDK];
    __shared__ __attribute__((aligned(16))) uint16_t sX[2][BN * kLDK];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave / WN, wn = wave % WN;
    const int k0 = blockIdx.x * BN, n0 = blockIdx.y * BM;
    const int mz0 = blockIdx.z * a.m_chunk;
    const int mz1 = min(a.r.m_total, mz0 + a.m_chunk);

    // Fixed per thread: the channel group of each chunk; the pixels advance.
    int gt[CG], gco[CG];
    bool gok[CG];
#pragma unroll
    for (int i = 0; i < CG; ++i) {
        const int q = tid + kThreads * i;
        const int n = n0 + (q >> 4) * 8;
        gok[i] = q < PG && n < a.o.n_total;
        gt[i] = n / a.o.nout;
        gco[i] = n - gt[i] * a.o.nout;
    }
    KPos xk[CX];
    bool xok[CX];
#pragma unroll
    for (int i = 0; i < CX; ++i) {
        const int q = tid + kThreads * i;
        xok[i] = q < PX;
        kpos_init(xk[i], k0 + (q >> 4) * 8, a.g);
    }

    uint4 rg[CG][2], rx[CX][2];
    auto load = [&](int ms) {
#pragma unroll
        for (int i = 0; i < CG; ++i)
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int m = ms + 2 * ((tid + kThreads * i) & 15) + h;
                rg[i][h] = make_uint4(0u, 0u, 0u, 0u);
                if (gok[i] && m < mz1) {
                    int b, y, x;
                    decode(m, a.r.ho_log, a.r.wo_log, b, y, x);
                    const long long d = dest_pixel(a.o, b, y, x, gt[i]);
                    rg[i][h] = *reinterpret_cast<const uint4 *>(a.gy + d * a.gyc + gco[i]);
                }
            }
#pragma unroll
        for (int i = 0; i < CX; ++i)
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int m = ms + 2 * ((tid + kThreads * i) & 15) + h;
                int b, y, x;
                decode(m, a.r.ho_log, a.r.wo_log, b, y, x);
                rx[i][h] = gather8(a.g, b, y * a.g.stride - a.g.pad, x * a.g.stride - a.g.pad,
                                   xok[i] && m < mz1, xk[i]);
            }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int i = 0; i < CG; ++i) {
            const int q = tid + kThreads * i;
            if (q >= PG) continue;
            uint16_t *row = &sG[buf][((q >> 4) * 8) * kLDK + 2 * (q & 15)];
#pragma unroll
            for (int e = 0; e < 8; ++e)
                *reinterpret_cast<uint32_t *>(row + e * kLDK) = pack2(bf_at(rg[i][0], e), bf_at(rg[i][1], e));
        }
#pragma unroll
        for (int i = 0; i < CX; ++i) {
            const int q = tid + kThreads * i;
            if (q >= PX) continue;
            uint16_t *row = &sX[buf][((q >> 4) * 8) * kLDK + 2 * (q & 15)];
#pragma unroll
            for (int e = 0; e < 8; ++e)
                *reinterpret_cast<uint32_t *>(row + e * kLDK) = pack2(bf_at(rx[i][0], e), bf_at(rx[i][1], e));
        }
    };

    f32x16 acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
            for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.0f;

    const int nsteps = (mz1 > mz0) ? (mz1 - mz0 + kBK - 1) / kBK : 0;
    if (nsteps > 0) {
        load(mz0);
        store(0);
    }
    __syncthreads();
    for (int s = 0; s < nsteps; ++s) {
        const int cur = s & 1;
        if (s + 1 < nsteps) load(mz0 + (s + 1) * kBK);
        mfma_step<FM, FN>(acc, &sG[cur][wm * TM * kLDK], &sX[cur][wn * TN * kLDK], lane);
        if (s + 1 < nsteps) store(cur ^ 1);
        __syncthreads();
    }

    float *out = a.part + (long long)blockIdx.z * a.n_rows * a.kpad;
#pragma unroll
    for (int j = 0; j < FN; ++j) {
        const int k = k0 + wn * TN + j * 32 + (lane & 31);
        if (k >= a.kpad) continue;
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int n = n0 + wm * TM + i * 32 + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
                if (n < a.n_rows) out[(long long)n * a.kpad + k] = acc[i][j][e];
            }
    }
}

// grad[i] = sum_z part[z][i], z ascending.  Four consecutive elements per lane when count is a
// multiple of 4; the loads of 8 splits are issued before their (in-order) additions.
__global__ void sum_splits_kernel(const float *__restrict__ part, int splits, long long count, float *__restrict__ grad)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if ((count & 3) == 0) {
        const long long i = 4 * t;
        if (i >= count) return;
        float4 s = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll 8
        for (int z = 0; z < splits; ++z) {
            const float4 v = *reinterpret_cast<const float4 *>(part + (long long)z * count + i);
            s.x += v.x;
            s.y += v.y;
            s.z += v.z;
            s.w += v.w;
        }
        *reinterpret_cast<float4 *>(grad + i) = s;
    } else {
        if (t >= count) return;
        float s = 0.0f;
#pragma unroll 8
        for (int z = 0; z < splits; ++z) s += part[(long long)z * count + t];
        grad[t] = s;
    }
}

// Per-channel sums of an output gradient [pixels][gyc] over a pixel chunk.  A lane owns 8
// channels (one 16-byte load per pixel); the 256 lanes are gyc / 8 channel groups x phases over
// the chunk's pixels, reduced over phases in a fixed order.
__global__ __launch_bounds__(kThreads) void colsum_partial_kernel(const uint16_t *__restrict__ gy, int gyc, int nout,
                                                                  long long pixels, int chunk, float *__restrict__ part)
{
    __shared__ float red[kThreads * 8];
    const int tid = threadIdx.x;
    const int groups = gyc >> 3;                 // <= 32
    const int g = tid % groups, ph = tid / groups, nph = kThreads / groups;
    const long long p0 = (long long)blockIdx.x * chunk;
    const long long p1 = min(pixels, p0 + chunk);
    float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (ph < nph)
        for (long long p = p0 + ph; p < p1; p += nph) {
            const uint4 v = *reinterpret_cast<const uint4 *>(gy + p * gyc + g * 8);
#pragma unroll
            for (int e = 0; e < 8; ++e) acc[e] += bf2f(bf_at(v, e));
        }
#pragma unroll
    for (int e = 0; e < 8; ++e) red[tid * 8 + e] = acc[e];
    __syncthreads();
    for (int c = tid; c < nout; c += kThreads) {
        const int cg = c >> 3, e = c & 7;
        float t = 0.0f;
        for (int k = 0; k < nph; ++k) t += red[(k * groups + cg) * 8 + e];
        part[(long long)blockIdx.x * nout + c] = t;
    }
}

// Adam over a flat parameter vector (FP32 master weights).  c1 = 1 / (1 - beta1^t), c2 = 1 / (1 - beta2^t).
__global__ void adam_kernel(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                            float *__restrict__ v, long long count, float lr, float beta1, float beta2,
                            float eps, float c1, float c2)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const float gi = g[i];
    const float mi = beta1 * m[i] + (1.0f - beta1) * gi;
    const float vi = beta2 * v[i] + (1.0f - beta2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

// Forward bf16 copy of a weight matrix.
__global__ void to_bf16_kernel(const float *__restrict__ w, long long count, uint16_t *__restrict__ out)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) out[i] = f2bf(w[i]);
}

// Data-gradient weights  Wd[r][t' G + co]  (rows r = input channels, kd columns):
//   convolutions:        W[co][(taps - 1 - t') cin + r]   (flipped taps)
//   transposed conv.:    W[t' cout + co][r]
// zero for co >= cout and past taps * G.
__global__ void dgrad_weights_kernel(const float *__restrict__ w, int transposed, int taps, int cin, int cout,
                                     int G, int kpad, int rows, int kd, uint16_t *__restrict__ out)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long long)rows * kd) return;
    const int r = (int)(i / kd), c = (int)(i - (long long)r * kd);
    const int t = c / G, co = c - t * G;
    float val = 0.0f;
    if (t < taps && co < cout) {
        if (transposed) val = w[(long long)(t * cout + co) * kpad + r];
        else val = w[(long long)co * kpad + (taps - 1 - t) * cin + r];
    }
    out[i] = f2bf(val);
}

// 2x2 max pooling, 8 channels per lane.
__global__ void maxpool_kernel(const uint16_t *__restrict__ x, int c, int h_log, int w_log, long long count,
                               uint16_t *__restrict__ y)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;   // (pooled pixel, channel group)
    if (i >= count) return;
    const int groups = c >> 3;
    const long long pp = i / groups;
    const int cg = (int)(i - pp * groups) * 8;
    const int wo_log = w_log - 1, ho_log = h_log - 1;
    const int xo = (int)(pp & ((1 << wo_log) - 1));
    const int yo = (int)((pp >> wo_log) & ((1 << ho_log) - 1));
    const long long b = pp >> (wo_log + ho_log);
    uint4 v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const long long src = ((b << h_log) + 2 * yo + (q >> 1)) * (1LL << w_log) + 2 * xo + (q & 1);
        v[q] = *reinterpret_cast<const uint4 *>(x + src * c + cg);
    }
    uint32_t o[4];
#pragma unroll
    for (int e2 = 0; e2 < 4; ++e2) {
        uint32_t pair = 0;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int e = 2 * e2 + h;
            uint32_t best = bf_at(v[0], e);
#pragma unroll
            for (int q = 1; q < 4; ++q) {
                const uint32_t cand = bf_at(v[q], e);
                if (bf2f(cand) > bf2f(best)) best = cand;
            }
            pair |= best << (16 * h);
        }
        o[e2] = pair;
    }
    *reinterpret_cast<uint4 *>(y + pp * c + cg) = make_uint4(o[0], o[1], o[2], o[3]);
}

// Gradient at an encoder output a (post-ReLU) that feeds both the pooling and a skip
// connection:  d a = (route(d pooled) + d skip) * (a > 0), where route sends each pooled
// gradient to the first maximum of its window in the order (0,0), (0,1), (1,0), (1,1).
__global__ void maxpool_backward_kernel(const uint16_t *__restrict__ a, const uint16_t *__restrict__ gpool,
                                        const uint16_t *__restrict__ gskip, int c, int h_log, int w_log,
                                        long long count, uint16_t *__restrict__ ga)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const int groups = c >> 3;
    const long long pp = i / groups;
    const int cg = (int)(i - pp * groups) * 8;
    const int wo_log = w_log - 1, ho_log = h_log - 1;
    const int xo = (int)(pp & ((1 << wo_log) - 1));
    const int yo = (int)((pp >> wo_log) & ((1 << ho_log) - 1));
    const long long b = pp >> (wo_log + ho_log);
    long long src[4];
    uint4 v[4], sk[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        src[q] = ((b << h_log) + 2 * yo + (q >> 1)) * (1LL << w_log) + 2 * xo + (q & 1);
        v[q] = *reinterpret_cast<const uint4 *>(a + src[q] * c + cg);
        sk[q] = *reinterpret_cast<const uint4 *>(gskip + src[q] * c + cg);
    }
    const uint4 gp = *reinterpret_cast<const uint4 *>(gpool + pp * c + cg);
    uint32_t o[4][4] = {};
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        int arg = 0;
        float best = bf2f(bf_at(v[0], e));
#pragma unroll
        for (int q = 1; q < 4; ++q) {
            const float cand = bf2f(bf_at(v[q], e));
            if (cand > best) { best = cand; arg = q; }
        }
        const float g = bf2f(bf_at(gp, e));
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            float val = bf2f(bf_at(sk[q], e)) + (q == arg ? g : 0.0f);
            if (!(bf2f(bf_at(v[q], e)) > 0.0f)) val = 0.0f;
            o[q][e >> 1] |= (uint32_t)f2bf(val) << (16 * (e & 1));
        }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
        *reinterpret_cast<uint4 *>(ga + src[q] * c + cg) = make_uint4(o[q][0], o[q][1], o[q][2], o[q][3]);
}

// Centred mean-squared error, first pass: per (sample, pixel chunk, channel) sums of
// e = y - target and e^2 in FP64, fixed-order reduction inside the workgroup.
constexpr int kMseChunks = 64;   // pixel chunks per sample

__global__ __launch_bounds__(kThreads) void mse_partial_kernel(const float *__restrict__ y, const float *__restrict__ tg,
                                                               int oc, long long hw, double *__restrict__ part)
{
    __shared__ double red[kThreads];
    const int tid = threadIdx.x;
    const long long b = blockIdx.y;
    const long long chunk = (hw + kMseChunks - 1) / kMseChunks;
    const long long q0 = blockIdx.x * chunk, q1 = min(hw, q0 + chunk);
    const long long base = b * hw * oc;
    for (int c = 0; c < oc; ++c) {
        double s1 = 0.0, s2 = 0.0;
        for (long long q = q0 + tid; q < q1; q += kThreads) {
            const double e = (double)y[base + q * oc + c] - (double)tg[base + q * oc + c];
            s1 += e;
            s2 += e * e;
        }
        for (int pass = 0; pass < 2; ++pass) {
            red[tid] = pass ? s2 : s1;
            __syncthreads();
            for (int w = kThreads / 2; w > 0; w >>= 1) {
                if (tid < w) red[tid] += red[tid + w];
                __syncthreads();
            }
            if (tid == 0) part[((b * oc + c) * kMseChunks + blockIdx.x) * 2 + pass] = red[0];
            __syncthreads();
        }
    }
}

// The chunk partials of each (sample, channel) added in order.
__global__ void mse_stats_kernel(const double *__restrict__ part, int groups, double *__restrict__ stats)
{
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= groups) return;
    double s1 = 0.0, s2 = 0.0;
    for (int k = 0; k < kMseChunks; ++k) {
        s1 += part[((long long)g * kMseChunks + k) * 2];
        s2 += part[((long long)g * kMseChunks + k) * 2 + 1];
    }
    stats[2 * g] = s1;
    stats[2 * g + 1] = s2;
}

// Second pass: d loss / d y = 2 (e - mean e) / count, written as bf16 with gc channels a pixel
// (oc rounded up to a multiple of 8; channels >= oc are zero); the loss itself by one lane.
__global__ void mse_grad_kernel(const float *__restrict__ y, const float *__restrict__ tg, const double *__restrict__ stats,
                                int oc, int gc, long long hw, long long pixels, uint16_t *__restrict__ gy,
                                double *loss_out)
{
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const double count = (double)pixels * oc;
    if (p == 0 && loss_out) {
        const long long groups = pixels / hw * oc;
        double l = 0.0;
        for (long long q = 0; q < groups; ++q) l += stats[2 * q + 1] - stats[2 * q] * stats[2 * q] / (double)hw;
        *loss_out = l / count;
    }
    if (p >= pixels) return;
    const long long b = p / hw;
    for (int c8 = 0; c8 < gc; c8 += 8) {
        uint32_t o[4] = {0u, 0u, 0u, 0u};
        for (int c = c8; c < min(oc, c8 + 8); ++c) {
            const double mean = stats[(b * oc + c) * 2] / (double)hw;
            const double e = (double)y[p * oc + c] - (double)tg[p * oc + c];
            o[(c - c8) >> 1] |= (uint32_t)f2bf((float)(2.0 * (e - mean) / count)) << (16 * (c & 1));
        }
        *reinterpret_cast<uint4 *>(gy + p * gc + c8) = make_uint4(o[0], o[1], o[2], o[3]);
    }
}

// Direct 3x3 convolution (stride 1, zero padding 1) to 32 output channels, for the two finest
// levels: forward passes and data gradients (the same convolution of the output gradient with
// the flipped weights, and a ReLU mask).  A layer with 64 or 128 output channels takes one
// launch per 32; a gradient split over a concatenation's two sources sends each launch to its
// source.  The implicit GEMM gathers
// every input pixel's channels once per tap (nine times) through L2; this kernel stages the
// layer's weights once per workgroup and a (TH + 2) x 18 halo of input pixels per TH x 16 output
// tile in LDS, and reads the nine shifted A fragments from there.  Inputs: C = c0 + c1 channels
// per pixel (a second source is the skip of a concatenation); weights bf16 [32][kpad] with
// k = tap * C + channel (tap-major, the GEMM's order, so the sums are the GEMM's).  Each of the
// four wavefronts owns TH / 4 output rows (TH * 4 pixels = TH / 8 row blocks of 32).  With C = 8
// (the network's input, 6 channels padded to 8) one matrix-core step of K = 16 takes two taps,
// the lower half of the lanes the first and the upper half the second, and the ninth tap pairs
// with the weights' zero padding (k in [72, 80)).
struct Conv3Args {
    const uint16_t *src0, *src1;   // NHWC bf16
    int c0, c1;                    // channels of each source (c1 = 0: one source)
    int h_log, w_log;              // image height / width (log2)
    const uint16_t *w;             // [32][kpad]
    int kpad;
    const float *bias;             // [32] or null
    int relu;
    const uint16_t *mask;          // [pixels][ldd] bf16: output *= (mask > 0), or null (data gradients)
    uint16_t *dst;                 // NHWC bf16 with ldd channels a pixel; this launch writes 32 of them
    int ldd;                       // channels per output pixel (a multiple of 32: one launch per 32)
};

template <int TH, int C, int TY>
__global__ __launch_bounds__(kThreads) void conv3x3_kernel(const Conv3Args a)
{
    constexpr int TW = 16, HW = TW + 2, HP = (TH + 2) * HW;   // halo width and pixels
    constexpr int LDH = C + 8;                                // bf16 per halo pixel (bank padding)
    constexpr int K = 9 * C, LDW = K + 8;                     // weight row stride
    constexpr int KW = C == 8 ? 80 : K;                       // weight columns staged (C = 8: with the pad)
    constexpr int FM = TH / 8;                                // 32-pixel blocks per wavefront
    __shared__ __attribute__((aligned(16))) uint16_t halo[HP * LDH];
    __shared__ __attribute__((aligned(16))) uint16_t wl[32 * LDW];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int x0 = blockIdx.x * TW, b = blockIdx.z;
    const int H = 1 << a.h_log, W = 1 << a.w_log;
    for (int q = tid; q < 32 * (KW / 8); q += kThreads) {
        const int n = q / (KW / 8), k = (q % (KW / 8)) * 8;
        *reinterpret_cast<uint4 *>(&wl[n * LDW + k]) = *reinterpret_cast<const uint4 *>(a.w + (long long)n * a.kpad + k);
    }
    // this lane's A row: pixel p = i 32 + lane % 32 of the wavefront's rows
    const int r0 = wave * (TH / 4);
    int hbase[FM];
#pragma unroll
    for (int i = 0; i < FM; ++i) {
        const int p = i * 32 + (lane & 31);
        hbase[i] = ((r0 + p / TW) * HW + p % TW) * LDH + (C == 8 ? 0 : (lane >> 5) * 8);
    }
    const uint16_t *wrow = wl + (lane & 31) * LDW + (lane >> 5) * 8;
    const int co = lane & 31;
    const float bias = a.bias ? a.bias[co] : 0.0f;
    // TY tiles along y share the staged weights; the next tile's halo is loaded into
    // registers (16-byte pieces of 8 channels, zeros outside the image) while the matrix
    // cores work on the current one
    constexpr int NQ = HP * (C / 8), NCH = (NQ + kThreads - 1) / kThreads;
    uint4 rh[NCH];
    auto fetch = [&](int y0) {
#pragma unroll
        for (int r = 0; r < NCH; ++r) {
            const int q = tid + r * kThreads;
            rh[r] = make_uint4(0u, 0u, 0u, 0u);
            if (q < NQ) {
                const int pix = q / (C / 8), ch = (q % (C / 8)) * 8;
                const int y = y0 - 1 + pix / HW, x = x0 - 1 + pix % HW;
                if (y >= 0 && y < H && x >= 0 && x < W) {
                    const long long gp = ((long long)((b << a.h_log) + y) << a.w_log) + x;
                    rh[r] = ch < a.c0 ? *reinterpret_cast<const uint4 *>(a.src0 + gp * a.c0 + ch)
                                      : *reinterpret_cast<const uint4 *>(a.src1 + gp * a.c1 + (ch - a.c0));
                }
            }
        }
    };
    auto put = [&]() {
#pragma unroll
        for (int r = 0; r < NCH; ++r) {
            const int q = tid + r * kThreads;
            if (q < NQ) *reinterpret_cast<uint4 *>(&halo[(q / (C / 8)) * LDH + (q % (C / 8)) * 8]) = rh[r];
        }
    };
    fetch(blockIdx.y * TY * TH);
    put();
    __syncthreads();
    for (int ty = 0; ty < TY; ++ty) {
        const int y0 = (blockIdx.y * TY + ty) * TH;
        if (ty + 1 < TY) fetch(y0 + TH);

        f32x16 acc[FM];
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int e = 0; e < 16; ++e) acc[i][e] = 0.0f;
        if constexpr (C == 8) {
#pragma unroll
            for (int tp = 0; tp < 5; ++tp) {
                const int t = min(2 * tp + (lane >> 5), 8);     // this lane half's tap (the pad reads tap 8)
                const int shift = ((t / 3) * HW + t % 3) * LDH;
                const bf16x8 fb = *reinterpret_cast<const bf16x8 *>(wrow + tp * 16);
#pragma unroll
                for (int i = 0; i < FM; ++i) {
                    const bf16x8 fa = *reinterpret_cast<const bf16x8 *>(&halo[hbase[i] + shift]);
                    acc[i] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa, fb, acc[i], 0, 0, 0);
                }
            }
        } else {
#pragma unroll
            for (int t = 0; t < 9; ++t) {
                const int shift = ((t / 3) * HW + t % 3) * LDH;
#pragma unroll
                for (int kc = 0; kc < C / 16; ++kc) {
                    const bf16x8 fb = *reinterpret_cast<const bf16x8 *>(wrow + t * C + kc * 16);
#pragma unroll
                    for (int i = 0; i < FM; ++i) {
                        const bf16x8 fa = *reinterpret_cast<const bf16x8 *>(&halo[hbase[i] + shift + kc * 16]);
                        acc[i] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa, fb, acc[i], 0, 0, 0);
                    }
                }
            }
        }
        // Elements e and e + 1 of a lane are pixels x and x + 1 of its channel co; lanes co and co ^ 1
        // swap one of them so that each writes both channels of one pixel as a 32-bit word.
        const bool odd = co & 1;
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int e = 0; e < 16; e += 2) {
                float v0 = acc[i][e] + bias, v1 = acc[i][e + 1] + bias;
                if (a.relu) {
                    v0 = fmaxf(v0, 0.0f);
                    v1 = fmaxf(v1, 0.0f);
                }
                const float got = __shfl_xor(odd ? v0 : v1, 1, 64);
                float lo = odd ? got : v0, hi = odd ? v1 : got;      // channels co & ~1 and (co & ~1) + 1
                const int ee = odd ? e + 1 : e;
                const int p = i * 32 + 8 * (ee >> 2) + 4 * (lane >> 5) + (ee & 3);
                const int y = y0 + r0 + p / TW, x = x0 + p % TW;
                const long long d = ((((long long)(b << a.h_log) + y) << a.w_log) + x) * a.ldd + (co & ~1);
                if (a.mask) {
                    const uint32_t m = *reinterpret_cast<const uint32_t *>(a.mask + d);
                    if (!(bf2f(m & 0xffffu) > 0.0f)) lo = 0.0f;
                    if (!(bf2f(m >> 16) > 0.0f)) hi = 0.0f;
                }
                *reinterpret_cast<uint32_t *>(a.dst + d) = (uint32_t)f2bf(lo) | ((uint32_t)f2bf(hi) << 16);
            }
        if (ty + 1 < TY) {
            __syncthreads();   // every wavefront is done with this tile's halo
            put();
            __syncthreads();
        }
    }
}

// 1x1 convolution to a few FP32 channels (the network's head): one lane per pixel reads its C
// bf16 channels (16-byte pieces, all issued before the first is used: with C a run-time bound
// the loads went out one at a time and a wavefront's lines were fetched again between them), the
// weights (bf16 [cout][kpad]) and bias sit in LDS as FP32, sums in FP32.  cout <= kHeadMax,
// C = 8 C8 <= kHeadC.  (Four lanes per pixel, each reading a quarter of it so that a wavefront's
// loads are consecutive, measured slower.)
constexpr int kHeadMax = 8, kHeadC = 64;

template <int C8>
__global__ __launch_bounds__(256) void head_kernel(const uint16_t *in, const uint16_t *w, int kpad,
                                                   const float *bias, int cout, float *out, long long pixels)
{
    constexpr int C = 8 * C8;
    __shared__ float sw[kHeadMax][C];
    __shared__ float sb[kHeadMax];
    for (int i = threadIdx.x; i < cout * C; i += 256) sw[i / C][i % C] = bf2f(w[(size_t)(i / C) * kpad + i % C]);
    for (int i = threadIdx.x; i < cout; i += 256) sb[i] = bias ? bias[i] : 0.0f;
    __syncthreads();
    const long long px = (long long)blockIdx.x * 256 + threadIdx.x;
    if (px >= pixels) return;
    const uint4 *src = reinterpret_cast<const uint4 *>(in + px * C);
    uint4 v[C8];
#pragma unroll
    for (int c8 = 0; c8 < C8; ++c8) v[c8] = src[c8];
    float acc[kHeadMax];
#pragma unroll
    for (int o = 0; o < kHeadMax; ++o) acc[o] = 0.0f;
#pragma unroll
    for (int c8 = 0; c8 < C8; ++c8) {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const float x = bf2f(bf_at(v[c8], e));
#pragma unroll
            for (int o = 0; o < kHeadMax; ++o)
                if (o < cout) acc[o] = fmaf(sw[o][c8 * 8 + e], x, acc[o]);
        }
    }
    float *dst = out + px * cout;
    for (int o = 0; o < cout; ++o) dst[o] = acc[o] + sb[o];
}

}  // namespace unet
