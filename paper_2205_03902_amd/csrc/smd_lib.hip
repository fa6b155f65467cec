// libimsp: sparse matrix decomposition (Algorithm 2) behind the C ABI of include/smd.h.
//
// The matrices are N^2 x N^2 and dense, but every factor between the unknown diagonals is
// G_m = F^-1 diag(h_m) F: a product with G_m is one propagation of each image of the matrix,
// and F is one 2D DFT of each image.  Matrices are stored column-major (the transpose in
// row-major order), so that every such product acts on contiguous images:
//   A^T = O_1 G_1 O_2 ... G_{M-1} O_M   (every factor is symmetric),
//   S^T_{l+1} = S^T_l O_l G_l,   V^T_l = V^T_{l+1} conj(O_{l+1}) conj(G_l)   (V_l = R_l^H X),
// each a right product, i.e. an operation on the rows of the stored array.  The only dense
// products left are the two N^2 x N^2 x S products with the probe matrix in the A estimate
// (LDS-tiled kernels below).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdint>
#include <new>
#include <string>
#include <vector>

#include "fft_lines.hpp"
#include "ms.h"
#include "smd.h"

namespace {

using imsp::Win;

thread_local std::string s_err;

int32_t sfail(int32_t st, const std::string &msg)
{
    s_err = msg;
    return st;
}

constexpr size_t kAlign = 256;
constexpr int kRed = 256;        // reduction partials
constexpr int kTraceBlocks = 2048;   // partials of the lambda traces
constexpr int kDotChunks = 64;   // row chunks of the gradient's column sums

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
unsigned blocks(long long n) { return (unsigned)std::min<long long>(65535, (n + 255) / 256); }

// ---------------------------------------------------------------------------------------
// Image kernels: one workgroup per N x N image (a row of the stored array), the line-FFT
// machinery of the multislice kernels (16 complex values per lane, R = N / 16 lanes a line).

template <int N>
__device__ __forceinline__ void stage_tables(float2 *s_tw, const float2 *twg)
{
    for (int i = threadIdx.x; i < Win<N>::TW_WORDS; i += Win<N>::NT) s_tw[i] = twg[i];
}

// out_b = post o G(pre o in_b) (CONJ: conj(G)), G = F^-1 diag(h_y (x) h_x) F; hy, hx carry the
// 1/N of each inverse transform.  pre, post: N x N multipliers or null; pre_conj conjugates pre.
// in may equal out.
template <int N, bool CONJ>
__global__ __launch_bounds__(Win<N>::NT) void image_propagate_kernel(const float2 *in, float2 *out,
                                                                     const float2 *pre, int pre_conj,
                                                                     const float2 *post, const float2 *hy,
                                                                     const float2 *hx, const float2 *twg)
{
    using Wn = Win<N>;
    constexpr int R = Wn::R;
    __shared__ float2 lds[Wn::LDS_WORDS];
    __shared__ float2 s_tw[Wn::TW_WORDS];
    __shared__ float2 s_h[2 * N];
    const int line = threadIdx.x / R, j = threadIdx.x % R;
    const size_t base = (size_t)blockIdx.x * N * N;
    stage_tables<N>(s_tw, twg);
    for (int i = threadIdx.x; i < N; i += Wn::NT) {
        s_h[i] = hy[i];
        s_h[N + i] = hx[i];
    }
    float2 v[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) {   // rows: lane (y = line, j) holds x = j + R k
        const int x = Wn::nat(j, k);
        float2 a = in[base + (size_t)line * N + x];
        if (pre) {
            const float2 o = pre[line * N + x];
            a = pre_conj ? imsp::cmulc(a, o) : imsp::cmul(a, o);
        }
        v[k] = a;
    }
    __syncthreads();
    float2 *xb = lds + line * Wn::LD;
    imsp::line_fft_fwd<N>(v, s_tw, xb, j);
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const float2 h = s_h[N + Wn::spec(j, i)];
        v[i] = CONJ ? imsp::cmulc(v[i], h) : imsp::cmul(v[i], h);
    }
    imsp::line_fft_inv<N>(v, s_tw, xb, j);
    // columns: lane (x = line, j) holds y = j + R k
    if constexpr (R >= 4) imsp::transpose_nat<N, true>(v, lds, line, j);
    else imsp::transpose<N, true, false, false>(v, lds, line, j);
    imsp::line_fft_fwd<N>(v, s_tw, xb, j);
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const float2 h = s_h[Wn::spec(j, i)];
        v[i] = CONJ ? imsp::cmulc(v[i], h) : imsp::cmul(v[i], h);
    }
    imsp::line_fft_inv<N>(v, s_tw, xb, j);
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const int y = Wn::nat(j, k);
        float2 r = v[k];
        if (post) r = imsp::cmul(r, post[y * N + line]);
        out[base + (size_t)y * N + line] = r;
    }
}

// Unnormalised 2D DFT of every image, natural order in and out: F (INV = false) or
// F^H = N^2 F^-1 (INV = true).
template <int N, bool INV>
__global__ __launch_bounds__(Win<N>::NT) void image_dft_kernel(const float2 *in, float2 *out, const float2 *twg)
{
    using Wn = Win<N>;
    constexpr int R = Wn::R;
    __shared__ float2 lds[Wn::LDS_WORDS];
    __shared__ float2 s_tw[Wn::TW_WORDS];
    const int line = threadIdx.x / R, j = threadIdx.x % R;
    const size_t base = (size_t)blockIdx.x * N * N;
    stage_tables<N>(s_tw, twg);
    float2 v[16];
    float2 *xb = lds + line * Wn::LD;
    if (!INV) {
#pragma unroll
        for (int k = 0; k < 16; ++k) v[k] = in[base + (size_t)line * N + Wn::nat(j, k)];   // rows, natural x
        __syncthreads();
        imsp::line_fft_fwd<N>(v, s_tw, xb, j);                       // x frequencies, spectral order
        imsp::transpose<N, true, true, false>(v, lds, line, j);      // lane (kx = line, j) holds y = j + R k
        imsp::line_fft_fwd<N>(v, s_tw, xb, j);                       // y frequencies, spectral order
#pragma unroll
        for (int i = 0; i < 16; ++i) out[base + (size_t)Wn::spec(j, i) * N + line] = v[i];
    } else {
#pragma unroll
        for (int i = 0; i < 16; ++i) v[i] = in[base + (size_t)Wn::spec(j, i) * N + line];  // lane kx, spectral ky
        __syncthreads();
        imsp::line_fft_inv<N>(v, s_tw, xb, j);                       // natural y
        imsp::transpose<N, false, false, true>(v, lds, line, j);     // lane (y = line, j) holds spectral kx
        imsp::line_fft_inv<N>(v, s_tw, xb, j);                       // natural x
#pragma unroll
        for (int k = 0; k < 16; ++k) out[base + (size_t)line * N + Wn::nat(j, k)] = v[k];
    }
}

// ---------------------------------------------------------------------------------------
// The two products with the probe matrix in the A estimate: N^2 x N^2 by N^2 x S, with S
// small.  Both run on the FP32 matrix cores (v_mfma_f32_32x32x2_f32).  A workgroup of four
// wavefronts owns a 64 x 64 complex output tile, each wavefront a 32 x 32 quarter held as
// real and imaginary accumulators (16 + 16 registers a lane); a complex product is four
// real ones, (ar + i ai)(br + i bi) = (ar br - ai bi) + i (ar bi + ai br).  Operands are
// staged 16 K-rows at a time through LDS.  Matrix-core operand layouts (lane l of 64):
//   A (32 x 2): A[l % 32][l / 32];  B (2 x 32): B[l / 32][l % 32];
//   D (32 x 32), register r: D[8 (r / 4) + 4 (l / 32) + r % 4][l % 32].

constexpr int kTile = 64, kKStep = 16;
typedef float f32x16 __attribute__((ext_vector_type(16)));

// acc_re/acc_im (32 x 32 quarter) += A B over the 16 staged K-rows; sa[r][m] holds A[m][r]
// for this quarter's rows m (64-wide rows, offset m0), sb[r][n] holds B[r][n] (offset n0).
__device__ __forceinline__ void cmfma_16(f32x16 &acc_re, f32x16 &acc_im, const float2 (*sa)[kTile],
                                         const float2 (*sb)[kTile], int m0, int n0, int lane)
{
#pragma unroll
    for (int kk = 0; kk < kKStep; kk += 2) {
        const float2 a = sa[kk + lane / 32][m0 + lane % 32];
        const float2 b = sb[kk + lane / 32][n0 + lane % 32];
        acc_re = __builtin_amdgcn_mfma_f32_32x32x2f32(a.x, b.x, acc_re, 0, 0, 0);
        acc_re = __builtin_amdgcn_mfma_f32_32x32x2f32(-a.y, b.y, acc_re, 0, 0, 0);
        acc_im = __builtin_amdgcn_mfma_f32_32x32x2f32(a.x, b.y, acc_im, 0, 0, 0);
        acc_im = __builtin_amdgcn_mfma_f32_32x32x2f32(a.y, b.x, acc_im, 0, 0, 0);
    }
}

// part[c][s][k] = sum over the rows i of chunk c of P[i][s] At[i][k]   (P: n2 x S, At: n2 x n2).
// Grid (n2 / 64 column tiles, ceil(S / 64) position tiles, chunks); rows chunk c: [c rows, (c+1) rows).
__global__ __launch_bounds__(256) void pt_a_partial_kernel(const float2 *P, const float2 *At, int n2, int S, int rows,
                                                           float2 *part)
{
    __shared__ float2 sP[kKStep][kTile];   // [i][s]
    __shared__ float2 sA[kKStep][kTile];   // [i][k]
    const int t = threadIdx.x, w = t / 64, lane = t % 64;
    const int ms = 32 * (w / 2), nk = 32 * (w % 2);   // this wavefront's quarter (s, k)
    const int k0 = blockIdx.x * kTile, s0 = blockIdx.y * kTile;
    const int i_begin = blockIdx.z * rows, i_end = min(n2, i_begin + rows);
    f32x16 acc_re, acc_im;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc_re[r] = acc_im[r] = 0.f;
    // 16 x 64 of each operand, 4 values a lane; the next rows are loaded into registers
    // while the matrix cores work on the staged ones
    float2 ra[4], rp[4];
    auto fetch = [&](int i0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = t + 256 * q, r = e / kTile, col = e % kTile, i = i0 + r;
            const bool in_i = i < i_end;
            ra[q] = in_i ? At[(size_t)i * n2 + k0 + col] : make_float2(0.f, 0.f);
            rp[q] = (in_i && s0 + col < S) ? P[(size_t)i * S + s0 + col] : make_float2(0.f, 0.f);
        }
    };
    fetch(i_begin);
    for (int i0 = i_begin; i0 < i_end; i0 += kKStep) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = t + 256 * q, r = e / kTile, col = e % kTile;
            sA[r][col] = ra[q];
            sP[r][col] = rp[q];
        }
        __syncthreads();
        if (i0 + kKStep < i_end) fetch(i0 + kKStep);
        cmfma_16(acc_re, acc_im, sP, sA, ms, nk, lane);
        __syncthreads();
    }
    float2 *dst = part + (size_t)blockIdx.z * S * n2;
    const int k = k0 + nk + lane % 32;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int s_ = s0 + ms + 8 * (r / 4) + 4 * (lane / 32) + r % 4;
        if (s_ < S) dst[(size_t)s_ * n2 + k] = make_float2(acc_re[r], acc_im[r]);
    }
}

// Gram matrix g[s][t] = sum_i conj(P[i][s]) P[i][t] (S x S, FP64 sums); grid (ceil(S / 256), S).
__global__ __launch_bounds__(256) void gram_kernel(const float2 *P, int n2, int S, double2 *g)
{
    const int t = blockIdx.x * 256 + threadIdx.x, s = blockIdx.y;
    if (t >= S) return;
    double gr = 0.0, gi = 0.0;
    for (int i = 0; i < n2; ++i) {
        const float2 a = P[(size_t)i * S + s], b = P[(size_t)i * S + t];
        gr += (double)a.x * b.x + (double)a.y * b.y;
        gi += (double)a.x * b.y - (double)a.y * b.x;
    }
    g[(size_t)s * S + t] = make_double2(gr, gi);
}

// Y[e] = sum_c part[c][e] in chunk order.
__global__ void chunk_sum_kernel(const float2 *part, int nch, long long count, float2 *Y)
{
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < count;
         e += (long long)gridDim.x * blockDim.x) {
        float2 a = make_float2(0.f, 0.f);
        for (int c = 0; c < nch; ++c) {
            const float2 v = part[(size_t)c * count + e];
            a.x += v.x;
            a.y += v.y;
        }
        Y[e] = a;
    }
}

// At[i][k] += alpha sum_s Pc[i][s] Y[s][k]   (Pc: n2 x S, Y: S x n2), alpha real.
// Grid (n2 / 64 column tiles, n2 / 64 row tiles).
__global__ __launch_bounds__(256) void rank_update_kernel(float2 *At, const float2 *Pc, const float2 *Y, int n2, int S,
                                                          float alpha)
{
    __shared__ float2 sP[kKStep][kTile];   // [s][i]
    __shared__ float2 sY[kKStep][kTile];   // [s][k]
    const int t = threadIdx.x, w = t / 64, lane = t % 64;
    const int mi = 32 * (w / 2), nk = 32 * (w % 2);   // this wavefront's quarter (i, k)
    const int k0 = blockIdx.x * kTile, i0 = blockIdx.y * kTile;
    const int k = k0 + nk + lane % 32;
    // the updated tile is read up front, so that its latency hides behind the products
    float2 old[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) old[r] = At[(size_t)(i0 + mi + 8 * (r / 4) + 4 * (lane / 32) + r % 4) * n2 + k];
    f32x16 acc_re, acc_im;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc_re[r] = acc_im[r] = 0.f;
    float2 ry[4], rp[4];
    auto fetch = [&](int sb) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = t + 256 * q;
            {   // Y rows sb.., 64 columns
                const int r = e / kTile, col = e % kTile, s_ = sb + r;
                ry[q] = s_ < S ? Y[(size_t)s_ * n2 + k0 + col] : make_float2(0.f, 0.f);
            }
            {   // Pc rows i0.., 16 columns sb..
                const int row = e / kKStep, r = e % kKStep, s_ = sb + r;
                rp[q] = s_ < S ? Pc[(size_t)(i0 + row) * S + s_] : make_float2(0.f, 0.f);
            }
        }
    };
    fetch(0);
    for (int sb = 0; sb < S; sb += kKStep) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = t + 256 * q;
            sY[e / kTile][e % kTile] = ry[q];
            sP[e % kKStep][e / kKStep] = rp[q];   // element (row, s) stored transposed
        }
        __syncthreads();
        if (sb + kKStep < S) fetch(sb + kKStep);
        cmfma_16(acc_re, acc_im, sP, sY, mi, nk, lane);
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const size_t idx = (size_t)(i0 + mi + 8 * (r / 4) + 4 * (lane / 32) + r % 4) * n2 + k;
        At[idx] = make_float2(fmaf(alpha, acc_re[r], old[r].x), fmaf(alpha, acc_im[r], old[r].y));
    }
}

// ---------------------------------------------------------------------------------------
// Element-wise, diagonal and reduction kernels.

// P[i][s] = probe[(y - py) mod n][(x - px) mod n] (i = (y, x)); Pc = conj(P).
__global__ void probe_matrix_kernel(const float2 *probe, const int2 *pos, float2 *P, float2 *Pc, int n, long long S)
{
    const long long n2 = (long long)n * n;
    for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < n2 * S;
         t += (long long)gridDim.x * blockDim.x) {
        const long long i = t / S, s = t - i * S;
        const int y = (int)(i / n), x = (int)(i % n);
        const int2 p = pos[s];
        const int yy = ((y - p.x) % n + n) % n, xx = ((x - p.y) % n + n) % n;
        const float2 v = probe[yy * n + xx];
        P[t] = v;
        Pc[t] = make_float2(v.x, -v.y);
    }
}

// A = diag(scale d) (d null: the identity times scale).
__global__ void set_diag_kernel(float2 *A, const float2 *d, long long n2, float2 scale)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n2 * n2;
         i += (long long)gridDim.x * blockDim.x) {
        const long long r = i / n2, c = i - r * n2;
        float2 v = make_float2(0.f, 0.f);
        if (r == c) {
            const float2 e = d ? d[r] : make_float2(1.f, 0.f);
            v = make_float2(scale.x * e.x - scale.y * e.y, scale.x * e.y + scale.y * e.x);
        }
        A[i] = v;
    }
}

// X = lam A - B (FP64 products, one rounding).
__global__ void axpb_kernel(float2 *X, const float2 *A, const float2 *B, long long count, double lr, double li)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (long long)gridDim.x * blockDim.x) {
        const float2 a = A[i], b = B[i];
        X[i] = make_float2((float)(lr * a.x - li * a.y - b.x), (float)(lr * a.y + li * a.x - b.y));
    }
}

// Amplitude residual of Z^T = (F A P)^T, rows = positions, against I [S][N^2] (same index);
// FP64 loss partials.
__global__ __launch_bounds__(256) void smd_residual_kernel(float2 *Z, const float *I, long long count, double *part)
{
    __shared__ double red[256];
    double acc = 0.0;
    for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < count;
         t += (long long)gridDim.x * blockDim.x) {
        const float2 z = Z[t];
        const float m = I[t];
        const double a = sqrt((double)z.x * z.x + (double)z.y * z.y);
        const double d = sqrt((double)m) - a;
        acc += d * d;
        const float af = (float)a;
        Z[t] = (af == 0.0f) ? make_float2(0.f, 0.f)
                            : make_float2(z.x - sqrtf(m) * (z.x / af), z.y - sqrtf(m) * (z.y / af));
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// out = 1/2 sum of the partials (fixed order).
__global__ void half_sum_kernel(const double *part, int n, double *out)
{
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += part[i];
    *out = 0.5 * s;
}

// part[c][k] = sum over the rows j of chunk c of V[j][k] conj(S[j][k]) (FP64); V = (R^H X)^T and
// S = S_l^T as stored, so that sum_c part[c][k] = diag(R^H X S^H)_k.
__global__ __launch_bounds__(256) void coldot_kernel(const float2 *V, const float2 *S, int n2, int rows, double2 *part)
{
    const int k = blockIdx.x * 256 + threadIdx.x, c = blockIdx.y;
    if (k >= n2) return;
    const int j0 = c * rows, j1 = min(n2, j0 + rows);
    double ar = 0.0, ai = 0.0;
    // eight rows of loads in flight, summed in row order
    constexpr int kU = 8;
    for (int jb = j0; jb < j1; jb += kU) {
        float2 u[kU], w[kU];
#pragma unroll
        for (int q = 0; q < kU; ++q) {
            const bool in = jb + q < j1;
            u[q] = in ? V[(size_t)(jb + q) * n2 + k] : make_float2(0.f, 0.f);
            w[q] = in ? S[(size_t)(jb + q) * n2 + k] : make_float2(0.f, 0.f);
        }
#pragma unroll
        for (int q = 0; q < kU; ++q) {
            ar += (double)u[q].x * w[q].x + (double)u[q].y * w[q].y;
            ai += (double)u[q].y * w[q].x - (double)u[q].x * w[q].y;
        }
    }
    part[(size_t)c * n2 + k] = make_double2(ar, ai);
}

// max |d|^2 of each of M diagonals (one block each).
__global__ __launch_bounds__(256) void peak_kernel(const float2 *d, long long n2, double *peak2)
{
    __shared__ double red[256];
    const float2 *v = d + (long long)blockIdx.x * n2;
    double mx = 0.0;
    for (long long i = threadIdx.x; i < n2; i += 256) mx = fmax(mx, (double)v[i].x * v[i].x + (double)v[i].y * v[i].y);
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) peak2[blockIdx.x] = red[0];
}

// Proximal step of one layer, before the projection: onew[k] = o[k] - conj(lambda) / c grad[k],
// grad[k] = sum_c part[c][k] in chunk order, c = |lambda|^2 prod_{m != l} peak2_m (FP64);
// npart[block] = the block's sum of |onew|^2.
__global__ __launch_bounds__(256) void prox_step_kernel(const float2 *o, const double2 *part, int nparts,
                                                        const double *peak2, int M, int l, double lr, double li, int n2,
                                                        double2 *onew, double *npart)
{
    __shared__ double red[256];
    const int k = blockIdx.x * 256 + threadIdx.x;
    double c = lr * lr + li * li;
    for (int m = 0; m < M; ++m)
        if (m != l) c *= peak2[m];
    const double inv = c > 0.0 ? 1.0 / c : 0.0;
    double a2 = 0.0;
    if (k < n2) {
        double gr = 0.0, gi = 0.0;
        for (int q = 0; q < nparts; ++q) {
            const double2 g = part[(size_t)q * n2 + k];
            gr += g.x;
            gi += g.y;
        }
        const double tr = lr * gr + li * gi, ti = lr * gi - li * gr;   // conj(lambda) grad
        const double nr = (double)o[k].x - inv * tr, ni = (double)o[k].y - inv * ti;
        onew[k] = make_double2(nr, ni);
        a2 = nr * nr + ni * ni;
    }
    red[threadIdx.x] = a2;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) npart[blockIdx.x] = red[0];
}

// The projection: out = onew / ||onew|| (the block sums added in order), rounded once.
__global__ __launch_bounds__(256) void prox_project_kernel(const double2 *onew, const double *npart, int nblocks,
                                                           int n2, float2 *out)
{
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= n2) return;
    double s = 0.0;
    for (int b = 0; b < nblocks; ++b) s += npart[b];
    const double sc = s > 0.0 ? 1.0 / sqrt(s) : 0.0;
    const double2 v = onew[k];
    out[k] = make_float2((float)(v.x * sc), (float)(v.y * sc));
}

// Partials of Tr(At^H Ah) (re, im) and Tr(At^H At).
__global__ __launch_bounds__(256) void trace_kernel(const float2 *At, const float2 *Ah, long long count, double *part)
{
    __shared__ double r0[256], r1[256], r2[256];
    double a = 0.0, b = 0.0, c = 0.0;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (long long)gridDim.x * blockDim.x) {
        const float2 t = At[i], h = Ah[i];
        a += (double)t.x * h.x + (double)t.y * h.y;
        b += (double)t.x * h.y - (double)t.y * h.x;
        c += (double)t.x * t.x + (double)t.y * t.y;
    }
    r0[threadIdx.x] = a;
    r1[threadIdx.x] = b;
    r2[threadIdx.x] = c;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            r0[threadIdx.x] += r0[threadIdx.x + w];
            r1[threadIdx.x] += r1[threadIdx.x + w];
            r2[threadIdx.x] += r2[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[3 * blockIdx.x] = r0[0];
        part[3 * blockIdx.x + 1] = r1[0];
        part[3 * blockIdx.x + 2] = r2[0];
    }
}

// out = s in (complex scalar s, FP64 product).
__global__ void scale_kernel(float2 *out, const float2 *in, long long count, double sr, double si)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (long long)gridDim.x * blockDim.x) {
        const float2 v = in[i];
        out[i] = make_float2((float)(sr * v.x - si * v.y), (float)(sr * v.y + si * v.x));
    }
}

}  // namespace

struct smd_plan {
    int n = 0, n2 = 0, M = 0;
    long long S = 0;
    double dx = 0, lambda = 0;
    std::vector<double> dz;
    std::vector<int> pos;   // (y, x) pairs
    char *ws = nullptr;
    size_t tw, hprop, P, Pc, Y, Z, W, sfx, old, dot, onew, npart, peak, part, ypart, gram, posd, total;
    double mu_a = 0.0;
    bool ready = false;

    template <class T>
    T *at(size_t off) const { return reinterpret_cast<T *>(ws + off); }
    size_t mat() const { return (size_t)n2 * n2; }
    // propagator factors of gap g (h_y then h_x, N each, divided by N)
    const float2 *hy(int g) const { return at<float2>(hprop) + (size_t)g * 2 * n; }
    const float2 *hx(int g) const { return hy(g) + n; }
};

namespace {

// Row chunks of the P^T A^T product (split over K for enough workgroups).
int chunks_of(int n2) { return std::min(16, std::max(1, n2 / 64)); }

void plan_layout(smd_plan &p)
{
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t r = o;
        o = align_up(o + std::max<size_t>(bytes, 1));
        return r;
    };
    const size_t mb = p.mat() * 8, sb = (size_t)p.n2 * p.S * 8;
    p.tw = take((size_t)(p.n / 16) * 17 * 8);
    p.hprop = take((size_t)std::max(p.M - 1, 1) * 2 * p.n * 8);
    p.P = take(sb);
    p.Pc = take(sb);
    p.Y = take(sb);
    p.Z = take(sb);
    p.W = take(mb);
    p.sfx = take(mb * p.M);
    p.old = take((size_t)p.M * p.n2 * 8);
    p.dot = take((size_t)kDotChunks * p.n2 * 16);
    p.onew = take((size_t)p.n2 * 16);
    p.npart = take((size_t)((p.n2 + 255) / 256) * 8);
    p.peak = take((size_t)p.M * 8);
    p.part = take((size_t)std::max(kRed, kTraceBlocks) * 3 * 8);
    p.ypart = take((size_t)chunks_of(p.n2) * p.S * p.n2 * 8);
    p.gram = take((size_t)p.S * p.S * 16);
    p.posd = take((size_t)p.S * 8);
    p.total = o;
}

int32_t check_problem(const smd_problem *pb)
{
    if (!pb) return sfail(MS_ERR_INVALID_ARG, "problem is NULL");
    const int n = pb->n;
    if (n != 16 && n != 32 && n != 64)
        return sfail(MS_ERR_INVALID_ARG, "n must be 16, 32 or 64 (N^2 x N^2 matrices)");
    if (pb->n_slices < 1 || pb->n_slices > 16) return sfail(MS_ERR_INVALID_ARG, "n_slices must be in [1, 16]");
    if (pb->n_pos < 1 || pb->n_pos > (int64_t)n * n) return sfail(MS_ERR_INVALID_ARG, "n_pos must be in [1, N^2]");
    if (!pb->positions || (pb->n_slices > 1 && !pb->dz)) return sfail(MS_ERR_INVALID_ARG, "positions or dz is NULL");
    for (long long s = 0; s < pb->n_pos; ++s)
        for (int c = 0; c < 2; ++c) {
            const double v = pb->positions[2 * s + c];
            if (!std::isfinite(v) || v != std::floor(v) || std::fabs(v) > 1e6)
                return sfail(MS_ERR_INVALID_ARG, "positions must be integer shifts (full-field model)");
        }
    for (int m = 0; m + 1 < pb->n_slices; ++m)
        if (!std::isfinite(pb->dz[m])) return sfail(MS_ERR_INVALID_ARG, "dz must be finite");
    if (!(pb->pixel_size > 0) || !(pb->wavelength > 0)) return sfail(MS_ERR_INVALID_ARG, "need positive dx, lambda");
    return MS_OK;
}

int32_t hip_ok(const char *what)
{
    const hipError_t e = hipGetLastError();
    if (e == hipSuccess) return MS_OK;
    return sfail(MS_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

// Every one of `count` images: out = post o G_g(pre o in) (conj_g: conj(G_g)).
void propagate_rows(smd_plan *p, hipStream_t st, int g, bool conj_g, const float2 *in, float2 *out, long long count,
                    const float2 *pre, bool pre_conj, const float2 *post)
{
    const float2 *hy = p->hy(g), *hx = p->hx(g), *tw = p->at<float2>(p->tw);
    const dim3 grid((unsigned)count);
    const int pc = pre_conj ? 1 : 0;
    switch (p->n) {
        case 16:
            if (conj_g) image_propagate_kernel<16, true><<<grid, Win<16>::NT, 0, st>>>(in, out, pre, pc, post, hy, hx, tw);
            else image_propagate_kernel<16, false><<<grid, Win<16>::NT, 0, st>>>(in, out, pre, pc, post, hy, hx, tw);
            break;
        case 32:
            if (conj_g) image_propagate_kernel<32, true><<<grid, Win<32>::NT, 0, st>>>(in, out, pre, pc, post, hy, hx, tw);
            else image_propagate_kernel<32, false><<<grid, Win<32>::NT, 0, st>>>(in, out, pre, pc, post, hy, hx, tw);
            break;
        default:
            if (conj_g) image_propagate_kernel<64, true><<<grid, Win<64>::NT, 0, st>>>(in, out, pre, pc, post, hy, hx, tw);
            else image_propagate_kernel<64, false><<<grid, Win<64>::NT, 0, st>>>(in, out, pre, pc, post, hy, hx, tw);
            break;
    }
}

// Every one of `count` images: out = F in (inverse: F^H in).
void dft_rows(smd_plan *p, hipStream_t st, bool inverse, const float2 *in, float2 *out, long long count)
{
    const float2 *tw = p->at<float2>(p->tw);
    const dim3 grid((unsigned)count);
    switch (p->n) {
        case 16:
            if (inverse) image_dft_kernel<16, true><<<grid, Win<16>::NT, 0, st>>>(in, out, tw);
            else image_dft_kernel<16, false><<<grid, Win<16>::NT, 0, st>>>(in, out, tw);
            break;
        case 32:
            if (inverse) image_dft_kernel<32, true><<<grid, Win<32>::NT, 0, st>>>(in, out, tw);
            else image_dft_kernel<32, false><<<grid, Win<32>::NT, 0, st>>>(in, out, tw);
            break;
        default:
            if (inverse) image_dft_kernel<64, true><<<grid, Win<64>::NT, 0, st>>>(in, out, tw);
            else image_dft_kernel<64, false><<<grid, Win<64>::NT, 0, st>>>(in, out, tw);
            break;
    }
}

// A^T = scale O_1 G_1 O_2 ... G_{M-1} O_M into `out` (A column-major).
void compose_into(smd_plan *p, hipStream_t st, const float2 *sl, std::complex<float> scale, float2 *out)
{
    const long long n2 = p->n2;
    set_diag_kernel<<<blocks(n2 * n2), 256, 0, st>>>(out, sl, n2, make_float2(scale.real(), scale.imag()));
    for (int g = 0; g + 1 < p->M; ++g)
        propagate_rows(p, st, g, false, out, out, n2, nullptr, false, sl + (size_t)(g + 1) * n2);
}

}  // namespace

extern "C" {

int32_t smd_workspace_size(const smd_problem *pb, size_t *ws_bytes)
{
    int32_t s = check_problem(pb);
    if (s != MS_OK) return s;
    if (!ws_bytes) return sfail(MS_ERR_INVALID_ARG, "ws_bytes is NULL");
    smd_plan p;
    p.n = pb->n;
    p.n2 = pb->n * pb->n;
    p.M = pb->n_slices;
    p.S = pb->n_pos;
    plan_layout(p);
    *ws_bytes = p.total;
    return MS_OK;
}

int32_t smd_plan_create(const smd_problem *pb, void *workspace, size_t ws_bytes, smd_plan **out)
{
    int32_t s = check_problem(pb);
    if (s != MS_OK) return s;
    if (!out || !workspace || (reinterpret_cast<uintptr_t>(workspace) % kAlign))
        return sfail(MS_ERR_INVALID_ARG, "out or a 256-byte aligned workspace missing");
    smd_plan *p = new (std::nothrow) smd_plan;
    if (!p) return sfail(MS_ERR_INVALID_ARG, "out of host memory");
    p->n = pb->n;
    p->n2 = pb->n * pb->n;
    p->M = pb->n_slices;
    p->S = pb->n_pos;
    p->dx = pb->pixel_size;
    p->lambda = pb->wavelength;
    if (p->M > 1) p->dz.assign(pb->dz, pb->dz + (p->M - 1));
    for (long long i = 0; i < p->S; ++i) {
        p->pos.push_back((int)pb->positions[2 * i]);
        p->pos.push_back((int)pb->positions[2 * i + 1]);
    }
    plan_layout(*p);
    if (ws_bytes < p->total) {
        const size_t need = p->total;
        delete p;
        return sfail(MS_ERR_BUDGET, "workspace too small: " + std::to_string(need) + " bytes needed");
    }
    p->ws = static_cast<char *>(workspace);
    // twiddles W_N^{j k1} of lane j (rows of 17) and the propagator of eq. (fresnel_element)
    // split per axis, exp(-i pi dz lambda q^2) / N, in FP64 rounded once
    const int n = p->n, R = n / 16;
    const double PI = 3.14159265358979323846264338327950288;
    std::vector<float2> tw((size_t)R * 17, make_float2(1.f, 0.f));
    for (int j = 0; j < R; ++j)
        for (int k1 = 0; k1 < 16; ++k1) {
            const double a = -2.0 * PI * (double)(j * k1) / n;
            tw[(size_t)j * 17 + k1] = make_float2((float)std::cos(a), (float)std::sin(a));
        }
    std::vector<float2> hp((size_t)std::max(p->M - 1, 1) * 2 * n, make_float2(0.f, 0.f));
    for (int g = 0; g + 1 < p->M; ++g)
        for (int i = 0; i < n; ++i) {
            const double q = (double)(i < (n + 1) / 2 ? i : i - n) / ((double)n * p->dx);
            const double ph = -PI * p->dz[g] * p->lambda * q * q;
            const float2 h = make_float2((float)(std::cos(ph) / n), (float)(std::sin(ph) / n));
            hp[(size_t)g * 2 * n + i] = h;        // h_y
            hp[(size_t)g * 2 * n + n + i] = h;    // h_x
        }
    if (hipMemcpy(p->at<char>(p->tw), tw.data(), tw.size() * 8, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(p->at<char>(p->hprop), hp.data(), hp.size() * 8, hipMemcpyHostToDevice) != hipSuccess) {
        delete p;
        return sfail(MS_ERR_HIP, "table upload failed");
    }
    *out = p;
    return MS_OK;
}

void smd_plan_destroy(smd_plan *p)
{
    delete p;
}

int32_t smd_set_probe(smd_plan *p, hipStream_t st, const void *probe)
{
    if (!p || !probe) return sfail(MS_ERR_INVALID_ARG, "NULL argument");
    const long long n2 = p->n2, S = p->S;
    if (hipMemcpyAsync(p->at<int2>(p->posd), p->pos.data(), (size_t)S * 8, hipMemcpyHostToDevice, st) != hipSuccess)
        return sfail(MS_ERR_HIP, "position upload failed");
    float2 *P = p->at<float2>(p->P);
    probe_matrix_kernel<<<blocks(n2 * S), 256, 0, st>>>(static_cast<const float2 *>(probe), p->at<int2>(p->posd), P,
                                                          p->at<float2>(p->Pc), p->n, S);
    // Gram matrix P^H P (S x S, S <= N^2)
    double2 *gram = p->at<double2>(p->gram);
    gram_kernel<<<dim3((unsigned)((S + 255) / 256), (unsigned)S), 256, 0, st>>>(P, p->n2, (int)S, gram);
    std::vector<std::complex<double>> g((size_t)S * S);
    if (hipMemcpyAsync(g.data(), gram, g.size() * 16, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return sfail(MS_ERR_HIP, "Gram matrix download failed");
    // largest eigenvalue of the Hermitian PSD Gram matrix: power iteration with Rayleigh quotients.
    // The start has golden-ratio phases: on a regular grid of shifts the Gram matrix is
    // circulant, its eigenvectors are Fourier modes, and the constant vector is one of them
    // (a power iteration started there never leaves it).
    std::vector<std::complex<double>> v((size_t)S), w((size_t)S);
    for (long long i = 0; i < S; ++i) {
        const double frac = std::fmod(0.6180339887498949 * (double)(i + 1), 1.0);
        v[i] = std::polar(1.0, 6.283185307179586 * frac);
    }
    double ev = 0.0;
    for (int it = 0; it < 5000; ++it) {
        double nrm = 0.0;
        for (long long i = 0; i < S; ++i) nrm += std::norm(v[i]);
        nrm = std::sqrt(nrm);
        for (auto &x : v) x /= nrm;
        for (long long i = 0; i < S; ++i) {
            std::complex<double> acc = 0.0;
            for (long long j = 0; j < S; ++j) acc += g[(size_t)i * S + j] * v[j];
            w[i] = acc;
        }
        double rq = 0.0;
        for (long long i = 0; i < S; ++i) rq += (std::conj(v[i]) * w[i]).real();
        // the Rayleigh quotient's error is quadratic in the eigenvector's: 1e-12 is far below FP32
        const bool done = it > 10 && std::fabs(rq - ev) <= 1e-12 * rq;
        ev = rq;
        v.swap(w);
        if (done) break;
    }
    p->mu_a = ev > 0.0 ? 1.0 / ((double)n2 * ev) : 0.0;
    p->ready = true;
    return hip_ok("smd_set_probe");
}

int32_t smd_compose(smd_plan *p, hipStream_t st, const void *slices, const double *lambda, void *a_out)
{
    if (!p || !slices || !lambda || !a_out) return sfail(MS_ERR_INVALID_ARG, "NULL argument");
    if (!p->ready) return sfail(MS_ERR_INVALID_ARG, "call smd_set_probe first");
    compose_into(p, st, static_cast<const float2 *>(slices), std::complex<float>((float)lambda[0], (float)lambda[1]),
                 static_cast<float2 *>(a_out));
    return hip_ok("smd_compose");
}

int32_t smd_estimate(smd_plan *p, hipStream_t st, const float *measured, void *a, int32_t steps, double *loss_first)
{
    if (!p || !measured || !a) return sfail(MS_ERR_INVALID_ARG, "NULL argument");
    if (!p->ready) return sfail(MS_ERR_INVALID_ARG, "call smd_set_probe first");
    if (steps < 0) return sfail(MS_ERR_INVALID_ARG, "steps must be >= 0");
    const int n2 = p->n2, S = (int)p->S;
    float2 *At = static_cast<float2 *>(a), *P = p->at<float2>(p->P), *Pc = p->at<float2>(p->Pc);
    float2 *Y = p->at<float2>(p->Y), *Z = p->at<float2>(p->Z);
    double *part = p->at<double>(p->part);
    const int nch = chunks_of(n2), rows = n2 / nch;
    float2 *ypart = p->at<float2>(p->ypart);
    for (int k = 0; k < steps; ++k) {
        // (A P)^T = P^T A^T, then the DFT of each position's image: Z^T = (F A P)^T
        pt_a_partial_kernel<<<dim3(n2 / kTile, (S + kTile - 1) / kTile, nch), 256, 0, st>>>(P, At, n2, S, rows, ypart);
        chunk_sum_kernel<<<blocks((long long)S * n2), 256, 0, st>>>(ypart, nch, (long long)S * n2, Y);
        dft_rows(p, st, false, Y, Z, S);
        smd_residual_kernel<<<kRed, 256, 0, st>>>(Z, measured, (long long)S * n2, part);
        if (k == 0 && loss_first) half_sum_kernel<<<1, 1, 0, st>>>(part, kRed, loss_first);
        dft_rows(p, st, true, Z, Y, S);   // (F^H r)^T
        // A^T -= mu (F^H r P^H)^T = mu conj(P) (F^H r)^T
        rank_update_kernel<<<dim3(n2 / kTile, n2 / kTile), 256, 0, st>>>(At, Pc, Y, n2, S, (float)-p->mu_a);
    }
    return hip_ok("smd_estimate");
}

int32_t smd_decompose(smd_plan *p, hipStream_t st, const void *a_hat, void *slices, double *lambda, void *a_tilde_out)
{
    if (!p || !a_hat || !slices || !lambda) return sfail(MS_ERR_INVALID_ARG, "NULL argument");
    if (!p->ready) return sfail(MS_ERR_INVALID_ARG, "call smd_set_probe first");
    const int n2 = p->n2, M = p->M;
    const long long nn = (long long)n2 * n2;
    const float2 *Ah = static_cast<const float2 *>(a_hat);
    float2 *sl = static_cast<float2 *>(slices);
    float2 *old = p->at<float2>(p->old), *W = p->at<float2>(p->W), *sfx = p->at<float2>(p->sfx);
    double2 *dot = p->at<double2>(p->dot);
    if (hipMemcpyAsync(old, sl, (size_t)M * n2 * 8, hipMemcpyDeviceToDevice, st) != hipSuccess)
        return sfail(MS_ERR_HIP, "slice copy failed");
    peak_kernel<<<M, 256, 0, st>>>(old, n2, p->at<double>(p->peak));
    // X^T = lambda A^T(old slices) - A_hat^T: for every layer R_l O_l S_l is the whole matrix
    compose_into(p, st, old, 1.0f, W);
    axpb_kernel<<<blocks(nn), 256, 0, st>>>(W, W, Ah, nn, lambda[0], lambda[1]);
    // suffixes S_l^T: S_0 = I, S^T_{l+1} = S^T_l O_l G_l
    set_diag_kernel<<<blocks(nn), 256, 0, st>>>(sfx, nullptr, n2, make_float2(1.f, 0.f));
    for (int l = 0; l + 1 < M; ++l)
        propagate_rows(p, st, l, false, sfx + (size_t)l * nn, sfx + (size_t)(l + 1) * nn, n2, old + (size_t)l * n2,
                       false, nullptr);
    // layers from the last: W holds V_l^T = (R_l^H X)^T, V_{M-1} = X
    const int rows = (n2 + kDotChunks - 1) / kDotChunks;
    for (int l = M - 1; l >= 0; --l) {
        coldot_kernel<<<dim3((n2 + 255) / 256, kDotChunks), 256, 0, st>>>(W, sfx + (size_t)l * nn, n2, rows, dot);
        const int nb = (n2 + 255) / 256;
        prox_step_kernel<<<nb, 256, 0, st>>>(old + (size_t)l * n2, dot, kDotChunks, p->at<double>(p->peak), M, l,
                                             lambda[0], lambda[1], n2, p->at<double2>(p->onew), p->at<double>(p->npart));
        prox_project_kernel<<<nb, 256, 0, st>>>(p->at<double2>(p->onew), p->at<double>(p->npart), nb, n2,
                                                sl + (size_t)l * n2);
        if (l > 0)   // V^T_{l-1} = V^T_l conj(O_l) conj(G_{l-1})
            propagate_rows(p, st, l - 1, true, W, W, n2, old + (size_t)l * n2, true, nullptr);
    }
    float2 *At = a_tilde_out ? static_cast<float2 *>(a_tilde_out) : W;
    compose_into(p, st, sl, 1.0f, At);
    double *part = p->at<double>(p->part);
    trace_kernel<<<kTraceBlocks, 256, 0, st>>>(At, Ah, nn, part);
    std::vector<double> h((size_t)kTraceBlocks * 3);
    if (hipMemcpyAsync(h.data(), part, h.size() * 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return sfail(MS_ERR_HIP, "trace download failed");
    double tr = 0.0, ti = 0.0, tt = 0.0;
    for (int i = 0; i < kTraceBlocks; ++i) {
        tr += h[3 * i];
        ti += h[3 * i + 1];
        tt += h[3 * i + 2];
    }
    if (tt > 0.0) {
        lambda[0] = tr / tt;
        lambda[1] = ti / tt;
    }
    return hip_ok("smd_decompose");
}

int32_t smd_result(smd_plan *p, hipStream_t st, const void *slices, const double *lambda, void *out)
{
    if (!p || !slices || !lambda || !out) return sfail(MS_ERR_INVALID_ARG, "NULL argument");
    const std::complex<double> root = std::pow(std::complex<double>(lambda[0], lambda[1]), 1.0 / p->M);
    const long long count = (long long)p->M * p->n2;
    scale_kernel<<<blocks(count), 256, 0, st>>>(static_cast<float2 *>(out), static_cast<const float2 *>(slices), count,
                                                root.real(), root.imag());
    return hip_ok("smd_result");
}

const char *smd_last_error(void) { return s_err.c_str(); }

}  // extern "C"
