// Line-resident multislice kernels for windows too large for one workgroup
// (N = 256: a 256 x 256 complex window is 512 KB, beyond the LDS and the
// register file of a CU).  A workgroup owns 16 lines of one position; each line
// is held by R = N/16 lanes of one wavefront exactly as in the fused kernel.
//
// The Fresnel propagator factorises over the two axes, so a propagation is a
// row pass and a column pass that commute.  Launch m works in frame m: the
// natural layout for even m (lines are rows), the transposed one for odd m
// (lines are columns).  Every per-position buffer a launch reads is stored in
// its own frame, so each line is one contiguous row of it: the half-propagated
// window A (written by the previous launch), the incident wave psi_m (stored by
// the forward launch of slice m for its adjoint), and for odd slices a
// transposed copy of the slice.  Launch m finishes the propagation of gap m-1
// along its lines, which yields psi_m, applies slice m, starts the propagation
// of gap m along the same lines and stores the result in the other frame for the
// next launch: one global round trip per slice, the store staged through LDS so
// that 16 lines go out as 128-byte pieces.  A alternates between two buffers
// (a launch reads one and writes every row of the other).
#pragma once

#include <hip/hip_runtime.h>

#include "fft_lines.hpp"
#include "ms_kernels.hpp"

namespace imsp {

constexpr int kLinesPerGroup = 16;

enum LineStage : int {
    kStageForward = 0,   // forward launch for slice m
    kStageFar = 1,       // second axis of the far-field FFT, residual (or intensities), first inverse axis
    kStageAdjoint = 2    // adjoint launch for slice m
};

struct LineParams {
    const float2 *class_probe;   // [C][N][N]
    const float2 *slices;        // [M][H][W]
    const float2 *slices_t;      // [M / 2][W][H]: odd slice 2 i + 1 transposed at i
    const int4 *pos_info;        // [S]
    const int *pos_list;         // [count]
    const float2 *tw;            // [R][17]
    const float2 *hy, *hx;       // [U][N] (divided by N)
    const int *gap_table;        // [M-1]
    const float *measured;       // [S][N][N]
    float *intensity;            // [S][N][N] (forward mode)
    float2 *exit_waves;          // [S][N][N] or null
    const float2 *A_in;          // [count][N][N] half-propagated window in this launch's frame
    float2 *A_out;               // [count][N][N] the same for the next launch, in the other frame
    float2 *probe_patch;         // [count][N][N] or null
    double *loss_part;           // [count][N / 16]
    int H, W, M, m;
    int mode;                    // kForward: intensities in the far-field launch; otherwise the residual
    int objective;               // 0 amplitude, 1 Poisson deviance
    // Per-launch destinations, each [count] x stride elements in the launch's frame (null: not
    // used by this launch).  Forward launch of slice m:
    const float2 *restart;       //   psi_m read from here (m > 0) instead of finishing the propagation in A
    long long restart_stride;
    float2 *psi_out;             //   psi_m stored here
    long long psi_out_stride;
    int stop_after_psi;          //   the launch ends once psi_m is stored (recomputing a wave)
    // Forward (layer mode) or adjoint (full-step overlap) launch of slice m:
    float *ovl_out;              //   |psi_m|^2
    long long ovl_stride;
    // Adjoint launch of slice m:
    const float2 *psi_in;        //   psi_m (null: the shifted probe, m = 0)
    long long psi_in_stride;
    float2 *patch_out;           //   dL/d conj(t_m) on the window, conj(psi_m) o g (may alias psi_in)
    long long patch_stride;
    int go_on;                   //   after the patch: conj(t_m), then G_{m-1}^H into A, or the probe patch
};

// Global-memory window access for a line group in either layout: lane (line, j) owns
// along its axis the positions nat(j, k) (SPEC = false) or spec(j, i) (SPEC = true).
template <int N, bool ROW, bool SPEC>
__device__ __forceinline__ void gload(float2 (&v)[16], const float2 *src, int line, int j)
{
    using Wn = Win<N>;
    line = opaque(line);
    j = opaque(j);
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int a = SPEC ? Wn::spec(j, i) : Wn::nat(j, i);
        v[i] = ROW ? src[line * N + a] : src[a * N + line];
    }
}

template <int N, bool ROW, bool SPEC>
__device__ __forceinline__ void gstore(const float2 (&v)[16], float2 *dst, int line, int j)
{
    using Wn = Win<N>;
    line = opaque(line);
    j = opaque(j);
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int a = SPEC ? Wn::spec(j, i) : Wn::nat(j, i);
        if (ROW) dst[line * N + a] = v[i];
        else dst[a * N + line] = v[i];
    }
}

// Column-resident launches move their 16 columns of an image through LDS, so that global
// accesses are rows of 16 consecutive columns (128 contiguous bytes) instead of 32-byte pieces
// of 16 rows per wavefront.  Column c of the tile lives at c * LD (the line's own exchange
// region) with its rows XOR-swizzled by c (the low four bits of the row index; a row stays in
// its block of 16).  The 16 lanes that fill one row then hit 16 distinct bank pairs whatever
// LD mod 16 is, and the lanes of one column read 16 distinct rows mod 16: no bank conflicts at
// N = 64, 128, 256 (with 4 * ((c / 2) mod 4) the fill and drain were 4-way conflicted).
// tile_fill / tile_drain are collective (every lane of the workgroup calls them; they
// synchronise the workgroup).
__device__ __forceinline__ int tile_swz(int c) { return c & 15; }

// Swizzled tile row of the k-th row a lane fills or drains (rows r0 + RP k, RP = R <= 16 rows
// apart): as for tile_idx below, one of 16 / RP per-lane bases plus a multiple of 16 known at
// compile time.
template <int N>
__device__ __forceinline__ int tile_row(int r0, int k, int sw)
{
    constexpr int RP = kLinesPerGroup * Win<N>::R / 16, G = 16 / RP;
    return ((r0 + RP * (k % G)) ^ sw) + 16 * (k / G);
}

template <int N, class F>
__device__ __forceinline__ void tile_fill(float2 *tile, F load)
{
    constexpr int RP = kLinesPerGroup * Win<N>::R / 16;
    const int c = threadIdx.x & 15, r0 = threadIdx.x >> 4, sw = tile_swz(c);
    __syncthreads();
    constexpr int K = N / RP, G = K < 8 ? K : 8;   // G loads in flight before their LDS writes
#pragma unroll
    for (int k0 = 0; k0 < K; k0 += G) {
        float2 buf[G];
#pragma unroll
        for (int k = 0; k < G; ++k) buf[k] = load(r0 + (k0 + k) * RP, c);
#pragma unroll
        for (int k = 0; k < G; ++k) tile[c * Win<N>::LD + tile_row<N>(r0, k0 + k, sw)] = buf[k];
    }
    __syncthreads();
}

template <int N, class F>
__device__ __forceinline__ void tile_drain(const float2 *tile, F store)
{
    constexpr int RP = kLinesPerGroup * Win<N>::R / 16;
    const int c = threadIdx.x & 15, r0 = threadIdx.x >> 4, sw = tile_swz(c);
    __syncthreads();
#pragma unroll 4
    for (int k = 0; k < N / RP; ++k) store(r0 + RP * k, c, tile[c * Win<N>::LD + tile_row<N>(r0, k, sw)]);
    __syncthreads();
}

// Tile index of register i (natural or spectral order) under the swizzle sw.  The swizzle acts
// on the low four bits, which hold the lane's part of the index, so the index is one of 16 / R
// per-lane bases plus a multiple of 16 known at compile time (16 R times a register's index
// would otherwise be 16 addresses kept live).
template <int N, bool SPEC>
__device__ __forceinline__ int tile_idx(int j, int i, int sw)
{
    constexpr int R = Win<N>::R, G = Win<N>::G;
    if (SPEC) return ((j * G + i / R) ^ sw) + 16 * (i % R);
    return ((j + R * (i % G)) ^ sw) + 16 * (i / G);
}

template <int N, bool SPEC>
__device__ __forceinline__ void tile_get(float2 (&v)[16], const float2 *tile, int lloc, int j)
{
    using Wn = Win<N>;
    const float2 *col = tile + lloc * Wn::LD;
    const int sw = tile_swz(lloc);
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = col[tile_idx<N, SPEC>(j, i, sw)];
}

template <int N, bool SPEC>
__device__ __forceinline__ void tile_put(const float2 (&v)[16], float2 *tile, int lloc, int j)
{
    using Wn = Win<N>;
    float2 *col = tile + lloc * Wn::LD;
    const int sw = tile_swz(lloc);
#pragma unroll
    for (int i = 0; i < 16; ++i) col[tile_idx<N, SPEC>(j, i, sw)] = v[i];
}

// Where this lane's line is: (line) for row launches; for column launches also the
// workgroup's first column c0 and the lane's column within the tile, lloc.
struct LinePos {
    int line, lloc, j, c0;
};

template <int N, bool ROW, bool SPEC>
__device__ __forceinline__ void line_load(float2 (&v)[16], const float2 *src, const LinePos &q, float2 *tile)
{
    if (ROW) {
        gload<N, true, SPEC>(v, src, q.line, q.j);
    } else {
        tile_fill<N>(tile, [&](int r, int c) { return src[r * N + q.c0 + c]; });
        tile_get<N, SPEC>(v, tile, q.lloc, q.j);
    }
}

template <int N, bool ROW, bool SPEC>
__device__ __forceinline__ void line_store(const float2 (&v)[16], float2 *dst, const LinePos &q, float2 *tile)
{
    if (ROW) {
        gstore<N, true, SPEC>(v, dst, q.line, q.j);
    } else {
        tile_put<N, SPEC>(v, tile, q.lloc, q.j);
        tile_drain<N>(tile, [&](int r, int c, float2 x) { dst[r * N + q.c0 + c] = x; });
    }
}

// |v|^2 into a float image (SPEC: at spectral positions).
template <int N, bool ROW, bool SPEC>
__device__ __forceinline__ void line_store_abs2(const float2 (&v)[16], float *dst, const LinePos &q, float2 *tile)
{
    using Wn = Win<N>;
    if (ROW) {
        const int l2 = opaque(q.line), j2 = opaque(q.j);
#pragma unroll
        for (int i = 0; i < 16; ++i) dst[l2 * N + (SPEC ? Wn::spec(j2, i) : Wn::nat(j2, i))] = cabs2(v[i]);
    } else {
        float2 a[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) a[i] = make_float2(cabs2(v[i]), 0.0f);
        tile_put<N, SPEC>(a, tile, q.lloc, q.j);
        tile_drain<N>(tile, [&](int r, int c, float2 x) { dst[r * N + q.c0 + c] = x.x; });
    }
}

// Residual at spectral positions against measured intensities (as residual<>, with the
// measured values already in registers); returns this lane's FP64 loss share.
template <int N>
__device__ __forceinline__ double residual_vals(float2 (&v)[16], const float (&mv)[16], int poisson)
{
    double acc = 0.0;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const float m = mv[i];
        const float2 z = v[i];
        const float a2 = cabs2(z);
        const double a2d = (double)z.x * (double)z.x + (double)z.y * (double)z.y;
        if (poisson) {
            if (a2d != 0.0) acc += a2d - (double)m + (m > 0.0f ? (double)m * log((double)m / a2d) : 0.0);
            if (a2 != 0.0f) {
                const float k = m / a2;
                v[i] = make_float2(z.x - k * z.x, z.y - k * z.y);
            }
        } else {
            acc += amp_residual(m, v[i]);
        }
    }
    return acc;
}

template <int N, bool ROW>
__device__ __forceinline__ double line_residual(float2 (&v)[16], const float *meas, const LinePos &q, float2 *tile,
                                                int poisson)
{
    if (ROW) return residual<N, true>(v, meas, q.line, q.j, poisson);
    tile_fill<N>(tile, [&](int r, int c) { return make_float2(meas[r * N + q.c0 + c], 0.0f); });
    float2 t[16];
    tile_get<N, true>(t, tile, q.lloc, q.j);
    float mv[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) mv[i] = t[i].x;
    return residual_vals<N>(v, mv, poisson);
}

// 1D propagation along the owned axis with the factor table h (LDS), or its adjoint.
template <int N, bool CONJ>
__device__ __forceinline__ void prop_axis(float2 (&v)[16], const float2 *tw, float2 *xb, const float2 *h, int j)
{
    using Wn = Win<N>;
    line_fft_fwd<N>(v, tw, xb, j);
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        float2 f = h[Wn::spec(j, i)];
        v[i] = CONJ ? cmulc(v[i], f) : cmul(v[i], f);
    }
    line_fft_inv<N>(v, tw, xb, j);
}

template <int N>
__device__ __forceinline__ double group_sum(double x, double *red)
{
    constexpr int NT = kLinesPerGroup * Win<N>::R;
    constexpr int NW = (NT + 63) / 64;
    for (int off = (NT < 64 ? NT / 2 : 32); off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x / 64] = x;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < NW; ++i) t += red[i];
    return t;
}

// Transmission by slice m (or its conjugate) on this launch's lines, with wrap-around: rows of
// the slice (even m) or of its transposed copy (odd m), whose rows are the slice's columns.
template <int N, bool TR, bool CONJ>
__device__ __forceinline__ void frame_patch(float2 (&v)[16], const LineParams &p, int oy, int ox, int line, int j)
{
    const size_t hw = (size_t)p.H * p.W;
    if (TR) apply_patch<N, true, CONJ>(v, p.slices_t + (size_t)(p.m / 2) * hw, p.W, p.H, ox, oy, line, j);
    else apply_patch<N, true, CONJ>(v, p.slices + (size_t)p.m * hw, p.H, p.W, oy, ox, line, j);
}

// A window in the natural layout from a launch of either frame (SPEC: at spectral positions).
template <int N, bool TR, bool SPEC>
__device__ __forceinline__ void natural_store(const float2 (&v)[16], float2 *dst, const LinePos &q, float2 *tile)
{
    if constexpr (TR) line_store<N, false, SPEC>(v, dst, q, tile);
    else line_store<N, true, SPEC>(v, dst, q, tile);
}

template <int N, bool TR>
// At least 4 waves a SIMD (128 VGPRs): four workgroups a CU, as the LDS allows.
__global__ __launch_bounds__(kLinesPerGroup * Win<N>::R, 4) void line_kernel(LineParams p, int stage)
{
    using Wn = Win<N>;
    constexpr int R = Wn::R;
    constexpr int NT = kLinesPerGroup * R;
    constexpr size_t NN = (size_t)N * N;
    __shared__ float2 xbuf[kLinesPerGroup * Wn::LD];
    __shared__ float2 s_tw[Wn::TW_WORDS];
    __shared__ float2 s_h[N];
    __shared__ double red[(NT + 63) / 64];

    const int tid = threadIdx.x;
    const int lloc = tid / R, j = tid % R;
    const int line = blockIdx.x * kLinesPerGroup + lloc;
    const int b = blockIdx.y;
    const int s = p.pos_list[b];
    const int4 info = p.pos_info[s];
    const int oy = info.x, ox = info.y, cls = info.z;
    const int M = p.M, m = p.m;
    float2 *xb = xbuf + lloc * Wn::LD;
    const float2 *A_in = p.A_in + (size_t)b * NN;
    float2 *A_out = p.A_out + (size_t)b * NN;
    const float2 *probe = p.class_probe + (size_t)cls * NN;
    const float2 *hown = TR ? p.hy : p.hx;

    // tables for this launch: twiddles, and the own-axis factor of the gap that is finished,
    // later replaced by that of the gap that is started (one table of N: with 4 workgroups of
    // this kernel a CU's LDS holds, not 3)
    for (int i = tid; i < Wn::TW_WORDS; i += NT) s_tw[i] = p.tw[i];
    const bool restart = (stage == kStageForward) && p.restart && m > 0;
    int g_fin = -1, g_start = -1;
    if (stage == kStageForward) {
        g_fin = (m > 0 && !restart) ? m - 1 : -1;
        g_start = (m + 1 < M && !p.stop_after_psi) ? m : -1;
    } else if (stage == kStageAdjoint) {
        g_fin = (m + 1 < M) ? m : -1;
        g_start = (m > 0 && p.go_on) ? m - 1 : -1;
    }
    auto load_h = [&](int g) {
        for (int i = tid; i < N; i += NT) s_h[i] = hown[p.gap_table[g] * N + i];
    };
    // before the second propagation of a launch: every lane is done with the first table
    auto next_h = [&]() {
        if (g_fin >= 0) {
            __syncthreads();
            load_h(g_start);
            __syncthreads();
        }
    };
    if (g_fin >= 0) load_h(g_fin);
    else if (g_start >= 0) load_h(g_start);
    __syncthreads();

    const LinePos q{line, lloc, j, (int)blockIdx.x * kLinesPerGroup};
    float2 v[16];
    if (stage == kStageForward) {
        // ---- psi_m: the probe (m = 0, natural frame), a stored wave, or the propagation of gap
        // m-1 finished along this launch's lines ----
        if (m == 0) {
            line_load<N, true, false>(v, probe, q, xbuf);
        } else if (restart) {
            line_load<N, true, false>(v, p.restart + (size_t)b * p.restart_stride, q, xbuf);
        } else {
            line_load<N, true, false>(v, A_in, q, xbuf);
            prop_axis<N, false>(v, s_tw, xb, s_h, j);
        }
        if (p.psi_out) line_store<N, true, false>(v, p.psi_out + (size_t)b * p.psi_out_stride, q, xbuf);
        if (p.ovl_out) line_store_abs2<N, true, false>(v, p.ovl_out + (size_t)b * p.ovl_stride, q, xbuf);
        if (p.stop_after_psi) return;
        frame_patch<N, TR, false>(v, p, oy, ox, line, j);
        if (m + 1 < M) {
            next_h();
            prop_axis<N, false>(v, s_tw, xb, s_h, j);
            line_store<N, false, false>(v, A_out, q, xbuf);    // the next launch's frame
        } else {
            if (p.mode == kForward && p.exit_waves)
                natural_store<N, TR, false>(v, p.exit_waves + (size_t)s * NN, q, xbuf);
            line_fft_fwd<N>(v, s_tw, xb, j);
            line_store<N, false, true>(v, A_out, q, xbuf);     // spectral along these lines, at natural frequency
        }
        return;
    }

    if (stage == kStageFar) {
        // line index = frequency along the other axis (natural); FFT along these lines
        line_load<N, true, false>(v, A_in, q, xbuf);
        line_fft_fwd<N>(v, s_tw, xb, j);
        if (p.mode == kForward) {
            float *I = p.intensity + (size_t)s * NN;
            if constexpr (TR) line_store_abs2<N, false, true>(v, I, q, xbuf);
            else line_store_abs2<N, true, true>(v, I, q, xbuf);
            return;
        }
        const double part = line_residual<N, !TR>(v, p.measured + (size_t)s * NN, q, xbuf, p.objective);
        double tot = group_sum<N>(part, red);
        if (tid == 0) p.loss_part[(size_t)b * gridDim.x + blockIdx.x] = tot;
        line_fft_inv<N>(v, s_tw, xb, j);
        line_store<N, false, false>(v, A_out, q, xbuf);
        return;
    }

    // ---- adjoint launch for slice m ----
    if (m + 1 == M) {
        // finish F^H r along these lines: A holds it at natural frequency positions
        line_load<N, true, true>(v, A_in, q, xbuf);
        line_fft_inv<N>(v, s_tw, xb, j);
    } else {
        line_load<N, true, false>(v, A_in, q, xbuf);
        prop_axis<N, true>(v, s_tw, xb, s_h, j);
    }
    if (p.patch_out) {
        const float2 *psi = p.psi_in ? p.psi_in + (size_t)b * p.psi_in_stride : probe;
        float2 *dst = p.patch_out + (size_t)b * p.patch_stride;
        float *ovl = p.ovl_out ? p.ovl_out + (size_t)b * p.ovl_stride : nullptr;
        // reads before writes in two halves: vector memory operations retire in issue order, so
        // interleaved loads would each wait for the stores before them
        const int l2 = opaque(line), j2 = opaque(j);
#pragma unroll
        for (int h = 0; h < 16; h += 8) {
            float2 ps[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) ps[k] = psi[l2 * N + Wn::nat(j2, h + k)];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int idx = l2 * N + Wn::nat(j2, h + k);
                if (ovl) ovl[idx] = cabs2(ps[k]);
                dst[idx] = cconjmul(ps[k], v[h + k]);
            }
        }
    }
    if (!p.go_on) return;
    frame_patch<N, TR, true>(v, p, oy, ox, line, j);
    if (m > 0) {
        next_h();
        prop_axis<N, true>(v, s_tw, xb, s_h, j);
        line_store<N, false, false>(v, A_out, q, xbuf);
    } else if (p.probe_patch) {
        line_store<N, true, false>(v, p.probe_patch + (size_t)b * NN, q, xbuf);
    }
}

// Odd slices transposed for the line path's odd launches: out[i][x][y] = slices[2 i + 1][y][x]
// (32 x 32 tiles through LDS; grid (W / 32, H / 32, M / 2), 256 lanes).
__global__ __launch_bounds__(256) void transpose_odd_kernel(const float2 *slices, float2 *out, int H, int W)
{
    __shared__ float2 tile[32][33];
    const size_t hw = (size_t)H * W;
    const float2 *src = slices + (size_t)(2 * blockIdx.z + 1) * hw;
    float2 *dst = out + (size_t)blockIdx.z * hw;
    const int x0 = blockIdx.x * 32, y0 = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int r = ty; r < 32; r += 8) {
        const int y = y0 + r, x = x0 + tx;
        if (y < H && x < W) tile[r][tx] = src[(size_t)y * W + x];
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int x = x0 + r, y = y0 + tx;
        if (x < W && y < H) dst[(size_t)x * H + y] = tile[tx][r];
    }
}

// ---- band sums of the adjoint's gradient patches ----
//
// The gradient of slice m (Sec. 3.2) sums, over positions, the patch conj(psi_m) o g placed at the
// window's origin.  Windows of one scan column (one origin x) overlap row for row: a workgroup of an
// even slice's launch that takes 16 object rows, rather than 16 window rows, for every position of
// such a band sums the band's patches on those rows in registers and writes one (N + spread) x N
// band image instead of N x N values per position.  Odd slices do the same in their transposed
// frame: 16 object columns for the windows of one scan row (one origin y).  The scatter then reads
// bands.
//
// Workgroup w takes band lines u0 .. u0 + 15 of band `band`, u counted from the band's first
// origin across the lines; member i (origin delta_i further on) holds them as window lines
// u0 + l - delta_i.  Lines outside the window are computed on a clamped index and neither stored
// nor summed.
struct BandParams {
    const int4 *wg;              // per workgroup: (band, first member, end member, u0)
    const int *mem;              // batch-local position of each member
    const int *delta;            // each member's origin minus the band's first, across the lines
    float2 *band;                // [bands] x band_stride, (N + spread) x N each, in the launch's frame
    long long band_stride;
};

// Adjoint launch of slice m over band workgroups (1D grid); otherwise the adjoint stage of
// line_kernel for each member in turn, with both propagation tables kept in LDS.
template <int N, bool TR>
__global__ __launch_bounds__(kLinesPerGroup * Win<N>::R, 3) void line_band_kernel(LineParams p, BandParams bp)
{
    using Wn = Win<N>;
    constexpr int R = Wn::R;
    constexpr int NT = kLinesPerGroup * R;
    constexpr size_t NN = (size_t)N * N;
    __shared__ float2 xbuf[kLinesPerGroup * Wn::LD];
    __shared__ float2 s_tw[Wn::TW_WORDS];
    __shared__ float2 s_hf[N], s_hs[N];

    const int tid = threadIdx.x;
    const int M = p.M, m = p.m;
    const float2 *hown = TR ? p.hy : p.hx;
    const int g_fin = (m + 1 < M) ? m : -1;
    const int g_start = (m > 0 && p.go_on) ? m - 1 : -1;
    for (int i = tid; i < Wn::TW_WORDS; i += NT) s_tw[i] = p.tw[i];
    if (g_fin >= 0)
        for (int i = tid; i < N; i += NT) s_hf[i] = hown[p.gap_table[g_fin] * N + i];
    if (g_start >= 0)
        for (int i = tid; i < N; i += NT) s_hs[i] = hown[p.gap_table[g_start] * N + i];
    __syncthreads();

    const int4 w = bp.wg[blockIdx.x];
    float2 acc[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) acc[k] = make_float2(0.f, 0.f);
    for (int i = w.y; i < w.z; ++i) {
        // the lane's line and place, hidden from the optimiser each member: the LDS and global
        // addresses derived from them are recomputed where used rather than hoisted out of the
        // loop and kept live
        const int lloc = opaque(tid / R), j = opaque(tid % R);
        float2 *xb = xbuf + lloc * Wn::LD;
        const int b = bp.mem[i];
        const int4 info = p.pos_info[p.pos_list[b]];
        const int l0 = w.w - bp.delta[i];            // window line of lloc = 0
        const int wl = l0 + lloc;
        const bool valid = (unsigned)wl < (unsigned)N;
        const LinePos q{valid ? wl : 0, lloc, j, l0};
        const float2 *A_in = p.A_in + (size_t)b * NN;
        float2 v[16];
        if (m + 1 == M) {
            line_load<N, true, true>(v, A_in, q, xbuf);
            line_fft_inv<N>(v, s_tw, xb, j);
        } else {
            line_load<N, true, false>(v, A_in, q, xbuf);
            prop_axis<N, true>(v, s_tw, xb, s_hf, j);
        }
        if (valid) {
            // acc += conj(psi_m) o g
            const float2 *psi = p.psi_in ? p.psi_in + (size_t)b * p.psi_in_stride
                                         : p.class_probe + (size_t)info.z * NN;
            const int l2 = opaque(q.line), j2 = opaque(j);
#pragma unroll
            for (int k = 0; k < 16; ++k) acc[k] = cadd(acc[k], cconjmul(psi[l2 * N + Wn::nat(j2, k)], v[k]));
        }
        if (!p.go_on) continue;
        frame_patch<N, TR, true>(v, p, info.x, info.y, q.line, j);
        if (m > 0) {
            prop_axis<N, true>(v, s_tw, xb, s_hs, j);
            // into the other frame: window line l0 + c of row r, lines outside the window skipped
            float2 *A_out = p.A_out + (size_t)b * NN;
            tile_put<N, false>(v, xbuf, lloc, j);
            tile_drain<N>(xbuf, [&](int r, int c, float2 x) {
                if ((unsigned)(l0 + c) < (unsigned)N) A_out[r * N + l0 + c] = x;
            });
        } else if (p.probe_patch && valid) {
            gstore<N, true, false>(v, p.probe_patch + (size_t)b * NN, q.line, j);
        }
    }
    float2 *band = bp.band + (size_t)w.x * bp.band_stride;
    const int lloc = tid / R, j = tid % R;
    const int row = w.w + lloc;
#pragma unroll
    for (int k = 0; k < 16; ++k) band[(size_t)row * N + Wn::nat(j, k)] = acc[k];
}

}  // namespace imsp

namespace imsp {

// out[c] = in[c] filtered along one axis: F_a^{-1}(F_a in o t[c]) with t divided by N (CONJ: conj(t)),
// for the sub-pixel probe shift done as a row pass and a column pass.  identity[c] copies.
template <int N, bool ROW, bool CONJ>
__global__ __launch_bounds__(kLinesPerGroup * Win<N>::R) void line_filter_kernel(
    const float2 *in, long long in_stride, float2 *out, const float2 *table, const int *identity, const float2 *twg)
{
    using Wn = Win<N>;
    constexpr int R = Wn::R;
    constexpr int NT = kLinesPerGroup * R;
    constexpr size_t NN = (size_t)N * N;
    __shared__ float2 xbuf[kLinesPerGroup * Wn::LD];
    __shared__ float2 s_tw[Wn::TW_WORDS];
    __shared__ float2 s_h[N];
    const int tid = threadIdx.x;
    const int lloc = tid / R, j = tid % R;
    const int line = blockIdx.x * kLinesPerGroup + lloc;
    const int c = blockIdx.y;
    const float2 *src = in + (size_t)c * in_stride;
    float2 *dst = out + (size_t)c * NN;
    float2 v[16];
    gload<N, ROW, false>(v, src, line, j);
    if (identity[c]) {
        gstore<N, ROW, false>(v, dst, line, j);
        return;
    }
    for (int i = tid; i < Wn::TW_WORDS; i += NT) s_tw[i] = twg[i];
    for (int i = tid; i < N; i += NT) s_h[i] = table[(size_t)c * N + i];
    __syncthreads();
    prop_axis<N, CONJ>(v, s_tw, xbuf + lloc * Wn::LD, s_h, j);
    gstore<N, ROW, false>(v, dst, line, j);
}

// Probe (Sec. 2.1, Fig. 3) for line-resident windows.  Pass 1 (rows): the aperture
// lambda |q| <= alpha times the defocus propagator times (-1)^(ky+kx), inverse DFT along x.
// Pass 2 (columns): inverse DFT along y and FP64 energy partial per line group.
// Pass 3: scale to unit energy.
template <int N, bool ROW>
__global__ __launch_bounds__(kLinesPerGroup * Win<N>::R) void line_probe_kernel(
    float2 *out, double *energy_part, const float2 *twg, double dx, double lambda, double alpha, Aberrations ab)
{
#pragma clang fp contract(off)
    using Wn = Win<N>;
    constexpr int R = Wn::R;
    constexpr int NT = kLinesPerGroup * R;
    __shared__ float2 xbuf[kLinesPerGroup * Wn::LD];
    __shared__ float2 s_tw[Wn::TW_WORDS];
    __shared__ double red[(NT + 63) / 64];
    const int tid = threadIdx.x;
    const int lloc = tid / R, j = tid % R;
    const int line = blockIdx.x * kLinesPerGroup + lloc;
    for (int i = tid; i < Wn::TW_WORDS; i += NT) s_tw[i] = twg[i];
    __syncthreads();
    float2 *xb = xbuf + lloc * Wn::LD;
    float2 v[16];
    if (ROW) {
        const double nd = (double)N * dx;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int iy = line, ix = Wn::spec(j, i);
            const int ky = iy < N / 2 ? iy : iy - N;
            const int kx = ix < N / 2 ? ix : ix - N;
            const double qy = (double)ky / nd, qx = (double)kx / nd;
            const double q2 = qy * qy + qx * qx;
            float2 a = make_float2(0.f, 0.f);
            if (lambda * sqrt(q2) <= alpha) {
                const double ph = -aberration_phase(ab, lambda, qy, qx);
                const double sgn = ((iy + ix) & 1) ? -1.0 : 1.0;
                a = make_float2((float)(sgn * cos(ph)), (float)(sgn * sin(ph)));
            }
            v[i] = a;
        }
        line_fft_inv<N>(v, s_tw, xb, j);
        gstore<N, true, false>(v, out, line, j);
    } else {
        gload<N, false, true>(v, out, line, j);
        line_fft_inv<N>(v, s_tw, xb, j);
        double e = 0.0;
#pragma unroll
        for (int i = 0; i < 16; ++i) e += (double)v[i].x * v[i].x + (double)v[i].y * v[i].y;
        double t = group_sum<N>(e, red);
        if (tid == 0) energy_part[blockIdx.x] = t;
        gstore<N, false, false>(v, out, line, j);
    }
}

// x *= 1 / sqrt(sum of the energy partials), the partials summed in order.
__global__ __launch_bounds__(256) void scale_unit_energy_kernel(float2 *x, long long count, const double *part,
                                                                int n_part)
{
    double e = 0.0;
    for (int i = 0; i < n_part; ++i) e += part[i];
    const float sc = (float)(1.0 / sqrt(e));
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < count; i += (long long)gridDim.x * 256)
        x[i] = make_float2(x[i].x * sc, x[i].y * sc);
}

}  // namespace imsp
