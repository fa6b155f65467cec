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
// lines of a wavefront in a line workgroup of window side N (R = N / 16 lanes a line)
template <int N>
constexpr int lines_per_wave() { return (kLinesPerGroup * (N / 16) < 64 ? kLinesPerGroup * (N / 16) : 64) / (N / 16); }

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
    const float2 *A_in;          // [count][N][N + 16] half-propagated window in this launch's frame
    float2 *A_out;               // [count][N][N + 16] the same for the next launch, in the other frame
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
    // Layout of A (see Apitch): with offsets, lines in groups aligned in object coordinates
    int obj_in, obj_out;         //   A_in / A_out with the per-position offsets
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

// Transmission of slice m on this launch's lines, with wrap-around: rows of the slice (even m) or
// of its transposed copy (odd m), whose rows are the slice's columns.  A window inside the object
// (no index wraps; the same for every lane of a position) takes the loads at a per-lane base plus
// constant steps.
template <int N, bool TR>
__device__ __forceinline__ void frame_load(float2 (&t)[16], const LineParams &p, int oy, int ox, int line, int j)
{
    const size_t hw = (size_t)p.H * p.W;
    const bool inside = oy + N <= p.H && ox + N <= p.W;
    if (TR) load_patch<N, true>(t, p.slices_t + (size_t)(p.m / 2) * hw, p.W, p.H, ox, oy, line, j, inside);
    else load_patch<N, true>(t, p.slices + (size_t)p.m * hw, p.H, p.W, oy, ox, line, j, inside);
}

// v *= the transmission (or its conjugate).
template <int N, bool TR, bool CONJ>
__device__ __forceinline__ void frame_patch(float2 (&v)[16], const LineParams &p, int oy, int ox, int line, int j)
{
    float2 t[16];
    frame_load<N, TR>(t, p, oy, ox, line, j);
    mul_patch<CONJ>(v, t);
}

// ---- the half-propagated windows A ----
//
// A window written for a launch of frame F holds its line l (N lines) in a row of N + 16 elements,
// element a at column a + s.  Two layouts: s = 0 with each launch's 16 lines a group aligned in
// the window (the forward chain: every read and write aligned), or s = the position's origin
// along F's elements (x for frame 0, y for frame 1) modulo 16 with each launch's 16 lines a group
// aligned in object coordinates (its first line l0 has l0 + its line-axis origin = 0 modulo 16;
// a window then takes N / 16 + 1 groups, the outer two partly outside it).  The second is what
// band workgroups need (their members' lines are aligned in object coordinates, not in each
// window), and its transposed stores still write whole aligned 128-byte pieces; its reads start
// at s.  Launches always have N / 16 + 1 groups; with s = 0 the last one exits at once.
template <int N>
struct Apitch {
    static constexpr int P = N + 16;
};

// Line `line` of A in this launch's frame, natural (SPEC: spectral) register order.
template <int N, bool SPEC>
__device__ __forceinline__ void aload(float2 (&v)[16], const float2 *src, int line, int j, int s)
{
    using Wn = Win<N>;
    line = opaque(line);
    j = opaque(j);
    const float2 *row = src + line * Apitch<N>::P + s;
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = row[SPEC ? Wn::spec(j, i) : Wn::nat(j, i)];
}

// The workgroup's lines l0 .. l0 + 15 into the other frame through the LDS tile: element a of line
// l0 + c to dst[a * pitch + l0 + c + s]; lines outside the window skipped.  Collective.
template <int N, bool SPEC>
__device__ __forceinline__ void store_other(const float2 (&v)[16], float2 *dst, int pitch, int l0, int s, int lloc,
                                            int j, float2 *tile)
{
    tile_put<N, SPEC>(v, tile, lloc, j);
    tile_drain<N>(tile, [&](int r, int c, float2 x) {
        if ((unsigned)(l0 + c) < (unsigned)N) dst[(size_t)r * pitch + l0 + c + s] = x;
    });
}

// |v|^2 of the workgroup's lines into a natural-layout float image from a transposed launch
// (SPEC: at spectral positions).  Collective.
template <int N, bool SPEC>
__device__ __forceinline__ void store_other_abs2(const float2 (&v)[16], float *dst, int l0, int lloc, int j,
                                                 float2 *tile)
{
    float2 a[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) a[i] = make_float2(cabs2(v[i]), 0.0f);
    tile_put<N, SPEC>(a, tile, lloc, j);
    tile_drain<N>(tile, [&](int r, int c, float2 x) {
        if ((unsigned)(l0 + c) < (unsigned)N) dst[(size_t)r * N + l0 + c] = x.x;
    });
}

template <int N, bool TR>
// At least 4 waves a SIMD (128 VGPRs): four workgroups a CU, as the LDS allows.
__global__ __launch_bounds__(kLinesPerGroup * Win<N>::R, 4) void line_kernel(LineParams p, int stage)
{
    using Wn = Win<N>;
    constexpr int R = Wn::R;
    constexpr int NT = kLinesPerGroup * R;
    constexpr size_t NN = (size_t)N * N;
    constexpr size_t NA = (size_t)N * Apitch<N>::P;
    __shared__ float2 xbuf[kLinesPerGroup * Wn::LD];
    __shared__ float2 s_tw[Wn::TW_WORDS];
    __shared__ float2 s_h[N];
    __shared__ double red[(NT + 63) / 64];

    const int tid = threadIdx.x;
    const int lloc = tid / R, j = tid % R;
    const int b = blockIdx.y;
    const int s = p.pos_list[b];
    const int4 info = p.pos_info[s];
    const int oy = info.x, ox = info.y, cls = info.z;
    // offsets of A_in (the element-axis origin modulo 16) and A_out (the line-axis origin); this
    // group's first line
    const int s_line = p.obj_out ? (TR ? ox : oy) & 15 : 0, s_elem = p.obj_in ? (TR ? oy : ox) & 15 : 0;
    const int l0 = (int)blockIdx.x * kLinesPerGroup - s_line;
    if (l0 >= N) {                             // the extra group of an aligned window
        if (stage == kStageFar && p.mode != kForward && tid == 0)
            p.loss_part[(size_t)b * gridDim.x + blockIdx.x] = 0.0;
        return;
    }
    const int line_raw = l0 + lloc;
    const bool valid = (unsigned)line_raw < (unsigned)N;
    const int line = valid ? line_raw : 0;
    const int M = p.M, m = p.m;
    float2 *xb = xbuf + lloc * Wn::LD;
    const float2 *A_in = p.A_in + (size_t)b * NA;
    float2 *A_out = p.A_out + (size_t)b * NA;
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

    float2 v[16];
    if (stage == kStageForward) {
        // the transmission of slice m on these lines, loaded before the propagation that it
        // follows so that the loads' latency passes during it
        float2 tv[16];
        if (!p.stop_after_psi) frame_load<N, TR>(tv, p, oy, ox, line, j);
        // ---- psi_m: the probe (m = 0, natural frame), a stored wave, or the propagation of gap
        // m-1 finished along this launch's lines ----
        if (m == 0) {
            gload<N, true, false>(v, probe, line, j);
        } else if (restart) {
            gload<N, true, false>(v, p.restart + (size_t)b * p.restart_stride, line, j);
        } else {
            aload<N, false>(v, A_in, line, j, s_elem);
            prop_axis<N, false>(v, s_tw, xb, s_h, j);
        }
        if (valid && p.psi_out) gstore<N, true, false>(v, p.psi_out + (size_t)b * p.psi_out_stride, line, j);
        if (valid && p.ovl_out) {
            float *o = p.ovl_out + (size_t)b * p.ovl_stride;
            const int l2 = opaque(line), j2 = opaque(j);
#pragma unroll
            for (int i = 0; i < 16; ++i) o[l2 * N + Wn::nat(j2, i)] = cabs2(v[i]);
        }
        if (p.stop_after_psi) return;
        mul_patch<false>(v, tv);
        if (m + 1 < M) {
            next_h();
            prop_axis<N, false>(v, s_tw, xb, s_h, j);
            store_other<N, false>(v, A_out, Apitch<N>::P, l0, s_line, lloc, j, xbuf);
        } else {
            if (p.mode == kForward && p.exit_waves) {
                float2 *ew = p.exit_waves + (size_t)s * NN;
                if constexpr (TR) store_other<N, false>(v, ew, N, l0, 0, lloc, j, xbuf);
                else if (valid) gstore<N, true, false>(v, ew, line, j);
            }
            line_fft_fwd<N>(v, s_tw, xb, j);
            store_other<N, true>(v, A_out, Apitch<N>::P, l0, s_line, lloc, j, xbuf);   // spectral, natural frequency
        }
        return;
    }

    if (stage == kStageFar) {
        // line index = frequency along the other axis (natural); FFT along these lines.  The
        // measured values of the line are loaded first, so that their latency passes during the
        // FFT (whose wavefront fences keep the compiler from moving loads across it).
        aload<N, false>(v, A_in, line, j, s_elem);
        const float *meas = p.measured + (size_t)s * NN;
        float mv[16];
        if (p.mode != kForward) {
            if constexpr (TR) {
                // the measured column of this line through the tile (lines outside read a clamped
                // one); each line's values come back from its own exchange slot, which its
                // wavefront's FFT then reuses
                tile_fill<N>(xbuf, [&](int r, int c) {
                    const int cc = min(max(l0 + c, 0), N - 1);
                    return make_float2(meas[r * N + cc], 0.0f);
                });
                float2 t[16];
                tile_get<N, true>(t, xbuf, lloc, j);
#pragma unroll
                for (int i = 0; i < 16; ++i) mv[i] = t[i].x;
            } else {
                const int l2 = opaque(line), j2 = opaque(j);
#pragma unroll
                for (int i = 0; i < 16; ++i) mv[i] = meas[l2 * N + Wn::spec(j2, i)];
            }
        }
        line_fft_fwd<N>(v, s_tw, xb, j);
        if (p.mode == kForward) {
            float *I = p.intensity + (size_t)s * NN;
            if constexpr (TR) {
                store_other_abs2<N, true>(v, I, l0, lloc, j, xbuf);
            } else if (valid) {
                const int l2 = opaque(line), j2 = opaque(j);
#pragma unroll
                for (int i = 0; i < 16; ++i) I[l2 * N + Wn::spec(j2, i)] = cabs2(v[i]);
            }
            return;
        }
        const double part = residual_vals<N>(v, mv, p.objective);
        double tot = group_sum<N>(valid ? part : 0.0, red);
        if (tid == 0) p.loss_part[(size_t)b * gridDim.x + blockIdx.x] = tot;
        line_fft_inv<N>(v, s_tw, xb, j);
        store_other<N, false>(v, A_out, Apitch<N>::P, l0, s_line, lloc, j, xbuf);
        return;
    }

    // ---- adjoint launch for slice m ----
    if (m + 1 == M) {
        // finish F^H r along these lines: A holds it at natural frequency positions
        aload<N, true>(v, A_in, line, j, s_elem);
        line_fft_inv<N>(v, s_tw, xb, j);
    } else {
        aload<N, false>(v, A_in, line, j, s_elem);
        prop_axis<N, true>(v, s_tw, xb, s_h, j);
    }
    if (p.patch_out && valid) {
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
        store_other<N, false>(v, A_out, Apitch<N>::P, l0, s_line, lloc, j, xbuf);
    } else if (p.probe_patch && valid) {
        gstore<N, true, false>(v, p.probe_patch + (size_t)b * NN, line, j);
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
// origin across the lines and u0 + that origin = 0 modulo 16 (so u0 may be negative); member i
// (origin delta_i further on) holds them as window lines u0 + l - delta_i, an aligned group as in
// line_kernel.  Lines outside the window are computed on a clamped index and neither stored nor
// summed.
struct BandParams {
    const int4 *wg;              // per workgroup: (band, first member, end member, u0)
    const int *mem;              // batch-local position of each member
    const int *delta;            // each member's origin minus the band's first, across the lines
    float2 *band;                // [bands] x band_stride: rows x N each, in the launch's frame
    long long band_stride;
    int rows;                    // band image rows
};

// Adjoint launch of slice m over band workgroups (1D grid); otherwise the adjoint stage of
// line_kernel for each member in turn (A_out with offsets; A_in with or without, the first
// adjoint launch reading the far field's aligned windows).
//
// psi_m comes from psi_in as a stored wave, or (RECOMP, m > 0) as the window the forward launch
// of slice m read: rows of N + 16 aligned, in this launch's frame, from which psi_m is the
// propagation of gap m - 1 finished along the lines, as that launch did.  A forward chain that
// keeps those windows then stores no waves: it writes each window once, where the ping-pong
// would have overwritten it, and the adjoint reads it in place of the wave.
//
// Without RECOMP one propagation table in LDS, reloaded between the two propagations of a member,
// so that a CU holds four workgroups; with it the recomputed wave is a third window line in
// registers, three workgroups a CU fit, and both tables stay in LDS.
template <int N, bool TR, bool RECOMP>
__global__ __launch_bounds__(kLinesPerGroup * Win<N>::R, RECOMP ? 3 : 4) void line_band_kernel(LineParams p,
                                                                                              BandParams bp)
{
    using Wn = Win<N>;
    constexpr int R = Wn::R;
    constexpr int NT = kLinesPerGroup * R;
    constexpr size_t NN = (size_t)N * N;
    constexpr size_t NA = (size_t)N * Apitch<N>::P;
    __shared__ float2 xbuf[kLinesPerGroup * Wn::LD];
    __shared__ float2 s_tw[Wn::TW_WORDS];
    __shared__ float2 s_h[RECOMP ? 2 * N : N];

    const int tid = threadIdx.x;
    const int M = p.M, m = p.m;
    const float2 *hown = TR ? p.hy : p.hx;
    const int g_fin = (m + 1 < M) ? m : -1;
    const int g_start = (m > 0 && (p.go_on || RECOMP)) ? m - 1 : -1;
    // the tables of gaps m (finished here) and m - 1 (started here; finished by the forward
    // launch): one slot, filled on demand between barriers (every lane is done with the previous
    // table; slices of one distance share a table), or with RECOMP a slot each, filled once
    float2 *h_fin = s_h, *h_start = RECOMP ? s_h + N : s_h;
    int loaded = -1;
    auto load_h = [&](int g) {
        if (RECOMP) return;
        const int u = p.gap_table[g];
        if (u == loaded) return;
        __syncthreads();
        for (int i = tid; i < N; i += NT) s_h[i] = hown[u * N + i];
        __syncthreads();
        loaded = u;
    };
    for (int i = tid; i < Wn::TW_WORDS; i += NT) s_tw[i] = p.tw[i];
    if (RECOMP) {
        if (g_fin >= 0)
            for (int i = tid; i < N; i += NT) h_fin[i] = hown[p.gap_table[g_fin] * N + i];
        if (g_start >= 0)
            for (int i = tid; i < N; i += NT) h_start[i] = hown[p.gap_table[g_start] * N + i];
    }
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
        const int s_line = (TR ? info.y : info.x) & 15, s_elem = p.obj_in ? (TR ? info.x : info.y) & 15 : 0;
        const int l0 = w.w - bp.delta[i];            // window line of lloc = 0
        const int wl = l0 + lloc;
        const bool valid = (unsigned)wl < (unsigned)N;
        const int line = valid ? wl : 0;
        // a wavefront whose lines all lie outside this member's window (in the first or last
        // group of 16 object lines) skips the member's arithmetic; it still takes part in the
        // table loads and the LDS transpose, which synchronise the workgroup, and the transpose
        // stores none of its lines
        constexpr int LW = lines_per_wave<N>();
        const int lw = l0 + (tid / 64) * LW;
        const bool live = lw + LW > 0 && lw < N;
        const float2 *A_in = p.A_in + (size_t)b * NA;
        float2 v[16];
        if (m + 1 < M) load_h(g_fin);
        if (live) {
            float2 ps[16];
            if (RECOMP && m > 0) {
                // psi_m: the forward launch's window, the propagation of gap m - 1 finished
                aload<N, false>(ps, p.psi_in + (size_t)b * p.psi_in_stride, line, j, 0);
                prop_axis<N, false>(ps, s_tw, xb, h_start, j);
            }
            if (m + 1 == M) {
                aload<N, true>(v, A_in, line, j, s_elem);
                line_fft_inv<N>(v, s_tw, xb, j);
            } else {
                aload<N, false>(v, A_in, line, j, s_elem);
                prop_axis<N, true>(v, s_tw, xb, h_fin, j);
            }
            if (valid) {
                // acc += conj(psi_m) o g
                const int l2 = opaque(line), j2 = opaque(j);
                if (RECOMP && m > 0) {
#pragma unroll
                    for (int k = 0; k < 16; ++k) acc[k] = cadd(acc[k], cconjmul(ps[k], v[k]));
                } else {
                    const float2 *psi = p.psi_in && !RECOMP ? p.psi_in + (size_t)b * p.psi_in_stride
                                                            : p.class_probe + (size_t)info.z * NN;
#pragma unroll
                    for (int k = 0; k < 16; ++k)
                        acc[k] = cadd(acc[k], cconjmul(psi[l2 * N + Wn::nat(j2, k)], v[k]));
                }
            }
        } else {
#pragma unroll
            for (int k = 0; k < 16; ++k) v[k] = make_float2(0.f, 0.f);
        }
        if (!p.go_on) continue;
        if (m > 0) load_h(g_start);
        if (live) {
            frame_patch<N, TR, true>(v, p, info.x, info.y, line, j);
            if (m > 0) prop_axis<N, true>(v, s_tw, xb, h_start, j);
        }
        if (m > 0) {
            store_other<N, false>(v, p.A_out + (size_t)b * NA, Apitch<N>::P, l0, s_line, lloc, j, xbuf);
        } else if (p.probe_patch && valid) {
            gstore<N, true, false>(v, p.probe_patch + (size_t)b * NN, line, j);
        }
    }
    float2 *band = bp.band + (size_t)w.x * bp.band_stride;
    const int lloc = tid / R, j = tid % R;
    const int row = w.w + lloc;
    if ((unsigned)row < (unsigned)bp.rows) {
#pragma unroll
        for (int k = 0; k < 16; ++k) band[(size_t)row * N + Wn::nat(j, k)] = acc[k];
    }
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
