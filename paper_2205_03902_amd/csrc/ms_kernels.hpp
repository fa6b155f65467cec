// Device kernels of libimsp.  One workgroup owns one scan position: its N x N
// wave lives in registers (16 complex values per lane) for the whole multislice
// chain, LDS only carries line exchanges and transposes.  The Fresnel
// propagator of eq. (fresnel_element) factorises as h(q_y, q_x) = h_y(q_y) h_x(q_x),
// so V_z = (F_x^{-1} h_x F_x)(F_y^{-1} h_y F_y): one axis at a time, and the two
// factors commute, which lets consecutive slices alternate the axis order and
// pay a single transpose per propagation.
#pragma once

#include <hip/hip_runtime.h>

#include "fft_lines.hpp"

namespace imsp {

// Distinct slice distances whose propagator factors fit in LDS next to the window.
template <int N>
struct HCap {
    static constexpr int U = (N == 128) ? 8 : 4;
};

enum Mode : int {
    kForward = 0,   // intensities (and exit waves)
    kAdjoint = 1,   // loss, gradient patches of every slice and of the probe
    kLayer = 2,     // loss, gradient patch of one slice and its overlap patch
    kProbe = 3,     // loss and probe gradient patch
    kReplay = 4     // adjoint with recomputed incident waves: one slice's gradient patch a launch
};

struct FusedParams {
    const float2 *class_probe;   // [C][N][N] shifted probes
    const float2 *slices;        // [M][H][W]
    const int4 *pos_info;        // [S] (patch origin y in [0,H), x in [0,W), shift class, 0)
    const int *pos_list;         // [count] global position index of each workgroup
    const float2 *tw;            // [R][17] W_N^{j k1}
    const float2 *hy, *hx;       // [U][N] propagator factors of the distinct distances, divided by N
    const int *gap_table;        // [M-1] which of the U distinct distances each gap uses
    int n_tables;                // U <= HCap<N>::U
    const float *measured;       // [S][N][N]
    float *intensity;            // [S][N][N]
    float2 *exit_waves;          // [S][N][N] or null
    float2 *waves;               // per position wave_stride elements: incident waves, then gradient patches
                                 //   adjoint: slot m = psi_m; layer: slot 0 = psi_layer;
                                 //   replay: slots 0 .. nck-1 = psi_ck, psi_2ck, ..., slot nck = work
    long long wave_stride;
    float2 *probe_patch;         // [count][N][N] or null
    float *overlap_patch;        // per position ovl_stride elements: |psi_m|^2 (adjoint with full: slot m;
                                 //   layer and replay: slot 0)
    long long ovl_stride;
    double *loss_pos;            // [count]
    int H, W, M, layer;
    int objective;               // 0 amplitude, 1 Poisson deviance
    int full;                    // adjoint and replay modes: also write |psi_m|^2 of the patch's slice
    int ck;                      // replay: psi_m stored for m = ck, 2 ck, ... (ck >= 2)
    int seg;                     // replay: the slice whose patch this launch writes (M - 1 first)
    float2 *park;                // replay: [count][N][N] adjoint state between launches
    // line path, layer mode: the forward chain starts at launch chain_from (> 0: from the stored
    // wave chain_wave, psi of that slice, per position wave_stride apart); carry: psi_layer goes to
    // slot 1 of the waves and the patch to slot 0, so that the wave outlives the step
    int chain_from;
    const float2 *chain_wave;
    int carry;
};

// Incident-wave load/store in natural [y][x] order from either layout, with 32-bit element
// offsets from the window base (N^2 < 2^31), so that each access needs one address register.
template <int N, bool ROW>
__device__ __forceinline__ unsigned window_base(int line, int j)
{
    return ROW ? (unsigned)(line * N + j) : (unsigned)(j * N + line);
}

template <int N, bool ROW>
constexpr unsigned window_step()
{
    return ROW ? (unsigned)Win<N>::R : (unsigned)(Win<N>::R * N);
}

template <int N, bool ROW>
__device__ __forceinline__ void load_window(float2 (&v)[16], const float2 *src, int line, int j)
{
    const unsigned base = window_base<N, ROW>(opaque(line), opaque(j));
#pragma unroll
    for (int k = 0; k < 16; ++k) v[k] = src[base + window_step<N, ROW>() * k];
}

template <int N, bool ROW>
__device__ __forceinline__ void store_window(const float2 (&v)[16], float2 *dst, int line, int j)
{
    const unsigned base = window_base<N, ROW>(opaque(line), opaque(j));
#pragma unroll
    for (int k = 0; k < 16; ++k) dst[base + window_step<N, ROW>() * k] = v[k];
}

// |v|^2 of the window into a float image, natural order.
template <int N, bool ROW>
__device__ __forceinline__ void store_window_abs2(const float2 (&v)[16], float *dst, int line, int j)
{
    const unsigned base = window_base<N, ROW>(opaque(line), opaque(j));
#pragma unroll
    for (int k = 0; k < 16; ++k) dst[base + window_step<N, ROW>() * k] = cabs2(v[k]);
}

// t = the object patch t[(oy + y) mod H][(ox + x) mod W] (Sec. 1.3, 2.1) on this lane's 16 points.
// inside: the window lies inside the object (oy + N <= H, ox + N <= W), so no index wraps and every
// load is a per-lane base plus a constant step.
template <int N, bool ROW>
__device__ __forceinline__ void load_patch(float2 (&t)[16], const float2 *slice, int H, int W, int oy, int ox,
                                           int line, int j, bool inside = false)
{
    using Wn = Win<N>;
    constexpr int R = Wn::R;
    line = opaque(line);
    j = opaque(j);
    if (inside) {
        const unsigned base = ROW ? (unsigned)((oy + line) * W + ox + j) : (unsigned)((oy + j) * W + ox + line);
        const unsigned step = ROW ? (unsigned)R : (unsigned)(R * W);
#pragma unroll
        for (int k = 0; k < 16; ++k) t[k] = slice[base + step * k];
        return;
    }
    // 32-bit element offsets (H W <= 2^30): a step of R along the owned axis adds a constant,
    // and crossing the object edge subtracts one period.
    if (ROW) {
        int yy = oy + line;
        if (yy >= H) yy -= H;
        const unsigned row = (unsigned)(yy * W);
        const int x0 = ox + j;
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const int xx = x0 + R * k;
            const unsigned off = row + (unsigned)(xx >= W ? xx - W : xx);
            t[k] = slice[off];
        }
    } else {
        int xx = ox + line;
        if (xx >= W) xx -= W;
        const int y0 = oy + j;
        const unsigned base = (unsigned)(y0 * W + xx), wrap = (unsigned)(H * W), step = (unsigned)(R * W);
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const unsigned off = base + step * k - ((y0 + R * k >= H) ? wrap : 0u);
            t[k] = slice[off];
        }
    }
}

// v *= t (or conj(t)), pointwise.
template <bool CONJ>
__device__ __forceinline__ void mul_patch(float2 (&v)[16], const float2 (&t)[16])
{
#pragma unroll
    for (int k = 0; k < 16; ++k) v[k] = CONJ ? cconjmul(t[k], v[k]) : cmul(v[k], t[k]);
}

// v *= T (or conj(T)) on the window.
template <int N, bool ROW, bool CONJ>
__device__ __forceinline__ void apply_patch(float2 (&v)[16], const float2 *slice, int H, int W, int oy,
                                            int ox, int line, int j)
{
    float2 t[16];
    load_patch<N, ROW>(t, slice, H, W, oy, ox, line, j);
    mul_patch<CONJ>(v, t);
}

// One Fresnel propagation V_z (or its adjoint G^H when CONJ), starting in layout ROW
// and ending in the other layout.  hy/hx carry the 1/N factors of both inverse DFTs.
template <int N, bool ROW, bool CONJ>
__device__ __forceinline__ void propagate(float2 (&v)[16], const float2 *twg, float2 *lds, const float2 *hy,
                                          const float2 *hx, int line, int j)
{
    using Wn = Win<N>;
    line = opaque(line);
    j = opaque(j);
    float2 *xb = lds + line * Wn::LD;
    const float2 *h1 = ROW ? hx : hy;
    const float2 *h2 = ROW ? hy : hx;
    line_fft_fwd<N>(v, twg, xb, j);
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        float2 h = h1[Wn::spec(j, i)];
        v[i] = CONJ ? cmulc(v[i], h) : cmul(v[i], h);
    }
    line_fft_inv<N>(v, twg, xb, j);
    if constexpr (Wn::R >= 4) transpose_nat<N, ROW>(v, lds, line, j);
    else transpose<N, ROW, false, false>(v, lds, line, j);
    line_fft_fwd<N>(v, twg, xb, j);
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        float2 h = h2[Wn::spec(j, i)];
        v[i] = CONJ ? cmulc(v[i], h) : cmul(v[i], h);
    }
    line_fft_inv<N>(v, twg, xb, j);
}

template <int N>
__device__ __forceinline__ double block_sum(double x, double *red)
{
    // fixed-order tree: lanes of a wave by xor-shuffle, then waves in index order
    constexpr int NT = Win<N>::NT;
    constexpr int NW = (NT + 63) / 64;
    for (int off = (NT < 64 ? NT / 2 : 32); off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
    const int w = threadIdx.x / 64;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[w] = x;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < NW; ++i) t += red[i];
    return t;
}

// One pixel of the amplitude loss (Sec. 3.2): returns (sqrt(I) - |Psi|)^2 in FP64 and turns z = Psi
// into the residual Psi - sqrt(I) Psi / |Psi| (Psi itself where Psi = 0: the phase is taken as 0).
// Both come from d = sqrt(I) - |Psi| = (I - |Psi|^2) / (sqrt(I) + |Psi|) with I - |Psi|^2 formed in
// FP64, and the residual is Psi (-d / |Psi|): neither cancels when the fit is close (the form
// Psi - (sqrt(I) / |Psi|) Psi loses the digits that sqrt(I) / |Psi| shares with 1).  The two
// quotients use the FP32 reciprocal (1 ulp).
__device__ __forceinline__ double amp_residual(float m, float2 &z)
{
    const float a2 = cabs2(z);
    const float a = sqrtf(a2), sq = sqrtf(m);
    const double a2d = (double)z.x * (double)z.x + (double)z.y * (double)z.y;
    if (a2d == 0.0) return (double)m;   // Psi = 0: the term is I itself, the residual Psi
    // sqrt(I) + |Psi| is 0 only when I = 0 and |Psi|^2 underflows in FP32 (|Psi| < 1e-22)
    const float den = sq + a;
    const float d = den > 0.0f ? (float)((double)m - a2d) * __builtin_amdgcn_rcpf(den) : 0.0f;
    if (a2 != 0.0f) {
        const float f = -d * __builtin_amdgcn_rcpf(a);
        z = make_float2(z.x * f, z.y * f);
    }
    return (double)d * (double)d;
}

// Far field (Sec. 2.1) and amplitude residual (Sec. 3.2) on the 2D spectrum held in
// layout ROW2 (after the forward 2D FFT): r = Psi - sqrt(I) Psi / |Psi|, 0 where Psi = 0.
// Returns this lane's FP64 share of the loss: sum (sqrt(I) - |Psi|)^2 (amplitude) or, when
// poisson is set, sum |Psi|^2 - I + I log(I / |Psi|^2); v becomes the residual
// Psi - sqrt(I) Psi / |Psi| or Psi (1 - I / |Psi|^2) (Psi itself where Psi == 0).
template <int N, bool ROW2>
__device__ __forceinline__ double residual(float2 (&v)[16], const float *meas, int line, int j, int poisson)
{
    using Wn = Win<N>;
    line = opaque(line);
    j = opaque(j);
    double acc = 0.0;
    if (poisson) {
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            int f = Wn::spec(j, i);
            int fy = ROW2 ? line : f, fx = ROW2 ? f : line;
            float m = meas[fy * N + fx];
            float2 z = v[i];
            float a2 = cabs2(z);
            double a2d = (double)z.x * (double)z.x + (double)z.y * (double)z.y;
            if (a2d != 0.0) acc += a2d - (double)m + (m > 0.0f ? (double)m * log((double)m / a2d) : 0.0);
            if (a2 != 0.0f) {
                float k = m / a2;
                v[i] = make_float2(z.x - k * z.x, z.y - k * z.y);
            }
        }
        return acc;
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        int f = Wn::spec(j, i);
        int fy = ROW2 ? line : f, fx = ROW2 ? f : line;
        acc += amp_residual(meas[fy * N + fx], v[i]);
    }
    return acc;
}

// Copies n complex values into LDS with the whole workgroup.
template <int N>
__device__ __forceinline__ void stage(float2 *dst, const float2 *src, int n)
{
    for (int i = threadIdx.x; i < n; i += Win<N>::NT) dst[i] = src[i];
}

// Where psi_m goes in the forward chain (null: not stored).  wave: this position's wave region.
template <int MODE>
__device__ __forceinline__ float2 *forward_store(const FusedParams &p, float2 *wave, int m, size_t NN)
{
    if (m == 0) return nullptr;                                   // psi_0 is the shifted probe
    if (MODE == kAdjoint) return wave + m * NN;
    if (MODE == kLayer) return m == p.layer ? wave : nullptr;
    if (MODE == kReplay) {
        const int nck = (p.M - 1) / p.ck;
        if (m % p.ck == 0) return wave + (size_t)(m / p.ck - 1) * NN;
        if (m == p.M - 1) return wave + (size_t)nck * NN;         // the head launch's own slice
    }
    return nullptr;
}

template <int N, int MODE>
__global__ __launch_bounds__(Win<N>::NT) __attribute__((amdgpu_waves_per_eu(4))) void fused_kernel(FusedParams p)
{
    using Wn = Win<N>;
    constexpr int R = Wn::R;
    constexpr size_t NN = (size_t)N * N;
    __shared__ float2 lds[Wn::LDS_WORDS];
    __shared__ float2 s_tw[Wn::TW_WORDS];
    __shared__ float2 s_hy[HCap<N>::U * N], s_hx[HCap<N>::U * N];
    __shared__ double red[(Wn::NT + 63) / 64];

    const int tid = threadIdx.x;
    const int line = tid / R, j = tid % R;
    const int b = blockIdx.x;
    const int s = p.pos_list[b];
    const int4 info = p.pos_info[s];
    const int oy = info.x, ox = info.y, cls = info.z;
    const int H = p.H, W = p.W, M = p.M;
    const bool inside = (oy + N <= H) && (ox + N <= W);   // the patch does not wrap

    // twiddles and propagator factors live in LDS for the whole chain
    stage<N>(s_tw, p.tw, Wn::TW_WORDS);
    stage<N>(s_hy, p.hy, p.n_tables * N);
    stage<N>(s_hx, p.hx, p.n_tables * N);
    __syncthreads();
    const float2 *tw = s_tw;

    float2 *wave = p.waves ? p.waves + (size_t)b * p.wave_stride : nullptr;
    const float2 *probe = p.class_probe + (size_t)cls * NN;
    float2 *xb = lds + line * Wn::LD;
    float2 v[16];
    // Replay launches after the first: the adjoint of slice seg alone, from the state the
    // previous launch parked, with psi_seg recomputed from the nearest stored wave below it.
    const bool head = (MODE != kReplay) || (p.seg == M - 1);
    const int m_stop = (MODE == kLayer) ? p.layer : (MODE == kReplay ? p.seg : 0);
    int m_hi = M - 1;

    if (head) {
        load_window<N, true>(v, probe, line, j);

        // ---- forward multislice: E_1 = P^s o X_1, E_m = V(E_{m-1}) o X_m (Sec. 2.1) ----
        for (int m = 0; m < M; ++m) {
            const bool row = !(m & 1);
            const float2 *slice = p.slices + (size_t)m * H * W;
            float2 *st = forward_store<MODE>(p, wave, m, NN);
            float *ovl = (MODE == kLayer && m == p.layer) ? p.overlap_patch + (size_t)b * p.ovl_stride : nullptr;
            if (row) {
                // the transmission loads go out before this step's stores: the vector memory
                // counter retires in issue order, so waiting for them does not wait for the stores
                float2 t[16];
                load_patch<N, true>(t, slice, H, W, oy, ox, line, j, inside);
                if (st) store_window<N, true>(v, st, line, j);
                if (ovl) store_window_abs2<N, true>(v, ovl, line, j);
                mul_patch<false>(v, t);
                if (m + 1 < M) {
                    const int u = p.gap_table[m] * N;
                    propagate<N, true, false>(v, tw, lds, s_hy + u, s_hx + u, line, j);
                }
            } else {
                float2 t[16];
                load_patch<N, false>(t, slice, H, W, oy, ox, line, j, inside);
                if (st) store_window<N, false>(v, st, line, j);
                if (ovl) store_window_abs2<N, false>(v, ovl, line, j);
                mul_patch<false>(v, t);
                if (m + 1 < M) {
                    const int u = p.gap_table[m] * N;
                    propagate<N, false, false>(v, tw, lds, s_hy + u, s_hx + u, line, j);
                }
            }
        }

        // ---- far field Psi = F E_M ----
        const bool rowM = !((M - 1) & 1);
        if constexpr (MODE == kForward) {
            if (p.exit_waves) {
                float2 *ew = p.exit_waves + (size_t)s * NN;
                if (rowM) store_window<N, true>(v, ew, line, j);
                else store_window<N, false>(v, ew, line, j);
            }
        }
        line_fft_fwd<N>(v, tw, xb, j);
        if (rowM) transpose<N, true, true, false>(v, lds, line, j);
        else transpose<N, false, true, false>(v, lds, line, j);
        line_fft_fwd<N>(v, tw, xb, j);
        // now layout !rowM; line = frequency along the first axis, registers spectral along the second

        if constexpr (MODE == kForward) {
            float *out = p.intensity + (size_t)s * NN;
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                int f = Wn::spec(j, i);
                int fy = rowM ? f : line, fx = rowM ? line : f;
                out[fy * N + fx] = cabs2(v[i]);
            }
            return;
        }
        const float *meas = p.measured + (size_t)s * NN;
        double part = rowM ? residual<N, false>(v, meas, line, j, p.objective)
                           : residual<N, true>(v, meas, line, j, p.objective);
        double tot = block_sum<N>(part, red);
        if (tid == 0) p.loss_pos[b] = tot;

        // ---- adjoint: g = F^H r, then down the chain (Sec. 3.2 pulled back through eq. exit_wave_mslices) ----
        line_fft_inv<N>(v, tw, xb, j);
        if (rowM) transpose<N, false, false, true>(v, lds, line, j);
        else transpose<N, true, false, true>(v, lds, line, j);
        line_fft_inv<N>(v, tw, xb, j);
    } else if constexpr (MODE == kReplay) {
        // psi_seg from the stored wave psi_c (or the probe at c = 0), c = seg - seg mod ck
        const int seg = p.seg, c = seg - seg % p.ck;
        const int nck = (M - 1) / p.ck;
        if (c < seg) {
            const float2 *src = (c == 0) ? probe : wave + (size_t)(c / p.ck - 1) * NN;
            if (!(c & 1)) load_window<N, true>(v, src, line, j);
            else load_window<N, false>(v, src, line, j);
            for (int m = c; m < seg; ++m) {
                const bool row = !(m & 1);
                const float2 *slice = p.slices + (size_t)m * H * W;
                const int u = p.gap_table[m] * N;
                float2 t[16];
                if (row) {
                    load_patch<N, true>(t, slice, H, W, oy, ox, line, j, inside);
                    mul_patch<false>(v, t);
                    propagate<N, true, false>(v, tw, lds, s_hy + u, s_hx + u, line, j);
                } else {
                    load_patch<N, false>(t, slice, H, W, oy, ox, line, j, inside);
                    mul_patch<false>(v, t);
                    propagate<N, false, false>(v, tw, lds, s_hy + u, s_hx + u, line, j);
                }
            }
            float2 *work = wave + (size_t)nck * NN;
            if (!(seg & 1)) store_window<N, true>(v, work, line, j);
            else store_window<N, false>(v, work, line, j);
        }
        const float2 *pk = p.park + (size_t)b * NN;
        if (!(seg & 1)) load_window<N, true>(v, pk, line, j);
        else load_window<N, false>(v, pk, line, j);
        m_hi = seg;
    }

    if constexpr (MODE != kForward) {
        int m = m_hi;
        for (; m >= m_stop; --m) {
            const bool row = !(m & 1);
            const float2 *slice = p.slices + (size_t)m * H * W;
            const bool patch = (MODE == kAdjoint) || (MODE == kReplay) || (MODE == kLayer && m == p.layer);
            const bool go_on = (m > m_stop) || (MODE != kLayer && m == 0) || (MODE == kReplay);
            // Memory order of the step.  Vector memory operations retire in issue order, so a
            // wait for a load also waits for every store issued before it.  The transmission
            // loads go out first (they are consumed last); the incident wave is read and the
            // gradient patch written in two halves, which keeps the live registers within the
            // budget of 1024 lanes.  The layer mode, whose patch is one slice's, reads the
            // transmission after the patch instead (no spills in either form).
            constexpr bool kEarlyT = (MODE != kLayer);
            float2 t[16];
            if (kEarlyT && go_on) {
                if (row) load_patch<N, true>(t, slice, H, W, oy, ox, line, j, inside);
                else load_patch<N, false>(t, slice, H, W, oy, ox, line, j, inside);
            }
            if (patch) {
                const float2 *psi;
                float2 *dst;
                float *ovl = nullptr;
                if constexpr (MODE == kReplay) {
                    const int nck = (M - 1) / p.ck;
                    dst = wave + (size_t)nck * NN;
                    psi = (m == 0) ? probe : (m % p.ck == 0 ? wave + (size_t)(m / p.ck - 1) * NN : dst);
                    if (p.full) ovl = p.overlap_patch + (size_t)b * p.ovl_stride;
                } else if constexpr (MODE == kLayer) {
                    dst = wave;
                    psi = (m == 0) ? probe : wave;
                } else {
                    dst = wave + m * NN;
                    psi = (m == 0) ? probe : dst;
                    if (MODE == kAdjoint && p.full) ovl = p.overlap_patch + (size_t)b * p.ovl_stride + m * NN;
                }
                // 32-bit element offsets from the window base (N^2 < 2^31): one address
                // register per access instead of a 64-bit pointer each
                const int l2 = opaque(line), j2 = opaque(j);
                const unsigned base = row ? (unsigned)(l2 * N + j2) : (unsigned)(j2 * N + l2);
                const unsigned step = row ? (unsigned)R : (unsigned)(R * N);
#pragma unroll
                for (int h = 0; h < 16; h += 8) {
                    float2 ps[8];
#pragma unroll
                    for (int k = 0; k < 8; ++k) ps[k] = psi[base + step * (h + k)];
#pragma unroll
                    for (int k = 0; k < 8; ++k) {
                        const unsigned off = base + step * (h + k);
                        if (ovl) ovl[off] = cabs2(ps[k]);
                        dst[off] = cconjmul(ps[k], v[h + k]);   // dL/d conj(t_m) on the window: conj(psi_m) o g
                    }
                }
            }
            if (!go_on) break;
            if (!kEarlyT) {
                if (row) load_patch<N, true>(t, slice, H, W, oy, ox, line, j, inside);
                else load_patch<N, false>(t, slice, H, W, oy, ox, line, j, inside);
            }
            mul_patch<true>(v, t);
            if (m > 0) {
                // G_{m-1}^H: start on the axis this layout owns (the last one of the forward step)
                const int u = p.gap_table[m - 1] * N;
                if (row) propagate<N, true, true>(v, tw, lds, s_hy + u, s_hx + u, line, j);
                else propagate<N, false, true>(v, tw, lds, s_hy + u, s_hx + u, line, j);
            }
            if (MODE == kReplay) break;                  // one slice a launch
        }
        if constexpr (MODE == kReplay) {
            if (m_stop > 0) {
                // park the state for the launch of slice m_stop - 1, in that slice's layout
                float2 *pk = p.park + (size_t)b * NN;
                if (!((m_stop - 1) & 1)) store_window<N, true>(v, pk, line, j);
                else store_window<N, false>(v, pk, line, j);
                return;
            }
        }
        if constexpr (MODE == kAdjoint || MODE == kProbe || MODE == kReplay) {
            if (p.probe_patch) store_window<N, true>(v, p.probe_patch + (size_t)b * NN, line, j);
        }
    }
}

// ---------------------------------------------------------------------------
// Deterministic segmented scatter-add (the sum over positions of eq. Opt_Prob_Layerwise
// carried into object coordinates).  Positions of a batch are cut into at most kChunks
// chunks of consecutive positions.  Pass 1: block (tile, chunk, slice) adds, pixel by
// pixel and in ascending position order, the patches of the chunk's windows that touch
// the tile; pass 2 adds the chunk partials in chunk order.  The order is fixed by the
// plan, so results are reproducible bit for bit.
// Scatter tiles, one 256-lane block each.  16 x 16 pixels where images may be stored transposed
// (the line path): lanes run along x for images in the natural layout and along y for transposed
// ones, so that either reads 128-byte pieces.  64 x 4 pixels where every image is in the natural
// layout (the fused path): a lane row reads 512 contiguous bytes, so a window that starts off a
// 128-byte boundary over-fetches a quarter of a row rather than a whole row.
constexpr int kTileW = 16;
constexpr int kTileH = 16;
constexpr int kWideW = 64;
constexpr int kWideH = 4;
constexpr int kChunks = 16;  // chunks per batch
constexpr int kUnroll = 8;   // patch loads in flight per lane

// The images scattered are per-position patches (N x N) or band images of several positions (see
// line_band_kernel): an entry (image, origin y, origin x, extent) covers N rows and N + extent
// columns of the object (N + extent rows and N columns for vertical bands), element (y, x) of the
// image at y * ld + x, or at x * ld + y for images stored transposed (the line path's odd slices).
// Slices m0 + i of even and odd index have images, lists and geometry of their own.
struct ScatterParams {
    // image e of slice i of the launch: patches + e * pos_stride + i * slice_stride, per parity
    const float2 *patches0, *patches1;
    long long pos_stride0, pos_stride1, slice_stride0, slice_stride1;
    const float *wpatch;        // overlap patch of (position e, slice i): wpatch + e * w_stride + i * N * N
    const int *tile_off0, *tile_off1;    // this batch: [kChunks][n_tiles + 1]
    const int4 *entries0, *entries1;
    int ld0, ld1, vert0, vert1, trans0, trans1;
    int m0;                     // slice index of i = 0
    float2 *partial;            // [groups][n_m][H][W]
    float *wpartial;            // [groups][n_m][H][W] or null (patches only)
    long long w_stride;
    int H, W, N, tiles_x, n_tiles;
    int nch, cpb;               // chunks of the batch; consecutive chunks summed per block
};

template <int TW, int TH>
__global__ __launch_bounds__(256) void scatter_partial_kernel(ScatterParams p)
{
    static_assert(TW * TH == 256, "one lane a pixel");
    const int t = blockIdx.x, grp = blockIdx.y, mi = blockIdx.z, n_m = gridDim.z;
    const bool odd = ((p.m0 + mi) & 1) != 0;
    // transposed images only with square tiles
    const bool trans = TW == TH && (odd ? p.trans1 : p.trans0) != 0;
    const int ta = (int)(threadIdx.x / TW), tb = (int)(threadIdx.x % TW);
    const int y = (t / p.tiles_x) * TH + (trans ? tb : ta);
    const int x = (t % p.tiles_x) * TW + (trans ? ta : tb);
    const bool inside = y < p.H && x < p.W;
    const size_t NN = (size_t)p.N * p.N;
    const int *tile_off = odd ? p.tile_off1 : p.tile_off0;
    const int4 *entries = odd ? p.entries1 : p.entries0;
    const int ld = odd ? p.ld1 : p.ld0;
    const int vert = odd ? p.vert1 : p.vert0;
    const long long pos_stride = odd ? p.pos_stride1 : p.pos_stride0;
    const float2 *base = odd ? p.patches1 + (size_t)mi * p.slice_stride1 : p.patches0 + (size_t)mi * p.slice_stride0;
    const bool want_w = p.wpartial != nullptr;
    const float *wbase = want_w ? p.wpatch + (size_t)mi * NN : nullptr;
    float2 acc = make_float2(0.f, 0.f);
    float wacc = 0.f;
    const int c_end = inside ? min(p.nch, (grp + 1) * p.cpb) : 0;
    for (int c = grp * p.cpb; c < c_end; ++c) {
    const int *off = tile_off + (size_t)c * (p.n_tiles + 1);
    const int e0 = off[t], e1 = off[t + 1];
    for (int e = e0; e < e1; e += kUnroll) {
        int sl[kUnroll], loc[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            loc[u] = -1;
            sl[u] = 0;
            if (e + u < e1) {
                const int4 en = entries[e + u];
                int ly = y - en.y;
                if (ly < 0) ly += p.H;
                int lx = x - en.z;
                if (lx < 0) lx += p.W;
                sl[u] = en.x;
                const int rows = p.N + (vert ? en.w : 0), cols = p.N + (vert ? 0 : en.w);
                if (ly < rows && lx < cols) loc[u] = trans ? lx * ld + ly : ly * ld + lx;
            }
        }
        float2 v[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u)
            v[u] = loc[u] >= 0 ? base[(size_t)sl[u] * pos_stride + loc[u]] : make_float2(0.f, 0.f);
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) acc = cadd(acc, v[u]);
        if (want_w) {
            float w[kUnroll];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) w[u] = loc[u] >= 0 ? wbase[(size_t)sl[u] * p.w_stride + loc[u]] : 0.f;
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) wacc += w[u];
        }
    }
    }
    const size_t HW = (size_t)p.H * p.W;
    int yo = y, xo = x;
    if constexpr (TW == TH) {
        if (trans) {
            // back to lanes along x for the partial planes (natural layout)
            __shared__ float2 sacc[TH][TW + 1];
            __shared__ float swacc[TH][TW + 1];
            sacc[tb][ta] = acc;
            swacc[tb][ta] = wacc;
            __syncthreads();
            acc = sacc[ta][tb];
            wacc = swacc[ta][tb];
            yo = (t / p.tiles_x) * TH + ta;
            xo = (t % p.tiles_x) * TW + tb;
        }
    }
    if (yo >= p.H || xo >= p.W) return;
    const size_t pix = (size_t)yo * p.W + xo;
    p.partial[((size_t)grp * n_m + mi) * HW + pix] = acc;
    if (want_w) p.wpartial[((size_t)grp * n_m + mi) * HW + pix] = wacc;
}

// out[i] = (accumulate ? out[i] : 0) + sum_{c < nch} partial[c * plane + i], chunks in order.
template <typename T>
__device__ __forceinline__ T zero_of();
template <>
__device__ __forceinline__ float2 zero_of<float2>() { return make_float2(0.f, 0.f); }
template <>
__device__ __forceinline__ float zero_of<float>() { return 0.f; }
__device__ __forceinline__ float2 add_of(float2 a, float2 b) { return cadd(a, b); }
__device__ __forceinline__ float add_of(float a, float b) { return a + b; }

template <typename T>
__global__ __launch_bounds__(256) void chunk_reduce_kernel(const T *partial, int nch, long long plane, T *out,
                                                           int accumulate)
{
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < plane; i += (long long)gridDim.x * 256) {
        T a = accumulate ? out[i] : zero_of<T>();
        for (int c = 0; c < nch; ++c) a = add_of(a, partial[(size_t)c * plane + i]);
        out[i] = a;
    }
}

// Probe patches summed per shift class and chunk (ascending positions):
// cpart[chunk][class][pixel].  Grid (pixel blocks, classes, chunks).
__global__ __launch_bounds__(256) void class_partial_kernel(const float2 *probe_patch, const int *class_off,
                                                            const int *class_list, float2 *cpart, int n_classes,
                                                            int nn)
{
    const int pix = blockIdx.x * 256 + threadIdx.x;
    const int k = blockIdx.y, c = blockIdx.z;
    if (pix >= nn) return;
    const int *off = class_off + (size_t)c * (n_classes + 1);
    const int e0 = off[k], e1 = off[k + 1];
    float2 a = make_float2(0.f, 0.f);
    for (int e = e0; e < e1; e += kUnroll) {
        float2 v[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u)
            v[u] = (e + u < e1) ? probe_patch[(size_t)class_list[e + u] * nn + pix] : make_float2(0.f, 0.f);
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) a = cadd(a, v[u]);
    }
    cpart[((size_t)c * n_classes + k) * nn + pix] = a;
}

// out[c] = F^{-1}(F in[c] o (my[c] (x) mx[c])) with multipliers already divided by N:
// the sub-pixel probe shift of class c (CONJ = false) or its adjoint (CONJ = true).
// identity[c] != 0 copies instead (integer positions).
template <int N, bool CONJ>
__global__ __launch_bounds__(Win<N>::NT) void window_filter_kernel(const float2 *in, long long in_stride, float2 *out,
                                                                   const float2 *my, const float2 *mx,
                                                                   const int *identity, const float2 *twg)
{
    using Wn = Win<N>;
    constexpr int R = Wn::R;
    constexpr size_t NN = (size_t)N * N;
    __shared__ float2 lds[Wn::LDS_WORDS];
    const int c = blockIdx.x;
    const int line = threadIdx.x / R, j = threadIdx.x % R;
    const float2 *src = in + (size_t)c * in_stride;
    float2 *dst = out + (size_t)c * NN;
    float2 v[16];
    load_window<N, true>(v, src, line, j);
    if (identity[c]) {
        store_window<N, true>(v, dst, line, j);
        return;
    }
    __shared__ float2 s_tw[Wn::TW_WORDS];
    stage<N>(s_tw, twg, Wn::TW_WORDS);
    __syncthreads();
    propagate<N, true, CONJ>(v, s_tw, lds, my + (size_t)c * N, mx + (size_t)c * N, line, j);
    store_window<N, false>(v, dst, line, j);
}

// Probe of Sec. 2.1 / Fig. 3: aperture lambda |q| <= alpha times the defocus propagator
// times (-1)^(ky+kx) (centre at N/2), inverse 2D DFT, unit energy.  One workgroup.
// Aperture phase of the probe-forming lens: defocus C1, twofold astigmatism A1 at phi_A1,
// spherical aberration C3 (A, rad).  chi = pi lambda (C1 q^2 + A1 ((qx^2 - qy^2) cos 2 phi_A1
// + 2 qx qy sin 2 phi_A1)) + pi/2 lambda^3 C3 q^4, i.e. A1 q^2 cos 2(phi - phi_A1) written
// without the azimuth.  The probe takes exp(-i chi).
struct Aberrations {
    double c1, a1, cos2a, sin2a, c3;
};

__device__ __forceinline__ double aberration_phase(const Aberrations &ab, double lambda, double qy, double qx)
{
#pragma clang fp contract(off)
    const double PI = 3.14159265358979323846264338327950288;
    const double q2 = qy * qy + qx * qx;
    const double astig = (qx * qx - qy * qy) * ab.cos2a + 2.0 * qx * qy * ab.sin2a;
    return PI * lambda * (ab.c1 * q2 + ab.a1 * astig) + 0.5 * PI * lambda * lambda * lambda * ab.c3 * q2 * q2;
}

template <int N>
__global__ __launch_bounds__(Win<N>::NT) void make_probe_kernel(float2 *out, const float2 *twg, double dx,
                                                                double lambda, double alpha, Aberrations ab)
{
#pragma clang fp contract(off)
    using Wn = Win<N>;
    constexpr int R = Wn::R;
    __shared__ float2 lds[Wn::LDS_WORDS];
    __shared__ double red[(Wn::NT + 63) / 64];
    __shared__ double total;
    const int line = threadIdx.x / R, j = threadIdx.x % R;
    __shared__ float2 s_tw[Wn::TW_WORDS];
    stage<N>(s_tw, twg, Wn::TW_WORDS);
    __syncthreads();
    const float2 *tw = s_tw;
    const double nd = (double)N * dx;
    float2 v[16];
    // ROW layout, spectral along x: register i holds frequency (ky = line, kx = spec(j, i))
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        int iy = line, ix = Wn::spec(j, i);
        int ky = iy < N / 2 ? iy : iy - N;
        int kx = ix < N / 2 ? ix : ix - N;
        double qy = (double)ky / nd, qx = (double)kx / nd;
        double q2 = qy * qy + qx * qx;
        float2 a = make_float2(0.f, 0.f);
        if (lambda * sqrt(q2) <= alpha) {
            double ph = -aberration_phase(ab, lambda, qy, qx);
            double sgn = ((iy + ix) & 1) ? -1.0 : 1.0;
            a = make_float2((float)(sgn * cos(ph)), (float)(sgn * sin(ph)));
        }
        v[i] = a;
    }
    float2 *xb = lds + line * Wn::LD;
    line_fft_inv<N>(v, tw, xb, j);
    transpose<N, true, false, true>(v, lds, line, j);
    line_fft_inv<N>(v, tw, xb, j);
    double e = 0.0;
#pragma unroll
    for (int i = 0; i < 16; ++i) e += (double)v[i].x * v[i].x + (double)v[i].y * v[i].y;
    double t = block_sum<N>(e, red);
    if (threadIdx.x == 0) total = t;
    __syncthreads();
    const float sc = (float)(1.0 / sqrt(total));
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = make_float2(v[i].x * sc, v[i].y * sc);
    store_window<N, false>(v, out, line, j);
}

// ---------------------------------------------------------------------------
// Small reductions and updates (FP64 where the step size is concerned).

// Per-block maximum of |x|^2 (complex) or x (real) over segment blockIdx.y.
__global__ __launch_bounds__(256) void max_partial_kernel(const float2 *cx, const float *rx, long long seg_len,
                                                          float *partial)
{
    __shared__ float sm[256];
    const long long base = (long long)blockIdx.y * seg_len;
    float mx = 0.f;
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < seg_len; i += (long long)gridDim.x * 256) {
        float v = cx ? cabs2(cx[base + i]) : rx[base + i];
        mx = fmaxf(mx, v);
    }
    sm[threadIdx.x] = mx;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) sm[threadIdx.x] = fmaxf(sm[threadIdx.x], sm[threadIdx.x + off]);
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.y * gridDim.x + blockIdx.x] = sm[0];
}

__global__ __launch_bounds__(256) void max_final_kernel(const float *partial, int per_seg, float *out)
{
    __shared__ float sm[256];
    float mx = 0.f;
    for (int i = threadIdx.x; i < per_seg; i += 256) mx = fmaxf(mx, partial[blockIdx.x * per_seg + i]);
    sm[threadIdx.x] = mx;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) sm[threadIdx.x] = fmaxf(sm[threadIdx.x], sm[threadIdx.x + off]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = sm[0];
}

// Fixed-order FP64 sum of the per-position losses of one batch, added to *total.
__global__ __launch_bounds__(256) void loss_sum_kernel(const double *loss_pos, int count, double *total, int accumulate)
{
    __shared__ double sm[256];
    double a = 0.0;
    // lane l adds entries l, l + 256, l + 512, ... in that order, 16 loads in flight at a time
    constexpr int U = 16;
    int i = threadIdx.x;
    for (; i + (U - 1) * 256 < count; i += U * 256) {
        double v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = loss_pos[i + u * 256];
#pragma unroll
        for (int u = 0; u < U; ++u) a += v[u];
    }
    for (; i < count; i += 256) a += loss_pos[i];
    sm[threadIdx.x] = a;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) sm[threadIdx.x] += sm[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) *total = (accumulate ? *total : 0.0) + sm[0];
}

// mu = 1 / (nn * count * prod_{m in [m0, M)} maxt2[m] * wmax); wmax null means 1.
__global__ void step_size_kernel(const float *maxt2, int m0, int M, const float *wmax, double nn, double count,
                                 double *mu, double *mu_user, const double *loss, double *loss_user)
{
    double den = nn * count;
    for (int m = m0; m < M; ++m) den *= (double)maxt2[m];
    if (wmax) den *= (double)*wmax;
    double r = den > 0.0 ? 1.0 / den : 0.0;
    *mu = r;
    if (mu_user) *mu_user = r;
    if (loss_user) *loss_user = *loss;
}

// x <- x - mu * g, evaluated in FP64 and rounded once.
__global__ __launch_bounds__(256) void update_kernel(float2 *x, const float2 *g, long long count, const double *mu)
{
    const double m = *mu;
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < count; i += (long long)gridDim.x * 256) {
        float2 a = x[i], d = g[i];
        x[i] = make_float2((float)((double)a.x - m * (double)d.x), (float)((double)a.y - m * (double)d.y));
    }
}

// out = sum_c in[c] (fixed order).
__global__ __launch_bounds__(256) void sum_classes_kernel(const float2 *in, int n_classes, int nn, float2 *out)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= nn) return;
    float2 a = make_float2(0.f, 0.f);
    for (int c = 0; c < n_classes; ++c) a = cadd(a, in[(size_t)c * nn + i]);
    out[i] = a;
}

__global__ void copy_scalar_kernel(const double *src, double *dst) { *dst = *src; }

// Position gradient of one batch: block b takes position s = pos_list[b] of class c,
//   grad[s] = 2 Re sum conj(g_b) dP_c (y, x),  g_b the probe patch dL/dconj(P^s),
//   curv[s] = 2 nn prod_m maxt2[m] ||dP_c||^2,
// dprobe = [dP/df_y for every class][dP/df_x for every class].  FP64 sums, fixed order.
__global__ __launch_bounds__(256) void position_grad_kernel(const float2 *patch, const int *pos_list,
                                                            const int4 *pos_info, const float2 *dprobe,
                                                            long long class_plane, int nn, const float *maxt2,
                                                            int M, double *grad, double *curv)
{
    __shared__ double red[4][256];
    const int b = blockIdx.x, t = threadIdx.x;
    const int s = pos_list[b];
    const int c = pos_info[s].z;
    const float2 *g = patch + (size_t)b * nn;
    const float2 *dy = dprobe + (size_t)c * nn;
    const float2 *dx = dprobe + class_plane + (size_t)c * nn;
    double gy = 0.0, gx = 0.0, ny = 0.0, nx = 0.0;
    for (int i = t; i < nn; i += 256) {
        const float2 a = g[i], u = dy[i], v = dx[i];
        gy += (double)a.x * u.x + (double)a.y * u.y;
        gx += (double)a.x * v.x + (double)a.y * v.y;
        ny += (double)u.x * u.x + (double)u.y * u.y;
        nx += (double)v.x * v.x + (double)v.y * v.y;
    }
    red[0][t] = gy;
    red[1][t] = gx;
    red[2][t] = ny;
    red[3][t] = nx;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w)
#pragma unroll
            for (int q = 0; q < 4; ++q) red[q][t] += red[q][t + w];
        __syncthreads();
    }
    if (t == 0) {
        grad[2 * (size_t)s] = 2.0 * red[0][0];
        grad[2 * (size_t)s + 1] = 2.0 * red[1][0];
        if (curv) {
            double tp = 1.0;
            for (int m = 0; m < M; ++m) tp *= (double)maxt2[m];
            curv[2 * (size_t)s] = 2.0 * (double)nn * tp * red[2][0];
            curv[2 * (size_t)s + 1] = 2.0 * (double)nn * tp * red[3][0];
        }
    }
}

// Relative reconstruction error of the experiments (Sec. 5) at every translation tried.  Block
// (k, m) takes slice m of the estimate translated by d_k (periodically: est[(y - d_y) mod H]
// [(x - d_x) mod W] at reference pixel (y, x)), and over the reference pixels where mask > 0 forms in
// FP64, in a fixed order, <est_d, ref>, ||est_d||^2 and ||ref||^2; the error with the least-squares
// complex scale is sqrt(||ref||^2 - |<est_d, ref>|^2 / ||est_d||^2) / ||ref|| (1 where est_d is 0).
// d_k = (k / (2 r + 1) - r, k mod (2 r + 1) - r), r = max_shift < min(H, W).  err: [n_shifts][M + 1].
__global__ __launch_bounds__(256) void recon_shift_kernel(const float2 *est, const float2 *ref, const float *mask,
                                                          int H, int W, int max_shift, int M, double *err)
{
    __shared__ double red[4][256];
    const int k = blockIdx.x, m = blockIdx.y, t = threadIdx.x;
    const int side = 2 * max_shift + 1;
    const int dy = k / side - max_shift, dx = k % side - max_shift;
    const long long hw = (long long)H * W;
    const float2 *e = est + (size_t)m * hw, *r = ref + (size_t)m * hw;
    double xr = 0.0, xi = 0.0, ee = 0.0, rr = 0.0;
    for (long long i = t; i < hw; i += 256) {
        if (mask && !(mask[i] > 0.0f)) continue;
        const int y = (int)(i / W), x = (int)(i - (long long)y * W);
        int ys = y - dy, xs = x - dx;
        if (ys < 0) ys += H; else if (ys >= H) ys -= H;
        if (xs < 0) xs += W; else if (xs >= W) xs -= W;
        const float2 a = e[(size_t)ys * W + xs], b = r[i];
        xr += (double)a.x * b.x + (double)a.y * b.y;
        xi += (double)a.x * b.y - (double)a.y * b.x;
        ee += (double)a.x * a.x + (double)a.y * a.y;
        rr += (double)b.x * b.x + (double)b.y * b.y;
    }
    red[0][t] = xr;
    red[1][t] = xi;
    red[2][t] = ee;
    red[3][t] = rr;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w)
#pragma unroll
            for (int q = 0; q < 4; ++q) red[q][t] += red[q][t + w];
        __syncthreads();
    }
    if (t == 0) {
        const double x2 = red[0][0] * red[0][0] + red[1][0] * red[1][0], e2 = red[2][0], r2 = red[3][0];
        double v = 0.0;
        if (r2 > 0.0) v = e2 > 0.0 ? sqrt(fmax(0.0, r2 - x2 / e2) / r2) : 1.0;
        err[(size_t)k * (M + 1) + m] = v;
    }
}

// Mean error over the slices of every translation (slices in order), then the translation with the
// smallest mean, the first one in the order of k: its errors and mean into out[M + 1] and d into
// shift (if not null).  One thread.
__global__ void recon_select_kernel(double *err, int n_shifts, int M, int max_shift, double *out, int *shift)
{
    int best = 0;
    for (int k = 0; k < n_shifts; ++k) {
        double s = 0.0;
        for (int m = 0; m < M; ++m) s += err[(size_t)k * (M + 1) + m];
        err[(size_t)k * (M + 1) + M] = s / M;
        if (err[(size_t)k * (M + 1) + M] < err[(size_t)best * (M + 1) + M]) best = k;
    }
    for (int m = 0; m <= M; ++m) out[m] = err[(size_t)best * (M + 1) + m];
    if (shift) {
        const int side = 2 * max_shift + 1;
        shift[0] = best / side - max_shift;
        shift[1] = best % side - max_shift;
    }
}

// positions <- positions - scale grad / curv per coordinate (unchanged where curv is 0).
__global__ __launch_bounds__(256) void position_update_kernel(double *pos, const double *grad, const double *curv,
                                                              long long count, double scale)
{
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < count; i += (long long)gridDim.x * 256)
        if (curv[i] > 0.0) pos[i] -= scale * grad[i] / curv[i];
}

}  // namespace imsp
