// Register-resident FFT building blocks for gfx950 (wave64).
//
// A length-N line (N = 16 R) is held by R consecutive lanes of one wavefront,
// 16 complex values per lane: lane j owns x[j + R k], k = 0..15.  A forward
// transform is one radix-16 DFT in registers, a twiddle multiply, an exchange
// through the line's LDS slot and R-point DFTs (Cooley-Tukey with N = 16 x R):
//   X[k1 + 16 k2] = sum_j W_R^{j k2} W_N^{j k1} sum_k x[j + R k] W_16^{k k1}.
// The output stays in this "spectral" order, lane j holding k1 = j G + u
// (G = 16 / R, u < G) and k2 < R at register u R + k2.  Pointwise spectral
// multipliers only need the frequency of each register (spec()), and the
// inverse transform walks the same steps backwards, returning natural order.
// So a propagation FFT -> multiply -> IFFT never reorders data.
#pragma once

#include <hip/hip_runtime.h>

namespace imsp {

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b)
{
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
__device__ __forceinline__ float2 cmulc(float2 a, float2 b)
{
    return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
// conj(a) * b
__device__ __forceinline__ float2 cconjmul(float2 a, float2 b)
{
    return make_float2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ float cabs2(float2 a) { return a.x * a.x + a.y * a.y; }

// Returns x unchanged but hides its value from the optimiser, so that index
// arithmetic derived from it is recomputed where it is used instead of being
// hoisted out of the slice loop and kept live (which would spill).
__device__ __forceinline__ int opaque(int x)
{
    asm volatile("" : "+v"(x));
    return x;
}

// Orders LDS traffic between the lanes of one wavefront.
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// cos(2 pi e / 16) and sin(2 pi e / 16).
constexpr float kCos16[16] = {1.0f, 0.923879532511286756f, 0.707106781186547524f, 0.382683432365089772f,
                              0.0f, -0.382683432365089772f, -0.707106781186547524f, -0.923879532511286756f,
                              -1.0f, -0.923879532511286756f, -0.707106781186547524f, -0.382683432365089772f,
                              0.0f, 0.382683432365089772f, 0.707106781186547524f, 0.923879532511286756f};
constexpr float kSin16[16] = {0.0f, 0.382683432365089772f, 0.707106781186547524f, 0.923879532511286756f,
                              1.0f, 0.923879532511286756f, 0.707106781186547524f, 0.382683432365089772f,
                              0.0f, -0.382683432365089772f, -0.707106781186547524f, -0.923879532511286756f,
                              -1.0f, -0.923879532511286756f, -0.707106781186547524f, -0.382683432365089772f};

// a * W_16^E with W = exp(-2 pi i / 16) (forward) or exp(+2 pi i / 16) (INV).
template <int E, bool INV>
__device__ __forceinline__ float2 w16(float2 a)
{
    constexpr int e = E & 15;
    if constexpr (e == 0) {
        return a;
    } else if constexpr (e == 8) {
        return make_float2(-a.x, -a.y);
    } else if constexpr (e == 4) {             // -i forward, +i inverse
        return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
    } else if constexpr (e == 12) {            // +i forward, -i inverse
        return INV ? make_float2(a.y, -a.x) : make_float2(-a.y, a.x);
    } else {
        constexpr float c = kCos16[e];
        constexpr float s = INV ? kSin16[e] : -kSin16[e];
        return make_float2(a.x * c - a.y * s, a.x * s + a.y * c);
    }
}

template <bool INV>
__device__ __forceinline__ void dft2(float2 &a, float2 &b)
{
    float2 t = a;
    a = cadd(t, b);
    b = csub(t, b);
}

template <bool INV>
__device__ __forceinline__ void dft4(float2 &a0, float2 &a1, float2 &a2, float2 &a3)
{
    float2 t0 = cadd(a0, a2), t1 = csub(a0, a2);
    float2 t2 = cadd(a1, a3), t3 = w16<4, INV>(csub(a1, a3));
    a0 = cadd(t0, t2);
    a2 = csub(t0, t2);
    a1 = cadd(t1, t3);
    a3 = csub(t1, t3);
}

// 8-point DFT in natural order: radix-2 split into even and odd 4-point DFTs.
template <bool INV>
__device__ __forceinline__ void dft8(float2 *x)
{
    dft4<INV>(x[0], x[2], x[4], x[6]);
    dft4<INV>(x[1], x[3], x[5], x[7]);
    float2 e0 = x[0], e1 = x[2], e2 = x[4], e3 = x[6];
    float2 o0 = x[1], o1 = w16<2, INV>(x[3]), o2 = w16<4, INV>(x[5]), o3 = w16<6, INV>(x[7]);
    x[0] = cadd(e0, o0); x[4] = csub(e0, o0);
    x[1] = cadd(e1, o1); x[5] = csub(e1, o1);
    x[2] = cadd(e2, o2); x[6] = csub(e2, o2);
    x[3] = cadd(e3, o3); x[7] = csub(e3, o3);
}

// 16-point DFT in natural order as 4 x 4: input index n = 4 n1 + n2, output k = k1 + 4 k2,
//   X[k1 + 4 k2] = sum_n2 W_4^{n2 k2} W_16^{n2 k1} sum_n1 x[4 n1 + n2] W_4^{n1 k1}.
template <bool INV>
__device__ __forceinline__ void dft16(float2 *x)
{
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) dft4<INV>(x[n2], x[4 + n2], x[8 + n2], x[12 + n2]);
    // x[4 k1 + n2] now holds the inner sums; apply W_16^{n2 k1}
    x[5] = w16<1, INV>(x[5]);
    x[9] = w16<2, INV>(x[9]);
    x[13] = w16<3, INV>(x[13]);
    x[6] = w16<2, INV>(x[6]);
    x[10] = w16<4, INV>(x[10]);
    x[14] = w16<6, INV>(x[14]);
    x[7] = w16<3, INV>(x[7]);
    x[11] = w16<6, INV>(x[11]);
    x[15] = w16<9, INV>(x[15]);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) dft4<INV>(x[4 * k1], x[4 * k1 + 1], x[4 * k1 + 2], x[4 * k1 + 3]);
    float2 t[16];
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1)
#pragma unroll
        for (int k2 = 0; k2 < 4; ++k2) t[k1 + 4 * k2] = x[4 * k1 + k2];
#pragma unroll
    for (int i = 0; i < 16; ++i) x[i] = t[i];
}

template <int R, bool INV>
__device__ __forceinline__ void dft_small(float2 *x)
{
    if constexpr (R == 2) dft2<INV>(x[0], x[1]);
    else if constexpr (R == 4) dft4<INV>(x[0], x[1], x[2], x[3]);
    else if constexpr (R == 8) dft8<INV>(x);
    else if constexpr (R == 16) dft16<INV>(x);
}

// Geometry of a window of side N held by N * R lanes.
template <int N>
struct Win {
    static_assert(N == 16 || N == 32 || N == 64 || N == 128 || N == 256, "unsupported window");
    static constexpr int R = N / 16;        // lanes per line
    static constexpr int G = 16 / R;        // k1 values per lane after the exchange
    static constexpr int NT = N * R;        // lanes per window
    // LDS: line exchange slots of LD = N + R complex values (stride = R mod 16), and the
    // N x N transpose tiles; all are free of bank conflicts for the 64-bit accesses of a
    // wavefront (32 banks, 16 lanes per cycle).  In a slot, lane j writes its value k1 at
    // R k1 + k1 / G + j and reads (u, jj) back at 17 j + R u + jj (the same cell when
    // k1 = j G + u and jj is the writer): a per-lane base plus a constant on both sides.
    static constexpr int LD = N + R;
    static constexpr int LDS_WORDS = N * LD;            // complex values of LDS per window
    static constexpr int SWZ = (N == 64) ? 5 : 9;       // transpose swizzle multiplier
    __device__ static __forceinline__ int tpos(int y, int x) { return y * N + (x ^ ((SWZ * y) & 15)); }
    // twiddle table: W_N^{j k1} at j * 17 + k1 (rows padded to 17 so the lanes of a line hit distinct banks)
    static constexpr int TW_WORDS = R * 17;
    // natural position of register k along the owned axis
    __device__ static __forceinline__ int nat(int j, int k) { return j + R * k; }
    // frequency held by register i in spectral order
    __device__ static __forceinline__ int spec(int j, int i) { return (j * G + i / R) + 16 * (i % R); }
};

// Twiddles W_N^{j k1}, k1 = 1..15, of lane j from the table twg[j * 17 + k1].
template <int N>
__device__ __forceinline__ void load_twiddles(float2 (&tw)[16], const float2 *twg, int j)
{
    if constexpr (Win<N>::R > 1) {
        j = opaque(j);
#pragma unroll
        for (int k1 = 1; k1 < 16; ++k1) tw[k1] = twg[j * 17 + k1];
    }
}

// Forward DFT (unnormalised) of the line owned by lanes j = 0..R-1; natural -> spectral.
// tw from load_twiddles; xb is the line's LDS slot (N complex values).
template <int N>
__device__ __forceinline__ void line_fft_fwd(float2 (&v)[16], const float2 (&tw)[16], float2 *xb, int j)
{
    constexpr int R = Win<N>::R, G = Win<N>::G;
    dft16<false>(v);
    if constexpr (R > 1) {
#pragma unroll
        for (int k1 = 1; k1 < 16; ++k1) v[k1] = cmul(v[k1], tw[k1]);
        float2 *wb = xb + opaque(j);
#pragma unroll
        for (int k1 = 0; k1 < 16; ++k1) wb[k1 * R + k1 / G] = v[k1];
        wave_sync();
        const float2 *rb = xb + 17 * opaque(j);
#pragma unroll
        for (int u = 0; u < G; ++u)
#pragma unroll
            for (int jj = 0; jj < R; ++jj) v[u * R + jj] = rb[u * R + jj];
        wave_sync();
#pragma unroll
        for (int u = 0; u < G; ++u) dft_small<R, false>(&v[u * R]);
    }
}

// Inverse DFT without the 1/N factor; spectral -> natural.
template <int N>
__device__ __forceinline__ void line_fft_inv(float2 (&v)[16], const float2 (&tw)[16], float2 *xb, int j)
{
    constexpr int R = Win<N>::R, G = Win<N>::G;
    if constexpr (R > 1) {
#pragma unroll
        for (int u = 0; u < G; ++u) dft_small<R, true>(&v[u * R]);
        float2 *rb = xb + 17 * opaque(j);
#pragma unroll
        for (int u = 0; u < G; ++u)
#pragma unroll
            for (int jj = 0; jj < R; ++jj) rb[u * R + jj] = v[u * R + jj];
        wave_sync();
        const float2 *wb = xb + opaque(j);
#pragma unroll
        for (int k1 = 0; k1 < 16; ++k1) v[k1] = wb[k1 * R + k1 / G];
        wave_sync();
#pragma unroll
        for (int k1 = 1; k1 < 16; ++k1) v[k1] = cmulc(v[k1], tw[k1]);
    }
    dft16<true>(v);
}

// Same with the twiddles read from the table on the way (short register lifetime).
template <int N>
__device__ __forceinline__ void line_fft_fwd(float2 (&v)[16], const float2 *twg, float2 *xb, int j)
{
    float2 tw[16];
    load_twiddles<N>(tw, twg, j);
    line_fft_fwd<N>(v, tw, xb, j);
}

template <int N>
__device__ __forceinline__ void line_fft_inv(float2 (&v)[16], const float2 *twg, float2 *xb, int j)
{
    float2 tw[16];
    load_twiddles<N>(tw, twg, j);
    line_fft_inv<N>(v, tw, xb, j);
}

// Moves the window between the two layouts through LDS.  ROW: lane (line = y, j)
// owns x = j + R k; COL: lane (line = x, j) owns y = j + R k.  SPEC_IN / SPEC_OUT
// select spectral instead of natural positions along the owned axis.
template <int N, bool FROM_ROW, bool SPEC_IN, bool SPEC_OUT>
__device__ __forceinline__ void transpose(float2 (&v)[16], float2 *lds, int line, int j)
{
    using W = Win<N>;
    line = opaque(line);
    j = opaque(j);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        int a = SPEC_IN ? W::spec(j, i) : W::nat(j, i);
        if (FROM_ROW) lds[W::tpos(line, a)] = v[i];
        else lds[W::tpos(a, line)] = v[i];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        int b = SPEC_OUT ? W::spec(j, i) : W::nat(j, i);
        if (FROM_ROW) v[i] = lds[W::tpos(b, line)];
        else v[i] = lds[W::tpos(line, b)];
    }
    __syncthreads();
}

// Natural-order transpose for R >= 4 through the tile T(y, x) = y LD + (x ^ (y mod R)): the
// xor touches only the bits of x that the lane index fixes, so every access is a per-lane
// base plus a constant, and both sides are free of bank conflicts.
template <int N, bool FROM_ROW>
__device__ __forceinline__ void transpose_nat(float2 (&v)[16], float2 *lds, int line, int j)
{
    using W = Win<N>;
    constexpr int R = W::R, LD = W::LD;
    static_assert(R >= 4, "the constant-offset tile needs at least 4 lanes a line");
    line = opaque(line);
    j = opaque(j);
    float2 *row_base = lds + line * LD + (j ^ (line % R));   // lane owns row y = line
    float2 *col_base = lds + j * LD + (line ^ j);            // lane owns column x = line
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        if (FROM_ROW) row_base[R * i] = v[i];
        else col_base[R * LD * i] = v[i];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        if (FROM_ROW) v[i] = col_base[R * LD * i];
        else v[i] = row_base[R * i];
    }
    __syncthreads();
}

}  // namespace imsp
