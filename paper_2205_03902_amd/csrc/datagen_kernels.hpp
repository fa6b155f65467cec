// Training-data generation on the device: random lattice specimens, Poisson detector
// noise, and the crops that connect the multislice reconstruction to the network.
//
// Random numbers come from Philox4x32-10 (Salmon, Moraes, Dror and Shaw, "Parallel random
// numbers: as easy as 1, 2, 3", SC 2011): a counter-based generator, so every atom and every
// detector pixel draws from its own counter and no state is carried between lanes.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace datagen {

struct U4 {
    uint32_t x, y, z, w;
};

// Ten rounds of the Philox 4x32 bijection: two 32 x 32 -> 64-bit products per round with the
// published multipliers, the key advanced by the published Weyl constants between rounds.
__device__ __forceinline__ U4 philox(U4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        c = U4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// Uniform in [0, 1) with 32 random bits (FP64, exact).
__device__ __forceinline__ double unit(uint32_t r) { return (double)r * (1.0 / 4294967296.0); }

// Counter tags of the specimen streams.
constexpr uint32_t kTagSpecimen = 0xFFFFFFFFu;   // (tag, 0, 0, 0): lattice constant, vacancy rate
constexpr uint32_t kTagOrigin = 0xFFFFFFFEu;     // (tag, slice, 0, 0): lattice origin of a slice
constexpr uint32_t kTagAtom = 1u;                // (i, j, slice, tag): one lattice site

struct SpecimenParams {
    int M, H, W;              // slices, object pixels
    double dx;                // pixel size (A)
    double sigma;             // Gaussian atom radius (A)
    double jitter;            // site jitter standard deviation (A), truncated at 4 sigma
    double a_min, a_max;      // lattice constant range (A)
    double vacancy_max;       // vacancy rate ~ U[0, vacancy_max]
    int two_species;          // heavy species (amplitude x 2) with probability 1/2
    uint32_t key0, key1;      // specimen key (seed, specimen index)
};

struct Lattice {
    double a, vac;
};

__device__ __forceinline__ Lattice lattice_of(const SpecimenParams &p)
{
    const U4 r = philox(U4{kTagSpecimen, 0u, 0u, 0u}, p.key0, p.key1);
    return Lattice{p.a_min + (p.a_max - p.a_min) * unit(r.x), p.vacancy_max * unit(r.y)};
}

// One lattice site: position (unwrapped, A), amplitude (0 for a vacancy).
__device__ __forceinline__ void site(const SpecimenParams &p, const Lattice &lt, double y0, double x0, int m, int i,
                                     int j, double &py, double &px, double &amp)
{
    const U4 r = philox(U4{(uint32_t)i, (uint32_t)j, (uint32_t)m, kTagAtom}, p.key0, p.key1);
    // Box-Muller on (0, 1] x [0, 1), clamped to 4 standard deviations
    const double rho = sqrt(-2.0 * log((double)(r.x + 1.0) * (1.0 / 4294967296.0)));
    const double th = 6.283185307179586 * unit(r.y);
    const double lim = 4.0 * p.jitter;
    const double jy = fmin(fmax(p.jitter * rho * cos(th), -lim), lim);
    const double jx = fmin(fmax(p.jitter * rho * sin(th), -lim), lim);
    py = y0 + i * lt.a + jy;
    px = x0 + j * lt.a + jx;
    amp = 0.5 + unit(r.z);
    if (p.two_species && (r.w >> 31)) amp *= 2.0;
    if ((double)(r.w & 0xFFFFFFu) * (1.0 / 16777216.0) < lt.vac) amp = 0.0;
}

// V[m][y][x] = sum over sites of A exp(-|r - r_a|^2 / (2 sigma^2)) over the periodic object,
// each site counted once at its image nearest the pixel, sites farther than 5 sigma along y
// or x left out.  One lane per pixel: the lane enumerates the few lattice cells that can
// reach it, so the sum needs no atomics and is deterministic.  Optionally also writes the
// pure-phase transmission exp(i kappa V).
__global__ __launch_bounds__(256) void specimen_kernel(SpecimenParams p, double kappa, float *__restrict__ potential,
                                float2 *__restrict__ slices)
{
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long plane = (long long)p.H * p.W;
    if (idx >= plane * p.M) return;
    const int m = (int)(idx / plane);
    const int rem = (int)(idx - (long long)m * plane);
    const int yy = rem / p.W, xx = rem - (rem / p.W) * p.W;
    const Lattice lt = lattice_of(p);
    const U4 o = philox(U4{kTagOrigin, (uint32_t)m, 0u, 0u}, p.key0, p.key1);
    const double y0 = lt.a * unit(o.x), x0 = lt.a * unit(o.y);
    const double Ly = p.H * p.dx, Lx = p.W * p.dx;
    const int ny = (int)ceil((Ly - y0) / lt.a), nx = (int)ceil((Lx - x0) / lt.a);
    const double cut = 5.0 * p.sigma, reach = cut + 4.0 * p.jitter;
    const double Y = yy * p.dx, X = xx * p.dx;
    const double inv2s2 = 1.0 / (2.0 * p.sigma * p.sigma);
    double v = 0.0;
    for (int ky = -1; ky <= 1; ++ky) {
        const double ty = Y - ky * Ly - y0;
        const int i0 = max(0, (int)ceil((ty - reach) / lt.a)), i1 = min(ny - 1, (int)floor((ty + reach) / lt.a));
        for (int i = i0; i <= i1; ++i) {
            for (int kx = -1; kx <= 1; ++kx) {
                const double tx = X - kx * Lx - x0;
                const int j0 = max(0, (int)ceil((tx - reach) / lt.a)), j1 = min(nx - 1, (int)floor((tx + reach) / lt.a));
                for (int j = j0; j <= j1; ++j) {
                    double py, px, amp;
                    site(p, lt, y0, x0, m, i, j, py, px, amp);
                    const double dy = py + ky * Ly - Y, dxx = px + kx * Lx - X;
                    if (amp == 0.0 || fabs(dy) > cut || fabs(dxx) > cut) continue;
                    v += amp * exp(-(dy * dy + dxx * dxx) * inv2s2);
                }
            }
        }
    }
    if (potential) potential[idx] = (float)v;
    if (slices) {
        double s, c;
        sincos(kappa * v, &s, &c);
        slices[idx] = make_float2((float)c, (float)s);
    }
}

// Counts ~ Poisson(dose * I / n_pix) per detector pixel, returned as counts * n_pix / dose.
// Mean below 10: inversion (sequential search over the cumulative distribution);
// otherwise the transformed rejection with squeeze of Hormann (1993, "The transformed
// rejection method for generating Poisson random variables", PTRS).  Each pixel draws from
// the counters (pixel, block); attempts are capped (the acceptance rate is above 0.9, so the
// cap is never reached in practice; at the cap the mode is returned).
__device__ __forceinline__ double poisson_draw(double lam, uint32_t k0, uint32_t k1, uint32_t plo, uint32_t phi)
{
    uint32_t block = 0;
    U4 r = philox(U4{plo, phi, block, 0u}, k0, k1);
    if (lam < 10.0) {
        const double u = unit(r.x);
        double p = exp(-lam), F = p;
        int k = 0;
        while (u > F && k < 1000) {
            ++k;
            p *= lam / k;
            F += p;
        }
        return k;
    }
    const double slam = sqrt(lam), loglam = log(lam);
    const double b = 0.931 + 2.53 * slam;
    const double a = -0.059 + 0.02483 * b;
    const double invalpha = 1.1239 + 1.1328 / (b - 3.4);
    const double vr = 0.9277 - 3.6224 / (b - 2.0);
    for (int attempt = 0; attempt < 64; ++attempt) {
        const int slot = attempt & 1;
        if (attempt > 0 && slot == 0) r = philox(U4{plo, phi, ++block, 0u}, k0, k1);
        const double U = unit(slot ? r.z : r.x) - 0.5;
        const double V = unit(slot ? r.w : r.y);
        const double us = 0.5 - fabs(U);
        const double k = floor((2.0 * a / us + b) * U + lam + 0.43);
        if (us >= 0.07 && V <= vr) return k;
        if (k < 0.0 || (us < 0.013 && V > us)) continue;
        if (log(V) + log(invalpha) - log(a / (us * us) + b) <= -lam + k * loglam - lgamma(k + 1.0)) return k;
    }
    return floor(lam);
}

__global__ __launch_bounds__(256) void poisson_kernel(const float *__restrict__ intensity, long long count, double scale, double inv_scale,
                               uint32_t k0, uint32_t k1, float *__restrict__ out)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const double lam = fmax((double)intensity[i], 0.0) * scale;
    const double k = lam > 0.0 ? poisson_draw(lam, k0, k1, (uint32_t)i, (uint32_t)(i >> 32)) : 0.0;
    out[i] = (float)(k * inv_scale);
}

// Network input from reconstructed slices: phase of every slice over a crop, bf16 NHWC with
// in_pad channels (zeros past M).
__global__ void crop_phase_kernel(const float2 *__restrict__ slices, int M, int H, int W, int y0, int x0, int h,
                                  int w, int in_pad, uint16_t *__restrict__ out)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long long)h * w * in_pad) return;
    const int c = (int)(i % in_pad);
    const long long px = i / in_pad;
    const int y = (int)(px / w), x = (int)(px - (long long)(px / w) * w);
    float v = 0.0f;
    if (c < M) {
        const float2 t = slices[((long long)c * H + (y0 + y) % H) * W + (x0 + x) % W];
        v = atan2f(t.y, t.x);
    }
    uint32_t u = __float_as_uint(v);
    u += 0x7fffu + ((u >> 16) & 1u);
    out[i] = (uint16_t)(u >> 16);
}

// Training target: the potential over the same crop, float NHWC with M channels.
__global__ void crop_potential_kernel(const float *__restrict__ potential, int M, int H, int W, int y0, int x0, int h,
                                      int w, float *__restrict__ out)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long long)h * w * M) return;
    const int c = (int)(i % M);
    const long long px = i / M;
    const int y = (int)(px / w), x = (int)(px - (long long)(px / w) * w);
    out[i] = potential[((long long)c * H + (y0 + y) % H) * W + (x0 + x) % W];
}

// Learned initialisation: t = exp(i kappa V_hat) over the crop, the slices unchanged elsewhere.
__global__ void apply_init_kernel(const float *__restrict__ vhat, int M, int H, int W, int y0, int x0, int h, int w,
                                  float kappa, float2 *__restrict__ slices)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long long)h * w * M) return;
    const int c = (int)(i % M);
    const long long px = i / M;
    const int y = (int)(px / w), x = (int)(px - (long long)(px / w) * w);
    float s, co;
    sincosf(kappa * vhat[i], &s, &co);
    slices[((long long)c * H + (y0 + y) % H) * W + (x0 + x) % W] = make_float2(co, s);
}

}  // namespace datagen
