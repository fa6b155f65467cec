/*
 * FP64 CPU oracle for layer-wise inverse multislice ptychography, arXiv 2205.03902.
 *
 * TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU
 * baseline of the benchmark call it; the product path never does.  It shares
 * no code with the GPU library.  Conventions are stated in oracle.h.
 *
 * Nothing here is blocked, fused or reordered beyond what the paper's
 * definitions state: one scan position at a time, one slice at a time, one
 * 2D DFT at a time.  OpenMP only splits the positions over threads; each
 * thread sums its positions in ascending order into a private buffer and the
 * buffers are added in thread order, so a result depends only on the thread
 * count.
 */
#include "oracle.h"

#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

static const double PI = 3.14159265358979323846264338327950288;

static int is_pow2(int n) { return n >= 1 && (n & (n - 1)) == 0; }
static long wrap(long i, long n) { long r = i % n; return r < 0 ? r + n : r; }

int orc_max_threads(void) { return omp_get_max_threads(); }

/* ------------------------------------------------------------------ */
/* Physics constants, Sec. 5.3.2: lambda = h c / sqrt(e^2 U^2 + 2 e U m c^2). */
double orc_wavelength(double volts)
{
    const double h = 6.62607015e-34;      /* Planck constant (J s), exact SI       */
    const double c = 299792458.0;         /* speed of light (m/s), exact SI         */
    const double e = 1.602176634e-19;     /* elementary charge (C), exact SI        */
    const double m = 9.1093837015e-31;    /* electron rest mass (kg), CODATA 2018   */
    double eu = e * volts;
    return h * c / sqrt(eu * eu + 2.0 * eu * m * c * c) * 1e10;
}

/* ------------------------------------------------------------------ */
/* Fourier transforms (Sec. 1.3: F is the discrete 2D Fourier transform). */

void orc_dft1d(const double complex *in, double complex *out, int n, int sign)
{
    for (int k = 0; k < n; ++k) {
        double complex acc = 0.0;
        for (int j = 0; j < n; ++j) {
            long jk = ((long)j * k) % n;   /* reduce the angle exactly before scaling */
            double a = sign * 2.0 * PI * (double)jk / (double)n;
            acc += in[j] * (cos(a) + I * sin(a));
        }
        out[k] = acc;
    }
}

/* Iterative radix-2 Cooley-Tukey: bit-reversal permutation, then log2(n)
 * butterfly stages.  Each twiddle is evaluated directly from cos/sin. */
int orc_fft1d(double complex *x, int n, int sign)
{
    if (!is_pow2(n)) return -1;
    for (int i = 1, j = 0; i < n; ++i) {
        int bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) { double complex t = x[i]; x[i] = x[j]; x[j] = t; }
    }
    for (int len = 2; len <= n; len <<= 1) {
        int half = len / 2;
        for (int start = 0; start < n; start += len) {
            for (int k = 0; k < half; ++k) {
                double a = sign * 2.0 * PI * (double)k / (double)len;
                double complex w = cos(a) + I * sin(a);
                double complex u = x[start + k];
                double complex v = x[start + k + half] * w;
                x[start + k] = u + v;
                x[start + k + half] = u - v;
            }
        }
    }
    return 0;
}

int orc_fft2d(double complex *x, int n, int sign)
{
    if (!is_pow2(n)) return -1;
    double complex *col = (double complex *)malloc(sizeof(double complex) * (size_t)n);
    if (!col) return -2;
    for (int y = 0; y < n; ++y) orc_fft1d(x + (size_t)y * n, n, sign);
    for (int xx = 0; xx < n; ++xx) {
        for (int y = 0; y < n; ++y) col[y] = x[(size_t)y * n + xx];
        orc_fft1d(col, n, sign);
        for (int y = 0; y < n; ++y) x[(size_t)y * n + xx] = col[y];
    }
    free(col);
    return 0;
}

static void ifft2_normalised(double complex *x, int n)
{
    orc_fft2d(x, n, +1);
    double s = 1.0 / ((double)n * (double)n);
    for (size_t i = 0; i < (size_t)n * n; ++i) x[i] *= s;
}

void orc_fftfreq(int n, double d, double *q)
{
    for (int i = 0; i < n; ++i) {
        int k = (i < (n + 1) / 2) ? i : i - n;
        q[i] = (double)k / ((double)n * d);
    }
}

static int signed_k(int i, int n) { return (i < (n + 1) / 2) ? i : i - n; }

/* ------------------------------------------------------------------ */
/* Fresnel propagator, eq. (fresnel_element):
 * h = exp(-pi i dz lambda ((qy^2 + qx^2) + 2 (qx sin(tx) / lambda + qy sin(ty) / lambda))). */
void orc_propagator(int n, double dx, double lambda, double dz, double tilt_y, double tilt_x,
                    double complex *h)
{
    double *q = (double *)malloc(sizeof(double) * (size_t)n);
    orc_fftfreq(n, dx, q);
    for (int y = 0; y < n; ++y) {
        for (int x = 0; x < n; ++x) {
            double arg = (q[y] * q[y] + q[x] * q[x])
                       + 2.0 * (q[x] * sin(tilt_x) / lambda + q[y] * sin(tilt_y) / lambda);
            double ph = -PI * dz * lambda * arg;
            h[(size_t)y * n + x] = cos(ph) + I * sin(ph);
        }
    }
    free(q);
}

/* Probe, Sec. 2.1 and the caption of Fig. 3: the Airy probe is the inverse
 * Fourier transform of a circular aperture.  The aperture is the disk
 * lambda |q| <= alpha (boundary included); a defocus multiplies it by the
 * propagator of the same equation with distance `defocus`; the factor
 * (-1)^(ky + kx) moves the probe centre from (0, 0) to (n/2, n/2); the result
 * is scaled to unit energy. */
int orc_probe_aberrated(int n, double dx, double lambda, double alpha, double c1, double a1, double phi_a1,
                        double c3, double complex *p)
{
    if (!is_pow2(n) || n < 2) return -1;
    double *q = (double *)malloc(sizeof(double) * (size_t)n);
    orc_fftfreq(n, dx, q);
    for (int y = 0; y < n; ++y) {
        for (int x = 0; x < n; ++x) {
            double q2 = q[y] * q[y] + q[x] * q[x];
            double complex a = 0.0;
            if (lambda * sqrt(q2) <= alpha) {
                /* chi = pi lambda C1 q^2 + pi lambda A1 q^2 cos 2(phi - phi_A1) + pi/2 lambda^3 C3 q^4,
                 * the aperture multiplied by exp(-i chi) (C1 alone: the propagator of eq.
                 * fresnel_element over the defocus distance) */
                double phi = atan2(q[y], q[x]);
                double chi = PI * lambda * c1 * q2 + PI * lambda * a1 * q2 * cos(2.0 * (phi - phi_a1))
                             + 0.5 * PI * lambda * lambda * lambda * c3 * q2 * q2;
                a = cos(chi) - I * sin(chi);
                if ((x + y) & 1) a = -a;
            }
            p[(size_t)y * n + x] = a;
        }
    }
    free(q);
    orc_fft2d(p, n, +1);
    double e = 0.0;
    for (size_t i = 0; i < (size_t)n * n; ++i) e += creal(p[i]) * creal(p[i]) + cimag(p[i]) * cimag(p[i]);
    if (e <= 0.0) return -1;
    double s = 1.0 / sqrt(e);
    for (size_t i = 0; i < (size_t)n * n; ++i) p[i] *= s;
    return 0;
}

int orc_probe(int n, double dx, double lambda, double alpha, double defocus, double complex *p)
{
    if (!is_pow2(n) || n < 2) return -1;
    double *q = (double *)malloc(sizeof(double) * (size_t)n);
    orc_fftfreq(n, dx, q);
    for (int y = 0; y < n; ++y) {
        for (int x = 0; x < n; ++x) {
            double q2 = q[y] * q[y] + q[x] * q[x];
            double complex a = 0.0;
            if (lambda * sqrt(q2) <= alpha) {
                double ph = -PI * defocus * lambda * q2;
                a = cos(ph) + I * sin(ph);
                if ((x + y) & 1) a = -a;
            }
            p[(size_t)y * n + x] = a;
        }
    }
    free(q);
    orc_fft2d(p, n, +1);
    double e = 0.0;
    for (size_t i = 0; i < (size_t)n * n; ++i) e += creal(p[i]) * creal(p[i]) + cimag(p[i]) * cimag(p[i]);
    if (e <= 0.0) return -1;
    double s = 1.0 / sqrt(e);
    for (size_t i = 0; i < (size_t)n * n; ++i) p[i] *= s;
    return 0;
}

/* Shift by a fraction of a pixel, p_{y,x} -> p_{y - fy, x - fx} (Sec. 2.1), as a
 * phase ramp in Fourier space with signed frequencies. */
static int shift_with_sign(const double complex *p, int n, double fy, double fx, double complex *out, double sgn)
{
    if (!is_pow2(n)) return -1;
    size_t n2 = (size_t)n * n;
    memcpy(out, p, sizeof(double complex) * n2);
    if (fy == 0.0 && fx == 0.0) return 0;
    orc_fft2d(out, n, -1);
    for (int y = 0; y < n; ++y) {
        for (int x = 0; x < n; ++x) {
            double ph = sgn * -2.0 * PI * ((double)signed_k(y, n) * fy + (double)signed_k(x, n) * fx) / (double)n;
            out[(size_t)y * n + x] *= cos(ph) + I * sin(ph);
        }
    }
    ifft2_normalised(out, n);
    return 0;
}

int orc_shift(const double complex *p, int n, double fy, double fx, double complex *out)
{
    return shift_with_sign(p, n, fy, fx, out, +1.0);
}

int orc_unshift(const double complex *g, int n, double fy, double fx, double complex *out)
{
    return shift_with_sign(g, n, fy, fx, out, -1.0);
}

/* ------------------------------------------------------------------ */
/* The forward multislice model of Sec. 2.1 for one position.               */

typedef struct {
    const orc_problem *pb;
    double complex *h;      /* (M-1) x n x n propagators */
} model;

static int check_problem(const orc_problem *pb)
{
    if (!pb || !is_pow2(pb->n) || pb->n < 2) return -1;
    if (pb->obj_h < pb->n || pb->obj_w < pb->n || pb->n_slices < 1 || pb->n_pos < 0) return -1;
    if (pb->n_pos > 0 && !pb->positions) return -1;
    if (pb->n_slices > 1 && !pb->dz) return -1;
    if (!(pb->pixel_size > 0.0) || !(pb->wavelength > 0.0)) return -1;
    if (pb->objective != ORC_AMPLITUDE && pb->objective != ORC_POISSON) return -1;
    return 0;
}

static int model_init(model *md, const orc_problem *pb)
{
    md->pb = pb;
    size_t n2 = (size_t)pb->n * pb->n;
    int ng = pb->n_slices - 1;
    md->h = NULL;
    if (ng > 0) {
        md->h = (double complex *)malloc(sizeof(double complex) * n2 * (size_t)ng);
        if (!md->h) return -2;
        for (int g = 0; g < ng; ++g)
            orc_propagator(pb->n, pb->pixel_size, pb->wavelength, pb->dz[g], pb->tilt_y, pb->tilt_x,
                           md->h + (size_t)g * n2);
    }
    return 0;
}

static void model_free(model *md) { free(md->h); }

static void position_origin(const orc_problem *pb, long s, long *iy, long *ix, double *fy, double *fx)
{
    double py = pb->positions[2 * s], px = pb->positions[2 * s + 1];
    double fly = floor(py), flx = floor(px);
    *iy = (long)fly; *ix = (long)flx;
    *fy = py - fly; *fx = px - flx;
}

/* The object patch T_m^s: t_m[(iy + i) mod H][(ix + j) mod W] (indices wrap around). */
static void gather_patch(const orc_problem *pb, const double complex *slice, long iy, long ix, double complex *t)
{
    int n = pb->n;
    for (int i = 0; i < n; ++i) {
        long y = wrap(iy + i, pb->obj_h);
        for (int j = 0; j < n; ++j) {
            long x = wrap(ix + j, pb->obj_w);
            t[(size_t)i * n + j] = slice[(size_t)y * pb->obj_w + x];
        }
    }
}

/* V_z(E) = F^{-1}(F(E) o H), Sec. 2.1; conj_h applies the adjoint G^H = F^{-1} diag(conj h) F. */
static void propagate(double complex *e, const double complex *h, int n, int conj_h)
{
    orc_fft2d(e, n, -1);
    for (size_t i = 0; i < (size_t)n * n; ++i) e[i] *= conj_h ? conj(h[i]) : h[i];
    ifft2_normalised(e, n);
}

/* Incident waves psi[m] (the wave arriving at slice m; psi[0] is the shifted probe)
 * and the far field Psi = F E_M.  E_1 = P^s o X_1, E_m = V(E_{m-1}) o X_m, I = |F E_M|^2. */
static void forward_one(const model *md, long s, const double complex *probe, const double complex *slices,
                        double complex *psi, double complex *far, double complex *tpatch)
{
    const orc_problem *pb = md->pb;
    int n = pb->n, M = pb->n_slices;
    size_t n2 = (size_t)n * n, hw = (size_t)pb->obj_h * pb->obj_w;
    long iy, ix; double fy, fx;
    position_origin(pb, s, &iy, &ix, &fy, &fx);
    orc_shift(probe, n, fy, fx, psi);
    for (int m = 0; m < M; ++m) {
        gather_patch(pb, slices + (size_t)m * hw, iy, ix, tpatch);
        double complex *e = (m + 1 < M) ? psi + (size_t)(m + 1) * n2 : far;
        for (size_t i = 0; i < n2; ++i) e[i] = psi[(size_t)m * n2 + i] * tpatch[i];
        if (m + 1 < M) propagate(e, md->h + (size_t)m * n2, n, 0);
        else orc_fft2d(e, n, -1);
    }
}

int orc_forward(const orc_problem *pb, const double complex *probe, const double complex *slices,
                double *intensity, double complex *exit_waves)
{
    if (check_problem(pb) || !probe || !slices) return -1;
    model md;
    if (model_init(&md, pb)) return -2;
    int n = pb->n, M = pb->n_slices;
    size_t n2 = (size_t)n * n;
    int nt = pb->n_threads > 0 ? pb->n_threads : omp_get_max_threads();
    int bad = 0;
#pragma omp parallel num_threads(nt)
    {
        double complex *psi = (double complex *)malloc(sizeof(double complex) * n2 * (size_t)M);
        double complex *far = (double complex *)malloc(sizeof(double complex) * n2);
        double complex *tp = (double complex *)malloc(sizeof(double complex) * n2);
        if (!psi || !far || !tp) {
#pragma omp atomic write
            bad = 1;
        } else {
            int t = omp_get_thread_num();
            long lo = pb->n_pos * t / nt, hi = pb->n_pos * (t + 1) / nt;
            for (long s = lo; s < hi; ++s) {
                forward_one(&md, s, probe, slices, psi, far, tp);
                if (exit_waves) {
                    /* E_M = F^{-1} Psi */
                    double complex *ew = exit_waves + (size_t)s * n2;
                    memcpy(ew, far, sizeof(double complex) * n2);
                    ifft2_normalised(ew, n);
                }
                if (intensity)
                    for (size_t i = 0; i < n2; ++i)
                        intensity[(size_t)s * n2 + i] = creal(far[i]) * creal(far[i]) + cimag(far[i]) * cimag(far[i]);
            }
        }
        free(psi); free(far); free(tp);
    }
    model_free(&md);
    return bad ? -2 : 0;
}

/* ------------------------------------------------------------------ */
/* Loss and generalised Wirtinger gradients, Sec. 3.2:
 *   grad A(z) = Q^H (Q z - (Q z / |Q z|) o sqrt(y)), phase := 0 where (Q z)_k = 0.
 * Here Q z = Psi = F E_M, so the residual r = Psi - sqrt(I) Psi/|Psi| is pulled
 * back through the chain E_M = O_M G_{M-1} ... G_1 O_1 p^s (eq. exit_wave_mslices):
 *   F^H r, then for m = M..1:  dL/dconj(t_m) += conj(psi_m) o g,
 *   g <- conj(T_m) o g, g <- G_{m-1}^H g. */

typedef struct {
    double complex *gs;    /* slice gradient accumulator (M x H x W or H x W) */
    double complex *gp;    /* probe gradient accumulator (n x n)              */
    double *w;             /* overlap accumulator (H x W)                     */
    double *gpos, *cpos;   /* per-position gradient and curvature bound (S x 2), each s written once */
    double tprod;          /* prod_m max |t_m|^2 (for cpos)                   */
    double loss;
} accum;

/* Derivative of the shifted probe P(y, x) = p(y - fy, x - fx) of orc_shift in its shift along
 * `axis` (0: fy, 1: fx): the phase ramp e^{-2 pi i (k_y fy + k_x fx) / n} differentiated,
 * i.e. multiplied by -2 pi i k / n with the same signed frequencies. */
static void shift_derivative(const double complex *p, int n, double fy, double fx, int axis, double complex *out)
{
    size_t n2 = (size_t)n * n;
    memcpy(out, p, sizeof(double complex) * n2);
    orc_fft2d(out, n, -1);
    for (int y = 0; y < n; ++y) {
        for (int x = 0; x < n; ++x) {
            double ky = (double)signed_k(y, n), kx = (double)signed_k(x, n);
            double ph = -2.0 * PI * (ky * fy + kx * fx) / (double)n;
            double k = axis == 0 ? ky : kx;
            out[(size_t)y * n + x] *= (cos(ph) + I * sin(ph)) * (-2.0 * PI * I * k / (double)n);
        }
    }
    ifft2_normalised(out, n);
}

static void loss_grad_one(const model *md, long s, const double complex *probe, const double complex *slices,
                          const double *measured, int layer, int want_slices, int want_probe, accum *ac,
                          double complex *psi, double complex *far, double complex *tp, double complex *g,
                          double complex *tmp)
{
    const orc_problem *pb = md->pb;
    int n = pb->n, M = pb->n_slices;
    size_t n2 = (size_t)n * n, hw = (size_t)pb->obj_h * pb->obj_w;
    long iy, ix; double fy, fx;
    position_origin(pb, s, &iy, &ix, &fy, &fx);
    forward_one(md, s, probe, slices, psi, far, tp);

    const double *meas = measured + (size_t)s * n2;
    double loss = 0.0;
    if (pb->objective == ORC_POISSON) {
        /* deviance |Psi|^2 - I + I log(I / |Psi|^2), residual Psi (1 - I / |Psi|^2) */
        for (size_t k = 0; k < n2; ++k) {
            double a2 = creal(far[k]) * creal(far[k]) + cimag(far[k]) * cimag(far[k]);
            double y = meas[k];
            if (a2 == 0.0) {
                g[k] = far[k];
                continue;
            }
            loss += a2 - y + (y > 0.0 ? y * log(y / a2) : 0.0);
            g[k] = far[k] * (1.0 - y / a2);
        }
    } else {
        for (size_t k = 0; k < n2; ++k) {
            double a = cabs(far[k]);
            double sq = sqrt(meas[k]);
            double d = sq - a;
            loss += d * d;
            g[k] = (a == 0.0) ? far[k] : far[k] - sq * (far[k] / a);
        }
    }
    ac->loss += loss;

    /* F^H r = N^2 F^{-1} r: the unnormalised conjugate transform. */
    orc_fft2d(g, n, +1);

    int m_stop = (layer >= 0) ? layer : 0;
    for (int m = M - 1; m >= m_stop; --m) {
        const double complex *pm = psi + (size_t)m * n2;
        if (want_slices && (layer < 0 || layer == m)) {
            double complex *dst = ac->gs + (layer < 0 ? (size_t)m * hw : 0);
            for (int i = 0; i < n; ++i) {
                long y = wrap(iy + i, pb->obj_h);
                for (int j = 0; j < n; ++j) {
                    long x = wrap(ix + j, pb->obj_w);
                    dst[(size_t)y * pb->obj_w + x] += conj(pm[(size_t)i * n + j]) * g[(size_t)i * n + j];
                }
            }
        }
        if (layer == m && ac->w) {
            for (int i = 0; i < n; ++i) {
                long y = wrap(iy + i, pb->obj_h);
                for (int j = 0; j < n; ++j) {
                    long x = wrap(ix + j, pb->obj_w);
                    double complex v = pm[(size_t)i * n + j];
                    ac->w[(size_t)y * pb->obj_w + x] += creal(v) * creal(v) + cimag(v) * cimag(v);
                }
            }
        }
        if (m == m_stop && !(m == 0 && want_probe)) break;
        gather_patch(pb, slices + (size_t)m * hw, iy, ix, tp);
        for (size_t k = 0; k < n2; ++k) g[k] *= conj(tp[k]);
        if (m > 0) propagate(g, md->h + (size_t)(m - 1) * n2, n, 1);
    }
    if (want_probe && m_stop == 0) {
        /* g = dL/dconj(P^s), the gradient with respect to the shifted probe */
        if (ac->gpos) {
            /* the window sits at origin + (fy, fx): moving the position moves the probe's shift, so
             * dL/dp = 2 Re sum conj(g) dP^s/df; the second derivative along an axis is at most
             * 2 ||Q||^2 ||dP^s/df||^2 with ||Q||^2 <= N^2 prod_m max |t_m|^2 (every G_m unitary) */
            for (int axis = 0; axis < 2; ++axis) {
                shift_derivative(probe, n, fy, fx, axis, tmp);
                double gr = 0.0, nrm = 0.0;
                for (size_t k = 0; k < n2; ++k) {
                    gr += creal(conj(g[k]) * tmp[k]);
                    nrm += creal(tmp[k]) * creal(tmp[k]) + cimag(tmp[k]) * cimag(tmp[k]);
                }
                ac->gpos[2 * s + axis] = 2.0 * gr;
                if (ac->cpos) ac->cpos[2 * s + axis] = 2.0 * (double)n2 * ac->tprod * nrm;
            }
        }
        if (ac->gp) {
            orc_unshift(g, n, fy, fx, tmp);
            for (size_t k = 0; k < n2; ++k) ac->gp[k] += tmp[k];
        }
    }
}

static int loss_grad_impl(const orc_problem *pb, const double complex *probe, const double complex *slices,
                          const double *measured, const long *subset, long n_subset, int layer,
                          double complex *grad_slices, double complex *grad_probe, double *overlap,
                          double *grad_pos, double *curv_pos, double *loss);

int orc_loss_grad(const orc_problem *pb, const double complex *probe, const double complex *slices,
                  const double *measured, const long *subset, long n_subset, int layer,
                  double complex *grad_slices, double complex *grad_probe, double *overlap,
                  double *loss)
{
    return loss_grad_impl(pb, probe, slices, measured, subset, n_subset, layer, grad_slices, grad_probe, overlap,
                          NULL, NULL, loss);
}

int orc_position_grad(const orc_problem *pb, const double complex *probe, const double complex *slices,
                      const double *measured, double *grad_pos, double *curv_pos, double *loss)
{
    if (!grad_pos) return -1;
    return loss_grad_impl(pb, probe, slices, measured, NULL, 0, -1, NULL, NULL, NULL, grad_pos, curv_pos, loss);
}

static int loss_grad_impl(const orc_problem *pb, const double complex *probe, const double complex *slices,
                          const double *measured, const long *subset, long n_subset, int layer,
                          double complex *grad_slices, double complex *grad_probe, double *overlap,
                          double *grad_pos, double *curv_pos, double *loss)
{
    if (check_problem(pb) || !probe || !slices || !measured) return -1;
    if (layer >= pb->n_slices) return -1;
    if (grad_probe && layer > 0) return -1;   /* the probe gradient needs the full chain */
    long count = subset ? n_subset : pb->n_pos;
    if (count < 0) return -1;
    if (subset)
        for (long i = 0; i < count; ++i)
            if (subset[i] < 0 || subset[i] >= pb->n_pos) return -1;
    model md;
    if (model_init(&md, pb)) return -2;
    int n = pb->n, M = pb->n_slices;
    size_t n2 = (size_t)n * n, hw = (size_t)pb->obj_h * pb->obj_w;
    size_t gsz = (layer < 0) ? hw * (size_t)M : hw;
    int nt = pb->n_threads > 0 ? pb->n_threads : omp_get_max_threads();
    accum *acc = (accum *)calloc((size_t)nt, sizeof(accum));
    int bad = (acc == NULL);
    double tprod = 1.0;
    if (curv_pos)
        for (int m = 0; m < M; ++m) {
            double mx = 0.0;
            for (size_t i = 0; i < hw; ++i) {
                double complex v = slices[(size_t)m * hw + i];
                double a = creal(v) * creal(v) + cimag(v) * cimag(v);
                if (a > mx) mx = a;
            }
            tprod *= mx;
        }
    if (!bad) {
#pragma omp parallel num_threads(nt)
        {
            int t = omp_get_thread_num();
            accum *ac = &acc[t];
            ac->gpos = grad_pos;
            ac->cpos = curv_pos;
            ac->tprod = tprod;
            ac->gs = grad_slices ? (double complex *)calloc(gsz, sizeof(double complex)) : NULL;
            ac->gp = grad_probe ? (double complex *)calloc(n2, sizeof(double complex)) : NULL;
            ac->w = (overlap && layer >= 0) ? (double *)calloc(hw, sizeof(double)) : NULL;
            double complex *psi = (double complex *)malloc(sizeof(double complex) * n2 * (size_t)M);
            double complex *far = (double complex *)malloc(sizeof(double complex) * n2);
            double complex *tp = (double complex *)malloc(sizeof(double complex) * n2);
            double complex *g = (double complex *)malloc(sizeof(double complex) * n2);
            double complex *tmp = (double complex *)malloc(sizeof(double complex) * n2);
            int ok = psi && far && tp && g && tmp && (!grad_slices || ac->gs) && (!grad_probe || ac->gp)
                     && (!(overlap && layer >= 0) || ac->w);
            if (!ok) {
#pragma omp atomic write
                bad = 1;
            }
            /* Contiguous static blocks: thread t sums positions in ascending order. */
            long lo = count * t / nt, hi = count * (t + 1) / nt;
            if (ok)
                for (long i = lo; i < hi; ++i) {
                    long s = subset ? subset[i] : i;
                    loss_grad_one(&md, s, probe, slices, measured, layer, grad_slices != NULL,
                                  grad_probe != NULL || grad_pos != NULL, ac, psi, far, tp, g, tmp);
                }
            free(psi); free(far); free(tp); free(g); free(tmp);
        }
    }
    if (!bad) {
        double L = 0.0;
        if (grad_slices) memset(grad_slices, 0, sizeof(double complex) * gsz);
        if (grad_probe) memset(grad_probe, 0, sizeof(double complex) * n2);
        if (overlap && layer >= 0) memset(overlap, 0, sizeof(double) * hw);
        for (int t = 0; t < nt; ++t) {
            L += acc[t].loss;
            if (grad_slices) for (size_t i = 0; i < gsz; ++i) grad_slices[i] += acc[t].gs[i];
            if (grad_probe) for (size_t i = 0; i < n2; ++i) grad_probe[i] += acc[t].gp[i];
            if (overlap && layer >= 0) for (size_t i = 0; i < hw; ++i) overlap[i] += acc[t].w[i];
        }
        if (loss) *loss = L;
    }
    if (acc)
        for (int t = 0; t < nt; ++t) { free(acc[t].gs); free(acc[t].gp); free(acc[t].w); }
    free(acc);
    model_free(&md);
    return bad ? -2 : 0;
}

/* ------------------------------------------------------------------ */
/* Step sizes.  Sec. 3.2 takes mu = ||Q||^{-2}.  For the single-layer matrix
 * Q_l = [F R_l diag(S_l p^s) E_s]_s of eq. (Opt_Prob_Single_Layer_Matrix)
 * (E_s extracts the window of position s):
 *   Q_l^H Q_l = N^2 sum_s E_s^T diag(conj psi_l^s) R_l^H R_l diag(psi_l^s) E_s,
 * and ||R_l|| <= prod_{m > l} max|t_m| because every G_m is unitary, so
 *   ||Q_l||^2 <= N^2 * prod_{m > l} max|t_m|^2 * max_pixel sum_s |psi_l^s|^2,
 * with equality when the slices after l have unit modulus.  The step uses this
 * bound; for the probe the same argument gives
 *   ||Q_p||^2 <= N^2 * |subset| * prod_m max|t_m|^2. */

static double max_abs2(const double complex *t, size_t count)
{
    double mx = 0.0;
    for (size_t i = 0; i < count; ++i) {
        double a = creal(t[i]) * creal(t[i]) + cimag(t[i]) * cimag(t[i]);
        if (a > mx) mx = a;
    }
    return mx;
}

int orc_layer_step(const orc_problem *pb, const double complex *probe, double complex *slices,
                   const double *measured, int layer, int k_steps, double *loss_out, double *mu_out)
{
    if (check_problem(pb) || layer < 0 || layer >= pb->n_slices || k_steps < 0) return -1;
    size_t hw = (size_t)pb->obj_h * pb->obj_w;
    double n2 = (double)pb->n * (double)pb->n;
    double prod = 1.0;
    for (int m = layer + 1; m < pb->n_slices; ++m) prod *= max_abs2(slices + (size_t)m * hw, hw);
    double complex *g = (double complex *)malloc(sizeof(double complex) * hw);
    double *w = (double *)malloc(sizeof(double) * hw);
    if (!g || !w) { free(g); free(w); return -2; }
    int rc = 0;
    for (int k = 0; k < k_steps && rc == 0; ++k) {
        double L = 0.0;
        rc = orc_loss_grad(pb, probe, slices, measured, NULL, 0, layer, g, NULL, w, &L);
        if (rc) break;
        double wmax = 0.0;
        for (size_t i = 0; i < hw; ++i) if (w[i] > wmax) wmax = w[i];
        double mu = (wmax > 0.0 && prod > 0.0) ? 1.0 / (n2 * prod * wmax) : 0.0;
        if (pb->objective == ORC_POISSON) mu *= 0.5;
        double complex *o = slices + (size_t)layer * hw;
        for (size_t i = 0; i < hw; ++i) o[i] -= mu * g[i];
        if (loss_out) *loss_out = L;
        if (mu_out) *mu_out = mu;
    }
    free(g); free(w);
    return rc;
}

int orc_full_step(const orc_problem *pb, const double complex *probe, double complex *slices,
                  const double *measured, int k_steps, double step_scale, double *loss_out, double *mu_out)
{
    if (check_problem(pb) || k_steps < 0 || !(step_scale > 0.0)) return -1;
    const int M = pb->n_slices;
    size_t hw = (size_t)pb->obj_h * pb->obj_w;
    double n2 = (double)pb->n * (double)pb->n;
    double complex *g = (double complex *)malloc(sizeof(double complex) * hw * (size_t)M);
    double complex *gl = (double complex *)malloc(sizeof(double complex) * hw);
    double *w = (double *)malloc(sizeof(double) * hw);
    double *mu = (double *)malloc(sizeof(double) * (size_t)M);
    if (!g || !gl || !w || !mu) { free(g); free(gl); free(w); free(mu); return -2; }
    int rc = 0;
    for (int k = 0; k < k_steps && rc == 0; ++k) {
        double L = 0.0;
        rc = orc_loss_grad(pb, probe, slices, measured, NULL, 0, -1, g, NULL, NULL, &L);
        /* every step size at the current iterate, before any slice changes */
        for (int l = 0; l < M && rc == 0; ++l) {
            double dummy = 0.0;
            rc = orc_loss_grad(pb, probe, slices, measured, NULL, 0, l, gl, NULL, w, &dummy);
            double wmax = 0.0, prod = 1.0;
            for (size_t i = 0; i < hw; ++i) if (w[i] > wmax) wmax = w[i];
            for (int m = l + 1; m < M; ++m) prod *= max_abs2(slices + (size_t)m * hw, hw);
            mu[l] = (wmax > 0.0 && prod > 0.0) ? 1.0 / (n2 * prod * wmax) : 0.0;
            if (pb->objective == ORC_POISSON) mu[l] *= 0.5;
            mu[l] *= step_scale;
        }
        if (rc) break;
        for (int l = 0; l < M; ++l) {
            double complex *o = slices + (size_t)l * hw;
            const double complex *gg = g + (size_t)l * hw;
            for (size_t i = 0; i < hw; ++i) o[i] -= mu[l] * gg[i];
        }
        if (loss_out) *loss_out = L;
        if (mu_out) for (int l = 0; l < M; ++l) mu_out[l] = mu[l];
    }
    free(g); free(gl); free(w); free(mu);
    return rc;
}

int orc_probe_step(const orc_problem *pb, double complex *probe, const double complex *slices,
                   const double *measured, const long *subset, long n_subset, int k_steps,
                   double *loss_out, double *mu_out)
{
    if (check_problem(pb) || k_steps < 0) return -1;
    long count = subset ? n_subset : pb->n_pos;
    if (count <= 0) return -1;
    size_t hw = (size_t)pb->obj_h * pb->obj_w;
    size_t n2 = (size_t)pb->n * pb->n;
    double prod = 1.0;
    for (int m = 0; m < pb->n_slices; ++m) prod *= max_abs2(slices + (size_t)m * hw, hw);
    double complex *g = (double complex *)malloc(sizeof(double complex) * n2);
    if (!g) return -2;
    int rc = 0;
    for (int k = 0; k < k_steps && rc == 0; ++k) {
        double L = 0.0;
        rc = orc_loss_grad(pb, probe, slices, measured, subset, n_subset, -1, NULL, g, NULL, &L);
        if (rc) break;
        double mu = prod > 0.0 ? 1.0 / ((double)n2 * (double)count * prod) : 0.0;
        if (pb->objective == ORC_POISSON) mu *= 0.5;
        for (size_t i = 0; i < n2; ++i) probe[i] -= mu * g[i];
        if (loss_out) *loss_out = L;
        if (mu_out) *mu_out = mu;
    }
    free(g);
    return rc;
}
