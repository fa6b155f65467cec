/*
 * FP64 CPU oracle for layer-wise inverse multislice ptychography
 * (Bangun et al., "Inverse Multislice Ptychography by Layer-wise Optimisation
 * and Sparse Matrix Decomposition", arXiv 2205.03902).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU library
 * against a plain, slow and readable implementation of the same mathematics.
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark load it; the product path never does.  It shares no code, header,
 * table or helper with the GPU library.
 *
 * Conventions (each one a reading of the paper, repeated in the functions):
 *   - complex data is C99 `double complex`, arrays are row-major [y][x];
 *   - the forward DFT is unnormalised, F x[k] = sum_n x[n] exp(-2 pi i n k / N)
 *     (per axis), and F^{-1} = F^H / N^2 in 2D, so ||F||^2 = N^2 as in the
 *     step size of the matrix amplitude-flow step (Sec. 3.4);
 *   - spatial frequencies are q = k / (N dx) with k in FFT order
 *     (0, 1, ..., N/2 - 1, -N/2, ..., -1);
 *   - a scan position is the (y, x) corner of the N x N window in object
 *     pixels; its integer part selects the object patch (indices wrap around
 *     the H x W object, Sec. 1.3), its fractional part shifts the probe by a
 *     Fourier phase ramp;
 *   - the loss is L = sum_s sum_k (sqrt(I_k) - |Psi_k|)^2 without a factor 1/2
 *     (Sec. 3.2) and every gradient is the generalised Wirtinger gradient of
 *     Sec. 3.2, i.e. dL/d(conj z), with the phase set to 0 where Psi_k = 0;
 *   - with objective = ORC_POISSON the loss is the Poisson deviance that the
 *     outlook of Sec. 6 proposes for low-dose data,
 *       L = sum_s sum_k |Psi_k|^2 - I_k + I_k log(I_k / |Psi_k|^2)
 *     (the negative log-likelihood of counts with mean proportional to |Psi|^2,
 *     up to a constant and the dose factor; 0 log 0 = 0), whose Wirtinger
 *     gradient in Psi is Psi (1 - I / |Psi|^2); where Psi_k = 0 exactly the
 *     pixel adds nothing and its residual is Psi_k, as for the amplitude loss.
 *
 * Every function returns 0 on success and a negative value on invalid input.
 */
#ifndef IMSP_ORACLE_H
#define IMSP_ORACLE_H

#include <complex.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int n;                   /* window / detector side N (power of two)            */
    int obj_h, obj_w;        /* periodic object size H x W, H >= N and W >= N      */
    int n_slices;            /* M >= 1                                             */
    long n_pos;              /* S                                                  */
    const double *positions; /* S x 2, (y, x) window corners in object pixels      */
    const double *dz;        /* M - 1 Fresnel distances (A)                        */
    double pixel_size;       /* dx (A)                                             */
    double wavelength;       /* lambda (A)                                         */
    double tilt_y, tilt_x;   /* illumination tilts theta_y, theta_x (rad)          */
    int n_threads;           /* worker threads, 0 = OpenMP default                 */
    int objective;           /* ORC_AMPLITUDE (Sec. 3.2) or ORC_POISSON (Sec. 6)   */
} orc_problem;

enum { ORC_AMPLITUDE = 0, ORC_POISSON = 1 };

/* Threads the oracle uses when orc_problem.n_threads is 0. */
int orc_max_threads(void);

/* Electron wavelength (A) for an acceleration voltage U (V), Sec. 5.3.2. */
double orc_wavelength(double volts);

/* Brute-force DFT of length n, out[k] = sum_j in[j] exp(sign 2 pi i j k / n). */
void orc_dft1d(const double complex *in, double complex *out, int n, int sign);

/* Textbook iterative radix-2 FFT in place, same sign convention, unnormalised. */
int orc_fft1d(double complex *x, int n, int sign);

/* 2D FFT of an n x n array in place (rows, then columns), unnormalised. */
int orc_fft2d(double complex *x, int n, int sign);

/* Spatial frequencies q[k] = k / (n d) in FFT order. */
void orc_fftfreq(int n, double d, double *q);

/* Fresnel propagator H (n x n) of eq. (fresnel_element) for distance dz. */
void orc_propagator(int n, double dx, double lambda, double dz, double tilt_y, double tilt_x,
                    double complex *h);

/* Probe: inverse DFT of the disk lambda |q| <= alpha times the propagator for
 * `defocus`, centred at (n/2, n/2) and scaled to sum |p|^2 = 1. */
int orc_probe(int n, double dx, double lambda, double alpha, double defocus, double complex *p);

/* The same probe with a probe-forming lens that has, besides defocus C1, twofold
 * astigmatism A1 at angle phi_A1 and spherical aberration C3 (A, rad): the aperture times
 * exp(-i chi(q)), chi = pi lambda C1 q^2 + pi lambda A1 q^2 cos 2(phi - phi_A1)
 * + pi/2 lambda^3 C3 q^4 with phi the azimuth of q; C1 alone gives orc_probe. */
int orc_probe_aberrated(int n, double dx, double lambda, double alpha, double c1, double a1, double phi_a1,
                        double c3, double complex *p);

/* Sub-pixel shift out = F^{-1}( F p * exp(-2 pi i (ky fy + kx fx) / n) ), identity when fy = fx = 0. */
int orc_shift(const double complex *p, int n, double fy, double fx, double complex *out);

/* Adjoint of orc_shift: the conjugate phase ramp. */
int orc_unshift(const double complex *g, int n, double fy, double fx, double complex *out);

/* Forward multislice for every position: intensities (S x n x n) and, if
 * non-NULL, exit waves E_M (S x n x n). */
int orc_forward(const orc_problem *pb, const double complex *probe, const double complex *slices,
                double *intensity, double complex *exit_waves);

/* Loss and Wirtinger gradients over the positions in `subset` (NULL = all).
 *   layer < 0 : grad_slices (M x H x W) receives the gradient of every slice;
 *   layer >= 0: grad_slices (H x W) receives only the gradient of slice `layer`
 *               and overlap (H x W, may be NULL) receives sum_s |psi_layer^s|^2.
 * grad_slices, grad_probe (n x n) and loss may each be NULL. */
int orc_loss_grad(const orc_problem *pb, const double complex *probe, const double complex *slices,
                  const double *measured, const long *subset, long n_subset, int layer,
                  double complex *grad_slices, double complex *grad_probe, double *overlap,
                  double *loss);

/* Gradient of the loss with respect to every scan position (row f4: the positions of an
 * experiment deviate from the raster, Sec. 6).  A position is the window's corner plus a
 * sub-pixel shift of the probe (orc_shift), so grad_pos[s] (S x 2, y then x) is
 * 2 Re sum conj(dL/dconj(P^s)) dP^s/df along each axis.  curv_pos (S x 2, may be NULL)
 * receives 2 N^2 prod_m max|t_m|^2 ||dP^s/df||^2, which bounds the second derivative of the
 * quadratic model along that axis.  loss may be NULL. */
int orc_position_grad(const orc_problem *pb, const double complex *probe, const double complex *slices,
                      const double *measured, double *grad_pos, double *curv_pos, double *loss);

/* K amplitude-flow steps on slice `layer` (Algorithm 1, inner loop), in place.
 * loss_out: loss at the iterate before the last step; mu_out: its step size.
 * With the Poisson objective the step is half the amplitude-flow step: near the
 * data the deviance bends twice as fast along |Psi| as the amplitude loss. */
int orc_layer_step(const orc_problem *pb, const double complex *probe, double complex *slices,
                   const double *measured, int layer, int k_steps, double *loss_out, double *mu_out);

/* K full-gradient steps (the gradient-based alternative the introduction contrasts with
 * the layer-wise method): every slice takes the step it would take in a layer step of
 * Algorithm 1, all from the same iterate (Jacobi), i.e. t_m -= mu_m dL/dconj(t_m) with
 * mu_m the layer-step size of slice m times step_scale (> 0; 1 / M averages the M layer
 * steps).  loss_out: loss at the iterate before the last step; mu_out (M values, may be
 * NULL): the step sizes of the last step. */
int orc_full_step(const orc_problem *pb, const double complex *probe, double complex *slices,
                  const double *measured, int k_steps, double step_scale, double *loss_out, double *mu_out);

/* K amplitude-flow steps on the probe over `subset` (NULL = all), in place. */
int orc_probe_step(const orc_problem *pb, double complex *probe, const double complex *slices,
                   const double *measured, const long *subset, long n_subset, int k_steps,
                   double *loss_out, double *mu_out);

#ifdef __cplusplus
}
#endif
#endif
