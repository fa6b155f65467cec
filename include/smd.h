/* smd.h -- C ABI of the sparse matrix decomposition (Algorithm 2, Sec. 3.4) in libimsp.so.
 *
 * Algorithm 2 works on the full-field model of Sec. 2.2: the object is as large as the
 * N x N window, positions are integer shifts, and the whole specimen is the dense N^2 x N^2
 * transfer matrix A_M = O_M G_{M-1} ... G_1 O_1 (O_m = diag(t_m), G_m = F_2D^{-1} diag(h_m)
 * F_2D, h_m the propagator of eq. fresnel_element).  One iteration of Algorithm 2 is
 *   smd_estimate   amplitude-flow steps on A (eq. Opt_Prob_Matrix):
 *                  A <- A - mu F^H ((|F A P| - sqrt(I)) o F A P / |F A P|) P^H,
 *                  mu = 1 / (N^2 ||P||^2) with ||P|| the spectral norm of the probe matrix
 *                  (columns: the probe moved to each position, periodic);
 *   smd_decompose  one pass of proximal gradient steps on every diagonal O_l (eq. Prox_Min)
 *                  with the prefixes R_l and suffixes S_l of the incoming slices:
 *                  O_l <- Proj(O_l - conj(lambda) / c diag(R_l^H (lambda R_l O_l S_l - A_hat)
 *                  S_l^H)), c = (|lambda| prod_{m != l} max|o_m|)^2 (which is >= (|lambda|
 *                  ||R_l|| ||S_l||)^2 since G_m is unitary), Proj scaling the diagonal to unit
 *                  Frobenius norm; then the least-squares lambda = Tr(A~^H A_hat) / Tr(A~^H A~)
 *                  (eq. Update Lambda) with A~ = O_M prod G_m O_m;
 *   smd_compose    A = lambda A~ for the next iteration.
 * The result of the algorithm is lambda^(1/M) O_m (smd_result).
 *
 * Data layout.  N^2 x N^2 matrices are complex float (interleaved) in COLUMN-major order:
 * element (i, j) at j N^2 + i, so that column j -- the image of pixel j through the matrix --
 * is one contiguous N x N image.  Images, slices [M][N][N] and the probe are in FFT order as
 * in ms.h; measured intensities [S][N][N].  Device pointers unless marked (host).
 *
 * Implementation.  Products with G_m and F_2D never form those matrices: each is one
 * propagation or 2D DFT of every image of the stored array (in-register line FFTs, the
 * machinery of the multislice kernels).  The two products with the N^2 x S probe matrix in
 * smd_estimate are LDS-tiled kernels of this library.  smd_set_probe and smd_decompose
 * synchronise the stream (the spectral norm of P and the new lambda are finished on the host
 * from device reductions); the other calls only enqueue.  Errors return a negative status (the
 * ms_status codes of ms.h) with a message in
 * smd_last_error().
 */
#ifndef SMD_H
#define SMD_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t n;                  /* window side N: 16, 32 or 64                               */
    int32_t n_slices;           /* M >= 1                                                    */
    int64_t n_pos;              /* 1 <= S <= N^2                                             */
    const double *positions;    /* (host) S x 2 integer (y, x) shifts                        */
    const double *dz;           /* (host) M - 1 slice distances (A)                          */
    double pixel_size, wavelength;
} smd_problem;

typedef struct smd_plan smd_plan;

int32_t smd_workspace_size(const smd_problem *pb, size_t *ws_bytes);
int32_t smd_plan_create(const smd_problem *pb, void *workspace, size_t ws_bytes, smd_plan **out);
void smd_plan_destroy(smd_plan *plan);

/* Builds F_2D, every G_m and the probe matrix P from `probe` (N x N), and the step of
 * smd_estimate (host power iteration on the S x S Gram matrix P^H P).  Synchronises. */
int32_t smd_set_probe(smd_plan *plan, hipStream_t stream, const void *probe);

/* A (N^2 x N^2) = lambda O_M G_{M-1} ... G_1 O_1; slices [M][N][N]; lambda (host, re/im). */
int32_t smd_compose(smd_plan *plan, hipStream_t stream, const void *slices, const double *lambda, void *a_out);

/* `steps` amplitude-flow steps on A in place; loss_first (device double or NULL): the matrix
 * loss 1/2 ||sqrt(I) - |F A P|||^2 before the first step. */
int32_t smd_estimate(smd_plan *plan, hipStream_t stream, const float *measured, void *a, int32_t steps,
                     double *loss_first);

/* One decomposition pass: slices (in/out, [M][N][N]) and lambda (host in/out, re/im) from
 * A_hat; a_tilde_out (N^2 x N^2, or NULL) receives A~.  Synchronises. */
int32_t smd_decompose(smd_plan *plan, hipStream_t stream, const void *a_hat, void *slices, double *lambda,
                      void *a_tilde_out);

/* The result of the algorithm: out (may alias slices) = lambda^(1/M) O_m with the principal
 * M-th root of the host complex lambda (re, im). */
int32_t smd_result(smd_plan *plan, hipStream_t stream, const void *slices, const double *lambda, void *out);

const char *smd_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SMD_H */
