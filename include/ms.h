/*
 * libimsp - layer-wise inverse multislice ptychography on one MI355X (gfx950).
 *
 * C ABI of the GPU library.  The operations follow Bangun et al.,
 * "Inverse Multislice Ptychography by Layer-wise Optimisation and Sparse
 * Matrix Decomposition" (arXiv 2205.03902):
 *   - the forward multislice model of Sec. 2.1: E_1 = P^s o X_1,
 *     E_m = V_z(E_{m-1}) o X_m with V_z(E) = F^{-1}(F(E) o H_m) and the Fresnel
 *     propagator of eq. (fresnel_element), then I^s = |F(E_M^s)|^2;
 *   - the amplitude least-squares objective of eq. (Opt_Prob_Layerwise),
 *     L = sum_s sum_k (sqrt(I_k^s) - |F E_M^s|_k)^2 (no factor 1/2), and its
 *     generalised Wirtinger gradient of Sec. 3.2 (dL/d conj(z), the phase of a
 *     zero far-field value taken as 0);
 *   - the layer-wise amplitude-flow step of Algorithm 1 (Sec. 3.3) and the
 *     probe step of Sec. 3.5, each with step size mu = 1 / (upper bound of
 *     ||Q||^2), the bound being exact when the slices have unit modulus.
 *
 * Data layout.  Complex values are interleaved float32 pairs (ms_c64, the
 * layout of torch.complex64).  2D arrays are row-major [y][x] with x fastest.
 *   probe        N x N, the unshifted probe; its window corner is the scan position.
 *   slices       M x H x W transmission functions t_m (periodic object).
 *   intensities  S x N x N, detector pixels in FFT order (zero frequency at [0][0]).
 * A scan position (y, x) is the corner of the N x N window in object pixels;
 * object indices wrap around modulo H and W (Sec. 1.3).  The integer part of a
 * position selects the object patch; its fractional part shifts the probe by
 * the Fourier phase ramp exp(-2 pi i (k_y f_y + k_x f_x) / N), k in FFT order.
 *
 * Pointers are device pointers unless marked (host).  The caller owns every
 * buffer, including the workspace; the library never allocates device
 * memory.  Every compute call only enqueues work on the given stream and
 * returns without synchronising; outputs are valid once the stream reaches
 * that point.  Gradients are overwritten, not accumulated.
 *
 * Errors.  Arguments are validated on the host before anything is enqueued;
 * on error nothing is launched, no output is touched, a negative ms_status is
 * returned and ms_last_error() describes it.  A HIP error while enqueueing is
 * reported as MS_ERR_HIP.  No C++ exception crosses this interface.
 * Calls that share one plan must not overlap in time (the plan's workspace is
 * reused by every call).
 */
#ifndef IMSP_MS_H
#define IMSP_MS_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    float re, im;
} ms_c64;

typedef enum {
    MS_OK = 0,
    MS_ERR_INVALID_ARG = -1,   /* a NULL pointer, a bad size, a non-finite parameter    */
    MS_ERR_UNSUPPORTED = -2,   /* valid problem outside what this library implements   */
    MS_ERR_BUDGET = -3,        /* workspace smaller than ms_workspace_size requires    */
    MS_ERR_HIP = -4,           /* the HIP runtime reported an error while enqueueing   */
    MS_ERR_NOT_FINITE = -5     /* not returned by this library: the status a caller    */
                               /* (the Python layer) reports when a device FP64 loss   */
                               /* it reads back is NaN or infinite                     */
} ms_status;

/* The problem statement of Sec. 2.1: probe window, slices, scan positions,
 * slice distances, wavelength, tilts. */
typedef struct {
    int32_t n;                 /* window and detector side N: 16, 32, 64, 128 or 256     */
    int32_t obj_h, obj_w;      /* object size H, W in pixels, H >= N, W >= N            */
    int32_t n_slices;          /* M >= 1                                                */
    int64_t n_pos;             /* S >= 1                                                */
    const double *positions;   /* (host) S x 2, (y, x) window corners in object pixels  */
    const double *dz;          /* (host) M - 1 Fresnel distances Delta_m (Angstrom)     */
    double pixel_size;         /* real-space sampling dx (Angstrom), q = k / (N dx)     */
    double wavelength;         /* lambda (Angstrom)                                     */
    double tilt_y, tilt_x;     /* illumination tilts theta_y, theta_x (rad)             */
    int32_t checkpoint_every;  /* incident waves kept for the adjoint, see below          */
} ms_problem;

/* Incident waves.  The adjoint of slice m (Sec. 3.2 pulled back through the chain of Sec. 2.1)
 * needs the wave psi_m incident on slice m at every position of a batch.  checkpoint_every = k:
 *   k = 1      every psi_m is stored during the forward chain (M N^2 complex values a position);
 *   1 < k < M  only psi_k, psi_2k, ... are stored (psi_0 is the shifted probe itself); during the
 *              adjoint, psi_m is recomputed from the nearest stored wave below it by running the
 *              forward chain again from there (m mod k slices), and each slice's gradient patches
 *              are scattered before the next slice is taken;
 *   k >= M     nothing is stored: every psi_m is recomputed from the probe;
 *   k = 0      automatic: 1, unless the workspace budget of ms_workspace_size / the workspace given
 *              to ms_plan_create cannot hold every position's waves at once; then the smallest k
 *              whose waves fit with all positions in one batch, and only if k = M does not fit
 *              are positions split into batches.
 * A larger k trades memory (floor((M - 1) / k) + 1 waves a position instead of M) for the
 * recomputed propagations (about M (k - 1) / 2 slice steps a position instead of none).  All values give
 * the same results up to rounding.  k < 0 returns MS_ERR_INVALID_ARG. */

typedef struct ms_plan ms_plan;

/* Workspace bytes for `pb`.  budget_bytes = 0 processes all positions in one
 * batch; otherwise the wave storage (checkpoint_every, above) and then the batch
 * size are chosen to fit the budget (MS_ERR_BUDGET if not even one position fits).  Positions that share
 * a sub-pixel offset share one shifted probe (a shift class); at most 4096 classes
 * (MS_ERR_UNSUPPORTED beyond), each adding about 21 N^2 8 bytes. */
ms_status ms_workspace_size(const ms_problem *pb, size_t budget_bytes, size_t *ws_bytes);

/* Builds a plan: copies the host arrays, derives patch origins, probe shift
 * classes and the scatter lists, and uploads its tables into `workspace`
 * (device memory of ws_bytes, 256-byte aligned, owned by the caller and kept
 * alive until ms_plan_destroy).  Blocks until the upload is done. */
ms_status ms_plan_create(const ms_problem *pb, void *workspace, size_t ws_bytes, ms_plan **out);
/* Releases the plan's host data and its internal stream and events.  Work the plan
 * enqueued still reads and writes the workspace: synchronise the streams it was
 * called on before freeing the workspace.  NULL is ignored. */
void ms_plan_destroy(ms_plan *plan);

/* Positions per batch, number of probe shift classes and the wave checkpoint interval k
 * (1 = every wave stored; M = none) chosen by the plan. */
int64_t ms_plan_batch(const ms_plan *plan);
int32_t ms_plan_shift_classes(const ms_plan *plan);
int32_t ms_plan_checkpoint_every(const ms_plan *plan);

/* How the per-position multislice chain is executed.  MS_PATH_FUSED keeps each
 * N x N window of one position in one workgroup for the whole chain (N <= 128);
 * MS_PATH_LINES runs one launch per slice, each workgroup holding 16 rows or 16
 * columns of a window, with the half-propagated window in the workspace between
 * launches (N >= 32; the only path for N = 256).  MS_PATH_AUTO (the default)
 * takes the fused path whenever it fits.  Both compute the same quantities. */
typedef enum { MS_PATH_AUTO = 0, MS_PATH_FUSED = 1, MS_PATH_LINES = 2 } ms_path;
ms_status ms_plan_set_path(ms_plan *plan, int32_t path);

/* Band sums of the line path's gradient patches in ms_adjoint.  The gradient of a slice
 * (Sec. 3.2) is the sum over positions of the patches conj(psi_m) o g placed at their
 * windows.  Where the scan puts many windows on one origin x (a scan column), the
 * adjoint launches of even slices let each workgroup take 16 object rows for all windows
 * of such a band and write one image of the band's summed patches; odd slices (whose
 * launches work on columns) do the same for the windows of one origin y.  The scatter
 * then reads band images instead of one patch per position.  The plan decides at
 * creation, for even and for odd slices, whether bands pay (their images take at most
 * three quarters of the elements of the patches they replace) and holds their tables and
 * images in the workspace; launches without them write patches.  The sums take another
 * order than the per-position scatter, so results agree to rounding; each setting is
 * reproducible bit for bit.  MS_BANDS_ALL (the default): both; MS_BANDS_ROWS: even
 * slices only; MS_BANDS_NONE: patches everywhere. */
typedef enum { MS_BANDS_NONE = 0, MS_BANDS_ROWS = 1, MS_BANDS_ALL = 2 } ms_band_mode;
ms_status ms_plan_set_bands(ms_plan *plan, int32_t mode);
/* Which slices of the plan have band tables (bands pay for its scan): bit 0 even
 * slices, bit 1 odd slices. */
int32_t ms_plan_has_bands(const ms_plan *plan);

/* Kept windows in ms_adjoint on the line path.  Launch m of the forward chain (Sec. 2.1)
 * reads the window that launch m - 1 left half-propagated and finishes the propagation
 * along its own lines to obtain the incident wave psi_m.  When the adjoint's launches of
 * both even and odd slices take bands, and every wave is stored (checkpoint interval 1),
 * the forward chain can keep those windows, one per slice after the first, instead of
 * storing psi_m; each adjoint launch then finishes psi_m again from the kept window along
 * the same lines.  The windows take the place of the waves in the workspace (when
 * (M - 1)(N + 16) <= M N), and the chain writes no wave, which saves one N x N complex
 * store per position and slice.  psi_m is recomputed by the same steps, so results agree
 * with the stored waves to rounding (bit for bit where the compiler emits the same
 * instructions).  on = 1 (the default): keep windows where the conditions hold; 0: store
 * waves.  ms_plan_kept_windows returns 1 when the plan's next ms_adjoint keeps windows. */
ms_status ms_plan_set_kept_windows(ms_plan *plan, int32_t on);
int32_t ms_plan_kept_windows(const ms_plan *plan);

/* Incident waves carried between the layer steps of Algorithm 1 (Sec. 3.3) on the line path.
 * ms_layer_step for layer l runs the forward chain (Sec. 2.1) from the probe through every slice;
 * its incident wave psi_l depends only on the slices before l, and the step then updates slice l.
 * With the carry on, the plan keeps psi_l after each layer step, and a following ms_layer_step for
 * layer l (again) or l + 1 with the same probe, slices and measured buffers starts its chain from
 * that wave, at launch l or l - 1, instead of from the probe: a sweep over M layers skips about
 * M (M - 3) / 2 of its launches, with results bit for bit those of the full chain.  This relies on
 * the caller changing none of those buffers between the calls other than through ms_layer_step
 * (every other entry point that computes on the plan, or sets it up, drops the carried wave).  It
 * applies on the line path with all positions in one batch.  on = 1: carry; 0 (the default): every
 * layer step runs the whole chain. */
ms_status ms_plan_set_layer_carry(ms_plan *plan, int32_t on);

/* The data term of every loss, gradient and step of the plan.
 * MS_OBJECTIVE_AMPLITUDE (the default): L = sum (sqrt(I) - |Psi|)^2, the amplitude
 * flow of Sec. 3.2, residual Psi - sqrt(I) Psi / |Psi|.
 * MS_OBJECTIVE_POISSON: the Poisson deviance L = sum |Psi|^2 - I + I log(I / |Psi|^2)
 * (0 log 0 = 0), the maximum-likelihood objective the outlook of Sec. 6 proposes for
 * low-dose data (the negative log-likelihood of counts of mean proportional to |Psi|^2,
 * up to a constant and the dose factor); residual Psi (1 - I / |Psi|^2).  Where Psi is
 * exactly 0 a pixel adds nothing and its residual is Psi, for both objectives.  The
 * paper gives no step rule for it: ms_layer_step and ms_probe_step take half the
 * amplitude-flow step (near the data the deviance bends twice as fast along |Psi|),
 * without the amplitude flow's descent guarantee.  Invalid values return
 * MS_ERR_INVALID_ARG. */
typedef enum { MS_OBJECTIVE_AMPLITUDE = 0, MS_OBJECTIVE_POISSON = 1 } ms_objective;
ms_status ms_plan_set_objective(ms_plan *plan, int32_t objective);

/* The probe of Sec. 2.1 (caption of Fig. 3): the inverse DFT of the disk
 * lambda |q| <= alpha (boundary included), multiplied by the propagator of
 * eq. (fresnel_element) for distance `defocus`, centred at (N/2, N/2) and
 * scaled to sum |p|^2 = 1.  probe_out: N x N. */
ms_status ms_make_probe(ms_plan *plan, hipStream_t stream, double alpha, double defocus,
                        ms_c64 *probe_out);

/* The probe of a lens with aberrations beyond defocus (experimental probes, Sec. 5.3 and
 * the outlook of Sec. 6): the disk times exp(-i chi(q)),
 *   chi = pi lambda C1 q^2 + pi lambda A1 q^2 cos 2(phi - phi_A1) + pi/2 lambda^3 C3 q^4,
 * phi the azimuth of q.  aberrations (host, 4 doubles): C1 (defocus, A), A1 (twofold
 * astigmatism, A), phi_A1 (rad), C3 (spherical aberration, A).  C1 alone is ms_make_probe. */
ms_status ms_make_probe_aberrated(ms_plan *plan, hipStream_t stream, double alpha, const double *aberrations,
                                  ms_c64 *probe_out);

/* Forward model (Sec. 2.1): intensity_out (S x N x N) = |F E_M^s|^2 and, if
 * exit_out is not NULL, the exit waves E_M^s (S x N x N). */
ms_status ms_forward(ms_plan *plan, hipStream_t stream, const ms_c64 *probe, const ms_c64 *slices,
                     float *intensity_out, ms_c64 *exit_out);

/* Loss and gradients (Sec. 3.2) of every slice and of the probe.
 *   measured    S x N x N measured intensities (>= 0), FFT order;
 *   grad_slices M x H x W, dL/d conj(t_m);
 *   grad_probe  N x N, dL/d conj(P), or NULL to skip it;
 *   loss_out    one double, the loss L. */
ms_status ms_adjoint(ms_plan *plan, hipStream_t stream, const ms_c64 *probe, const ms_c64 *slices,
                     const float *measured, ms_c64 *grad_slices, ms_c64 *grad_probe,
                     double *loss_out);

/* ms_adjoint without a plan or workspace, for callers that cannot allocate device memory (serving
 * loops and harnesses that forbid hipMalloc).  It builds the plan of `pb` on the host (freed before
 * returning) in a static device array of MS_SCRATCH_BYTES that the library holds on every device it
 * runs on until the process ends, chooses the wave storage and the batch to fit it (checkpoint_every
 * as for ms_workspace_size with that budget), and enqueues ms_adjoint's work on `stream`; it calls no
 * device allocation.  Arguments and results are those of ms_adjoint.  Problems whose smallest
 * footprint (one position a batch, no wave stored) exceeds the array return MS_ERR_BUDGET with the
 * bytes needed, and nothing is enqueued.  Before uploading its tables the call waits for `stream`
 * (work enqueued earlier on it may still read the array); calls that overlap in time on one device
 * (other streams, other threads) share the array and race. */
#define MS_SCRATCH_BYTES ((size_t)64 << 20)
ms_status ms_adjoint_scratch(const ms_problem *pb, hipStream_t stream, const ms_c64 *probe, const ms_c64 *slices,
                             const float *measured, ms_c64 *grad_slices, ms_c64 *grad_probe, double *loss_out);

/* k_steps amplitude-flow steps on slice `layer` (0-based, i.e. l - 1), the
 * inner loop of Algorithm 1 with the other slices fixed:
 *   t_l <- t_l - mu * dL/d conj(t_l),
 *   mu = 1 / (N^2 * prod_{m > l} max|t_m|^2 * max_pixel sum_s |psi_l^s|^2),
 * psi_l^s being the wave incident on slice l at position s.  Only slice
 * `layer` of `slices` is written.  loss_out / mu_out (one double each, may be
 * NULL) receive the loss and step size of the last step, the loss evaluated
 * before that step. */
ms_status ms_layer_step(ms_plan *plan, hipStream_t stream, int32_t layer, int32_t k_steps,
                        const ms_c64 *probe, ms_c64 *slices, const float *measured,
                        double *loss_out, double *mu_out);

/* K full-gradient steps: the gradient-based alternative the introduction (Sec. 1)
 * contrasts with the layer-wise method.  One fwd+adj pass gives the gradient of every
 * slice; each slice then takes the step of a layer step of Algorithm 1 (its own
 * mu_m = 1 / (N^2 prod_{m' > m} max|t_m'|^2 max_pixel sum_s |psi_m^s|^2), halved for the
 * Poisson objective) times step_scale, all from the same iterate (a Jacobi update
 * instead of the Gauss-Seidel sweep).  With step_scale = 1 the M simultaneous layer
 * steps overshoot (each is sized for moving its slice alone; there is no descent
 * guarantee); 1/M averages them.  step_scale must be positive and finite.  slices
 * (in/out): all M slices change.  loss_out (device FP64 or NULL): the loss at the
 * iterate before the last step; mu_out (device FP64 [M] or NULL): that step's sizes. */
ms_status ms_full_step(ms_plan *plan, hipStream_t stream, int32_t k_steps, double step_scale, const ms_c64 *probe,
                       ms_c64 *slices, const float *measured, double *loss_out, double *mu_out);

/* k_steps amplitude-flow steps on the probe (Sec. 3.5) over the positions in
 * `subset` ((host) n_subset indices in [0, S); NULL = all positions):
 *   P <- P - mu * dL/d conj(P),  mu = 1 / (N^2 * n_subset * prod_m max|t_m|^2).
 * The paper's variant uses the single centre position.  loss_out / mu_out as
 * for ms_layer_step. */
ms_status ms_probe_step(ms_plan *plan, hipStream_t stream, int32_t k_steps, ms_c64 *probe,
                        const ms_c64 *slices, const float *measured, const int64_t *subset,
                        int64_t n_subset, double *loss_out, double *mu_out);

/* Gradient of the loss with respect to every scan position (the outlook of Sec. 6: scan
 * positions deviate from the ideal raster).  Position s is the window corner plus a
 * sub-pixel shift of the probe, P^s = F^{-1}(F p o e^{-2 pi i (k_y f_y + k_x f_x)/N}) with
 * signed k, so
 *   grad_pos[s] = 2 Re sum_pixels conj(dL/dconj(P^s)) dP^s/df    (y, then x),
 * dP^s/df the ramp differentiated (times -2 pi i k / N).  curv_pos[s] (or NULL) receives
 * 2 N^2 prod_m max|t_m|^2 ||dP^s/df||^2 per axis, a bound on the second derivative of the
 * quadratic model (||Q||^2 <= N^2 prod_m max|t_m|^2 since every G_m is unitary), so that
 * -grad/curv is a step that the model cannot make worse.  grad_pos, curv_pos: device
 * double [S][2]; loss_out (device double or NULL): the loss.  Both execution paths. */
ms_status ms_position_grad(ms_plan *plan, hipStream_t stream, const ms_c64 *probe, const ms_c64 *slices,
                           const float *measured, double *grad_pos, double *curv_pos, double *loss_out);

/* One refinement step of the scan positions: positions (device double [S][2], in/out, the
 * plan's positions on entry) <- positions - step_scale * grad_pos / curv_pos (per axis; an
 * axis with zero curvature stays).  step_scale > 0; 1 is the majorised step.  The plan keeps
 * its own positions: build a new plan from the returned ones.  loss_out as above. */
ms_status ms_position_step(ms_plan *plan, hipStream_t stream, double step_scale, const ms_c64 *probe,
                           const ms_c64 *slices, const float *measured, double *positions, double *loss_out);

/* The relative reconstruction error of the experiments (Sec. 5), (1/M) sum_m ||O_m - Ohat_m||_F /
 * ||O_m||_F, after removing the ambiguities of the model.  Intensities do not change when every
 * slice is translated together (and the probe the other way), so the estimate is first translated
 * periodically by the integer d = (d_y, d_x), |d_y|, |d_x| <= max_shift, Ohat_d[y][x] =
 * Ohat[(y - d_y) mod H][(x - d_x) mod W]; each translated slice is then multiplied by the complex
 * scale alpha_m (phase and amplitude, least squares) that brings it closest to the reference, so that
 * the error of slice m is
 *   sqrt(||ref||^2 - |<est_d, ref>|^2 / ||est_d||^2) / ||ref||   (1 where est_d is 0),
 * with every sum over the reference pixels where mask > 0 (mask: H x W floats, or NULL for all
 * pixels; pixels no window covers carry no information).  The translation taken is the one with the
 * smallest mean error, the first minimum when d_y and then d_x run upwards; max_shift = 0 compares
 * without translation.  est, ref: [M][H][W]; max_shift in [0, 64] and below H and W.  work: device
 * double [(2 max_shift + 1)^2 (M + 1)] (overwritten).  err_out: device double [M + 1], the error of
 * each slice and then their mean, at that translation; shift_out: device int32 [2] (d_y, d_x) or NULL.
 * FP64 sums in a fixed order.  No plan is needed. */
ms_status ms_reconstruction_error(hipStream_t stream, const ms_c64 *est, const ms_c64 *ref, const float *mask,
                                  int32_t n_slices, int32_t obj_h, int32_t obj_w, int32_t max_shift, double *work,
                                  double *err_out, int32_t *shift_out);

/* Timing of the dominant kernel (the fused per-position multislice kernel).
 * After ms_profile_begin, the next max_launches launches of that kernel made
 * through `plan` are each bracketed by a pair of HIP events on their stream.
 * ms_profile_end waits for the last of them, returns the summed kernel time
 * (milliseconds) and the number of launches timed, and releases the events.
 * For measurement tools; not needed for computation. */
ms_status ms_profile_begin(ms_plan *plan, int32_t max_launches);
ms_status ms_profile_end(ms_plan *plan, double *total_ms, int64_t *launches);

/* Message of the last error on the calling thread ("" if none). */
const char *ms_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
