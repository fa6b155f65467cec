/* datagen.h -- C ABI of the on-device training-data generator in libimsp.so.
 *
 * Specimens follow the synthetic stand-in for the paper's crystals (its Table 1
 * structures are not available): every slice is a square lattice of Gaussian atoms
 * (radius sigma) with a random origin, jittered sites, two species (amplitude x 2 with
 * probability 1/2) and vacancies, over a periodic object; t = exp(i kappa V).  Random
 * numbers are Philox4x32-10 (Salmon et al., SC 2011) with key (seed, specimen):
 *   counter (0xFFFFFFFF, 0, 0, 0)   lattice constant a = a_min + (a_max - a_min) u0,
 *                                    vacancy rate = vacancy_max u1;
 *   counter (0xFFFFFFFE, m, 0, 0)   origin of slice m: (a u0, a u1);
 *   counter (i, j, m, 1)            site (i, j) of slice m, sites at origin + (i a, j a) for
 *                                    0 <= i < ceil((H dx - y0) / a), likewise j: jitter by
 *                                    Box-Muller from (u0, u1) (u0 taken on (0, 1]), truncated at
 *                                    4 standard deviations; amplitude 0.5 + u2; heavy species
 *                                    if bit 31 of the fourth word is set; vacant if its low 24
 *                                    bits / 2^24 < vacancy rate;
 * with u_k = word_k / 2^32.  V sums each site at its periodic image nearest the pixel,
 * leaving out sites farther than 5 sigma along y or x.
 *
 * Detector noise (the paper's measurement model, Sec. 2.1, with a finite dose): counts
 * ~ Poisson(dose I / n_pix) per pixel, returned as counts n_pix / dose, drawn by inversion
 * below a mean of 10 and by Hormann's transformed rejection (PTRS, 1993) above.
 *
 * Device pointers unless marked; calls enqueue on the stream and do not synchronise;
 * arguments are checked on the host, errors return a negative status (the un_status
 * codes of unet.h) with a message in dg_last_error().
 */
#ifndef DATAGEN_H
#define DATAGEN_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t n_slices, obj_h, obj_w;
    double pixel_size;          /* A                                      */
    double sigma;               /* Gaussian atom radius (A), > 0          */
    double jitter;              /* site jitter standard deviation (A)     */
    double a_min, a_max;        /* lattice constant range (A), a_min > 0  */
    double vacancy_max;         /* in [0, 1]                              */
    int32_t two_species;        /* 0 or 1                                 */
    uint32_t seed, specimen;    /* Philox key                             */
} dg_specimen;

/* Potential V [M][H][W] (float, or NULL) and transmissions exp(i kappa V) [M][H][W]
 * (interleaved complex float, or NULL). */
int32_t dg_make_specimen(hipStream_t stream, const dg_specimen *spec, double kappa, float *potential,
                         void *slices);

/* out[i] = Poisson(dose intensity[i] / n_pix) n_pix / dose for i < count (out may alias
 * intensity); key (seed, stream_id), counter (i, block). */
int32_t dg_poisson(hipStream_t stream, const float *intensity, int64_t count, int32_t n_pix, double dose,
                   uint32_t seed, uint32_t stream_id, float *out);

/* Network input: phases of slices [M][H][W] (complex float) over the crop of h x w
 * pixels at (y0, x0) (indices wrap), as bf16 [h][w][in_pad] with zero channels past M. */
int32_t dg_crop_phase(hipStream_t stream, const void *slices, int32_t n_slices, int32_t obj_h, int32_t obj_w,
                      int32_t y0, int32_t x0, int32_t h, int32_t w, int32_t in_pad, uint16_t *out);

/* Training target: potential [M][H][W] over the same crop as float [h][w][M]. */
int32_t dg_crop_potential(hipStream_t stream, const float *potential, int32_t n_slices, int32_t obj_h,
                          int32_t obj_w, int32_t y0, int32_t x0, int32_t h, int32_t w, float *out);

/* Learned initialisation: slices over the crop <- exp(i kappa v_hat), v_hat [h][w][M] float;
 * the rest of the slices is left as it is. */
int32_t dg_apply_init(hipStream_t stream, const float *v_hat, int32_t n_slices, int32_t obj_h, int32_t obj_w,
                      int32_t y0, int32_t x0, int32_t h, int32_t w, float kappa, void *slices);

const char *dg_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* DATAGEN_H */
