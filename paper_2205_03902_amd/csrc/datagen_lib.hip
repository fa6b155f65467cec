// libimsp host side of the training-data generator (include/datagen.h).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <string>

#include "datagen.h"
#include "datagen_kernels.hpp"
#include "unet.h"

using namespace datagen;

namespace {

thread_local std::string d_err;

int32_t dfail(int32_t st, const std::string &msg)
{
    d_err = msg;
    return st;
}

int32_t launched(const char *what)
{
    const hipError_t e = hipGetLastError();
    if (e == hipSuccess) return UN_OK;
    return dfail(UN_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

bool crop_ok(int32_t M, int32_t H, int32_t W, int32_t y0, int32_t x0, int32_t h, int32_t w)
{
    return M >= 1 && H >= 1 && W >= 1 && h >= 1 && w >= 1 && h <= H && w <= W && y0 >= 0 && x0 >= 0 &&
           (long long)M * H * W < ((long long)1 << 40);
}

unsigned blocks(long long n) { return (unsigned)((n + 255) / 256); }

}  // namespace

extern "C" {

int32_t dg_make_specimen(hipStream_t stream, const dg_specimen *s, double kappa, float *potential, void *slices)
{
    if (!s) return dfail(UN_ERR_INVALID_ARG, "specimen is NULL");
    if (s->n_slices < 1 || s->obj_h < 1 || s->obj_w < 1 || (long long)s->n_slices * s->obj_h * s->obj_w > (1LL << 31))
        return dfail(UN_ERR_INVALID_ARG, "need n_slices, obj_h, obj_w >= 1 and fewer than 2^31 pixels");
    if (!(s->pixel_size > 0) || !(s->sigma > 0) || !(s->jitter >= 0) || !(s->a_min > 0) || !(s->a_max >= s->a_min) ||
        !(s->vacancy_max >= 0 && s->vacancy_max <= 1) || !std::isfinite(s->a_max) || !std::isfinite(kappa))
        return dfail(UN_ERR_INVALID_ARG, "need pixel_size, sigma, a_min > 0, jitter >= 0, a_max >= a_min, "
                                         "vacancy_max in [0, 1], finite kappa");
    const double Ly = s->obj_h * s->pixel_size, Lx = s->obj_w * s->pixel_size;
    if (Ly < 2.0 * (5.0 * s->sigma + 4.0 * s->jitter) + s->a_max || Lx < 2.0 * (5.0 * s->sigma + 4.0 * s->jitter) + s->a_max)
        return dfail(UN_ERR_INVALID_ARG, "object smaller than two atom reaches plus a lattice constant");
    if (!potential && !slices) return dfail(UN_ERR_INVALID_ARG, "nothing to write");
    SpecimenParams p{};
    p.M = s->n_slices;
    p.H = s->obj_h;
    p.W = s->obj_w;
    p.dx = s->pixel_size;
    p.sigma = s->sigma;
    p.jitter = s->jitter;
    p.a_min = s->a_min;
    p.a_max = s->a_max;
    p.vacancy_max = s->vacancy_max;
    p.two_species = s->two_species != 0;
    p.key0 = s->seed;
    p.key1 = s->specimen;
    const long long n = (long long)p.M * p.H * p.W;
    specimen_kernel<<<blocks(n), 256, 0, stream>>>(p, kappa, potential, static_cast<float2 *>(slices));
    return launched("dg_make_specimen");
}

int32_t dg_poisson(hipStream_t stream, const float *intensity, int64_t count, int32_t n_pix, double dose,
                   uint32_t seed, uint32_t stream_id, float *out)
{
    if (!intensity || !out || count < 0 || n_pix < 1 || !(dose > 0) || !std::isfinite(dose))
        return dfail(UN_ERR_INVALID_ARG, "need device buffers, count >= 0, n_pix >= 1 and a positive dose");
    if (count == 0) return UN_OK;
    poisson_kernel<<<blocks(count), 256, 0, stream>>>(intensity, count, dose / n_pix, n_pix / dose, seed, stream_id,
                                                      out);
    return launched("dg_poisson");
}

int32_t dg_crop_phase(hipStream_t stream, const void *slices, int32_t M, int32_t H, int32_t W, int32_t y0, int32_t x0,
                      int32_t h, int32_t w, int32_t in_pad, uint16_t *out)
{
    if (!slices || !out || !crop_ok(M, H, W, y0, x0, h, w) || in_pad < M || in_pad % 8)
        return dfail(UN_ERR_INVALID_ARG, "bad crop, buffers or in_pad (a multiple of 8, >= n_slices)");
    crop_phase_kernel<<<blocks((long long)h * w * in_pad), 256, 0, stream>>>(static_cast<const float2 *>(slices), M, H,
                                                                              W, y0, x0, h, w, in_pad, out);
    return launched("dg_crop_phase");
}

int32_t dg_crop_potential(hipStream_t stream, const float *potential, int32_t M, int32_t H, int32_t W, int32_t y0,
                          int32_t x0, int32_t h, int32_t w, float *out)
{
    if (!potential || !out || !crop_ok(M, H, W, y0, x0, h, w))
        return dfail(UN_ERR_INVALID_ARG, "bad crop or buffers");
    crop_potential_kernel<<<blocks((long long)h * w * M), 256, 0, stream>>>(potential, M, H, W, y0, x0, h, w, out);
    return launched("dg_crop_potential");
}

int32_t dg_apply_init(hipStream_t stream, const float *v_hat, int32_t M, int32_t H, int32_t W, int32_t y0, int32_t x0,
                      int32_t h, int32_t w, float kappa, void *slices)
{
    if (!v_hat || !slices || !crop_ok(M, H, W, y0, x0, h, w) || !std::isfinite(kappa))
        return dfail(UN_ERR_INVALID_ARG, "bad crop, buffers or kappa");
    apply_init_kernel<<<blocks((long long)h * w * M), 256, 0, stream>>>(v_hat, M, H, W, y0, x0, h, w, kappa,
                                                                         static_cast<float2 *>(slices));
    return launched("dg_apply_init");
}

const char *dg_last_error(void) { return d_err.c_str(); }

}  // extern "C"
