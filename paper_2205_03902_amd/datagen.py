"""ctypes binding of the on-device training-data generator (include/datagen.h).

Argument marshalling only: specimens, noise and crops are computed by the HIP
kernels behind the C ABI; torch provides the device buffers and the stream.
"""
from __future__ import annotations

import ctypes as C
import dataclasses

from . import abi

SYMBOLS = ("dg_make_specimen", "dg_poisson", "dg_crop_phase", "dg_crop_potential", "dg_apply_init",
           "dg_last_error")


class DgSpecimen(C.Structure):
    _fields_ = [("n_slices", C.c_int32), ("obj_h", C.c_int32), ("obj_w", C.c_int32), ("pixel_size", C.c_double),
                ("sigma", C.c_double), ("jitter", C.c_double), ("a_min", C.c_double), ("a_max", C.c_double),
                ("vacancy_max", C.c_double), ("two_species", C.c_int32), ("seed", C.c_uint32),
                ("specimen", C.c_uint32)]


@dataclasses.dataclass(frozen=True)
class SpecimenFamily:
    """A family of random lattice specimens (one member per index)."""
    n_slices: int
    obj_h: int
    obj_w: int
    pixel_size: float = 0.2
    sigma: float = 0.3
    jitter: float = 0.1
    a_min: float = 3.5
    a_max: float = 4.2
    vacancy_max: float = 0.05
    two_species: bool = True
    seed: int = 30

    def struct(self, index: int) -> DgSpecimen:
        return DgSpecimen(self.n_slices, self.obj_h, self.obj_w, self.pixel_size, self.sigma, self.jitter, self.a_min,
                          self.a_max, self.vacancy_max, int(self.two_species), self.seed & 0xFFFFFFFF,
                          int(index) & 0xFFFFFFFF)


_bound = False


def lib():
    global _bound
    L = abi.lib()
    if not _bound:
        P, I32, I64, D, U32 = C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_uint32
        L.dg_make_specimen.restype = I32
        L.dg_make_specimen.argtypes = [P, C.POINTER(DgSpecimen), D, P, P]
        L.dg_poisson.restype = I32
        L.dg_poisson.argtypes = [P, P, I64, I32, D, U32, U32, P]
        L.dg_crop_phase.restype = I32
        L.dg_crop_phase.argtypes = [P, P, I32, I32, I32, I32, I32, I32, I32, I32, P]
        L.dg_crop_potential.restype = I32
        L.dg_crop_potential.argtypes = [P, P, I32, I32, I32, I32, I32, I32, I32, P]
        L.dg_apply_init.restype = I32
        L.dg_apply_init.argtypes = [P, P, I32, I32, I32, I32, I32, I32, I32, C.c_float, P]
        L.dg_last_error.restype = C.c_char_p
        L.dg_last_error.argtypes = []
        _bound = True
    return L


def _check(status: int, what: str):
    if status != 0:
        raise abi.MsError(status, what, lib().dg_last_error().decode())


def _stream(t):
    import torch
    return torch.cuda.current_stream(t.device).cuda_stream


def _dev(t, dtype, shape, name):
    if not t.is_cuda or t.dtype != dtype or tuple(t.shape) != tuple(shape) or not t.is_contiguous():
        raise ValueError(f"{name}: expected a contiguous {dtype} CUDA tensor of shape {tuple(shape)}, "
                         f"got {t.dtype} {tuple(t.shape)} on {t.device}")


def make_specimen(fam: SpecimenFamily, index: int, kappa: float, potential=None, slices=None):
    """Writes V (M, H, W) float32 and/or t = exp(i kappa V) (M, H, W) complex64."""
    shape = (fam.n_slices, fam.obj_h, fam.obj_w)
    import torch
    if potential is not None:
        _dev(potential, torch.float32, shape, "potential")
    if slices is not None:
        _dev(slices, torch.complex64, shape, "slices")
    ref = potential if potential is not None else slices
    if ref is None:
        raise ValueError("nothing to write")
    s = fam.struct(index)
    _check(lib().dg_make_specimen(_stream(ref), C.byref(s), float(kappa),
                                  None if potential is None else potential.data_ptr(),
                                  None if slices is None else slices.data_ptr()), "dg_make_specimen")


def poisson(intensity, dose: float, seed: int, stream_id: int, out=None):
    """Counts ~ Poisson(dose I / N^2) per pixel as counts N^2 / dose; intensity (..., N, N) float32."""
    import torch
    if not intensity.is_cuda or intensity.dtype != torch.float32 or not intensity.is_contiguous():
        raise ValueError("intensity must be a contiguous float32 CUDA tensor")
    out = out if out is not None else torch.empty_like(intensity)
    n_pix = intensity.shape[-1] * intensity.shape[-2]
    _check(lib().dg_poisson(_stream(intensity), intensity.data_ptr(), intensity.numel(), n_pix, float(dose),
                            seed & 0xFFFFFFFF, stream_id & 0xFFFFFFFF, out.data_ptr()), "dg_poisson")
    return out


def crop_phase(slices, y0: int, x0: int, h: int, w: int, in_pad: int, out=None):
    """(h, w, in_pad) bfloat16 phases of slices (M, H, W) complex64 over a crop."""
    import torch
    M, H, W = slices.shape
    _dev(slices, torch.complex64, (M, H, W), "slices")
    out = out if out is not None else torch.empty((h, w, in_pad), dtype=torch.bfloat16, device=slices.device)
    _dev(out, torch.bfloat16, (h, w, in_pad), "out")
    _check(lib().dg_crop_phase(_stream(slices), slices.data_ptr(), M, H, W, y0, x0, h, w, in_pad, out.data_ptr()),
           "dg_crop_phase")
    return out


def crop_potential(potential, y0: int, x0: int, h: int, w: int, out=None):
    import torch
    M, H, W = potential.shape
    _dev(potential, torch.float32, (M, H, W), "potential")
    out = out if out is not None else torch.empty((h, w, M), dtype=torch.float32, device=potential.device)
    _dev(out, torch.float32, (h, w, M), "out")
    _check(lib().dg_crop_potential(_stream(potential), potential.data_ptr(), M, H, W, y0, x0, h, w, out.data_ptr()),
           "dg_crop_potential")
    return out


def apply_init(v_hat, slices, y0: int, x0: int, kappa: float):
    """slices (M, H, W) complex64 over the crop <- exp(i kappa v_hat), v_hat (h, w, M) float32."""
    import torch
    M, H, W = slices.shape
    h, w = v_hat.shape[0], v_hat.shape[1]
    _dev(slices, torch.complex64, (M, H, W), "slices")
    _dev(v_hat, torch.float32, (h, w, M), "v_hat")
    _check(lib().dg_apply_init(_stream(slices), v_hat.data_ptr(), M, H, W, y0, x0, h, w, float(kappa),
                               slices.data_ptr()), "dg_apply_init")
