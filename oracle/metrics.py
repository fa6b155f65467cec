"""FP64 reference of the relative reconstruction error of the experiments (Sec. 5).

TEST INFRASTRUCTURE ONLY: the tests use it to check the device implementation; the product
path never imports it.  Written out as the definition: the error of slice m is
||alpha_m Ohat_m - O_m||_F / ||O_m||_F with alpha_m the complex scale (phase and amplitude)
that minimises it -- the model cannot tell a slice from its phase-shifted or rescaled copy
(Sec. 3.4 notes the scale ambiguity prod alpha_m = 1) -- and the reported value is the mean
over the slices.  Sums run over the pixels where the mask is positive (pixels no scan window
covers carry no information).

The model also cannot tell the object from a copy of every slice translated together (with the
probe moved the other way, each far-field intensity is unchanged), so a reconstruction from an
estimated probe may come out shifted.  reconstruction_error_aligned takes, over the integer
translations d with |d_y|, |d_x| <= max_shift of every estimated slice (periodic object:
est_d[y][x] = est[(y - d_y) mod H][(x - d_x) mod W]), the one with the smallest mean error, the
first minimum when d_y and then d_x run upwards.
"""
from __future__ import annotations

import numpy as np


def reconstruction_error(est, ref, mask=None):
    """Returns (per-slice errors (M,), their mean) in FP64."""
    est = np.asarray(est, dtype=np.complex128)
    ref = np.asarray(ref, dtype=np.complex128)
    sel = np.ones(est.shape[1:], dtype=bool) if mask is None else np.asarray(mask) > 0
    errs = []
    for m in range(est.shape[0]):
        e, r = est[m][sel], ref[m][sel]
        rn = np.linalg.norm(r)
        if rn == 0.0:
            errs.append(0.0)
            continue
        ee = np.vdot(e, e).real
        alpha = np.vdot(e, r) / ee if ee > 0.0 else 0.0     # least-squares complex scale
        errs.append(float(np.linalg.norm(alpha * e - r) / rn))
    errs = np.array(errs)
    return errs, float(errs.mean())


def reconstruction_error_aligned(est, ref, mask=None, max_shift=0):
    """Returns (per-slice errors (M,), their mean, (d_y, d_x)) at the best translation."""
    est = np.asarray(est, dtype=np.complex128)
    best = None
    for dy in range(-max_shift, max_shift + 1):
        for dx in range(-max_shift, max_shift + 1):
            errs, mean = reconstruction_error(np.roll(est, (dy, dx), axis=(1, 2)), ref, mask)
            if best is None or mean < best[1]:
                best = (errs, mean, (dy, dx))
    return best
