"""FP64 reference of the relative reconstruction error of the experiments (Sec. 5).

TEST INFRASTRUCTURE ONLY: the tests use it to check the device implementation; the product
path never imports it.  Written out as the definition: the error of slice m is
||alpha_m Ohat_m - O_m||_F / ||O_m||_F with alpha_m the complex scale (phase and amplitude)
that minimises it -- the model cannot tell a slice from its phase-shifted or rescaled copy
(Sec. 3.4 notes the scale ambiguity prod alpha_m = 1) -- and the reported value is the mean
over the slices.  Sums run over the pixels where the mask is positive (pixels no scan window
covers carry no information).
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
