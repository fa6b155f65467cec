"""ctypes binding of the FP64 CPU oracle (liboracle.so, built from oracle.c).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark use it; the product path never imports it.  It shares no
code with the GPU library.  All arrays are numpy float64 / complex128.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SOURCES = [os.path.join(HERE, "oracle.c")]


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (plain FP64: no fast-math, no FMA contraction)."""
    if not force and os.path.exists(LIB_PATH):
        return LIB_PATH
    tmp = LIB_PATH + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-Wall", "-Wextra", "-o", tmp] + SOURCES + ["-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


class Problem(C.Structure):
    _fields_ = [("n", C.c_int), ("obj_h", C.c_int), ("obj_w", C.c_int), ("n_slices", C.c_int),
                ("n_pos", C.c_long), ("positions", C.c_void_p), ("dz", C.c_void_p),
                ("pixel_size", C.c_double), ("wavelength", C.c_double),
                ("tilt_y", C.c_double), ("tilt_x", C.c_double), ("n_threads", C.c_int), ("objective", C.c_int)]

AMPLITUDE, POISSON = 0, 1


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.orc_max_threads.restype = C.c_int
        L.orc_max_threads.argtypes = []
        L.orc_wavelength.restype = C.c_double
        L.orc_wavelength.argtypes = [C.c_double]
        L.orc_dft1d.restype = None
        L.orc_dft1d.argtypes = [P, P, C.c_int, C.c_int]
        L.orc_fft1d.argtypes = [P, C.c_int, C.c_int]
        L.orc_fft2d.argtypes = [P, C.c_int, C.c_int]
        L.orc_fftfreq.restype = None
        L.orc_fftfreq.argtypes = [C.c_int, C.c_double, P]
        L.orc_propagator.restype = None
        L.orc_propagator.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double, C.c_double, C.c_double, P]
        L.orc_probe.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double, C.c_double, P]
        L.orc_probe_aberrated.argtypes = [C.c_int] + [C.c_double] * 7 + [P]
        L.orc_shift.argtypes = [P, C.c_int, C.c_double, C.c_double, P]
        L.orc_unshift.argtypes = [P, C.c_int, C.c_double, C.c_double, P]
        L.orc_forward.argtypes = [C.POINTER(Problem), P, P, P, P]
        L.orc_loss_grad.argtypes = [C.POINTER(Problem), P, P, P, P, C.c_long, C.c_int, P, P, P, P]
        L.orc_layer_step.argtypes = [C.POINTER(Problem), P, P, P, C.c_int, C.c_int, P, P]
        L.orc_probe_step.argtypes = [C.POINTER(Problem), P, P, P, P, C.c_long, C.c_int, P, P]
        L.orc_full_step.argtypes = [C.POINTER(Problem), P, P, P, C.c_int, C.c_double, P, P]
        L.orc_position_grad.argtypes = [C.POINTER(Problem), P, P, P, P, P, P]
        _lib = L
    return _lib


def _c128(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.complex128)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"oracle {what} failed with code {rc}")


def max_threads() -> int:
    return lib().orc_max_threads()


def wavelength(volts: float) -> float:
    return lib().orc_wavelength(float(volts))


def dft1d(x, sign=-1):
    x = _c128(x)
    out = np.empty_like(x)
    lib().orc_dft1d(_ptr(x), _ptr(out), x.shape[0], sign)
    return out


def fft1d(x, sign=-1):
    x = _c128(x).copy()
    _check(lib().orc_fft1d(_ptr(x), x.shape[0], sign), "fft1d")
    return x


def fft2d(x, sign=-1):
    x = _c128(x).copy()
    _check(lib().orc_fft2d(_ptr(x), x.shape[0], sign), "fft2d")
    return x


def fftfreq(n, d):
    q = np.empty(n, dtype=np.float64)
    lib().orc_fftfreq(n, float(d), _ptr(q))
    return q


def propagator(n, dx, lam, dz, tilt_y=0.0, tilt_x=0.0):
    h = np.empty((n, n), dtype=np.complex128)
    lib().orc_propagator(n, float(dx), float(lam), float(dz), float(tilt_y), float(tilt_x), _ptr(h))
    return h


def probe(n, dx, lam, alpha, defocus):
    p = np.empty((n, n), dtype=np.complex128)
    _check(lib().orc_probe(n, float(dx), float(lam), float(alpha), float(defocus), _ptr(p)), "probe")
    return p


def probe_aberrated(n, dx, lam, alpha, c1, a1=0.0, phi_a1=0.0, c3=0.0):
    """Probe with defocus C1, twofold astigmatism A1 at phi_A1 and spherical aberration C3."""
    out = np.empty((n, n), dtype=np.complex128)
    _check(lib().orc_probe_aberrated(int(n), float(dx), float(lam), float(alpha), float(c1), float(a1),
                                     float(phi_a1), float(c3), _ptr(out)), "probe_aberrated")
    return out


def shift(p, fy, fx):
    p = _c128(p)
    out = np.empty_like(p)
    _check(lib().orc_shift(_ptr(p), p.shape[0], float(fy), float(fx), _ptr(out)), "shift")
    return out


def unshift(g, fy, fx):
    g = _c128(g)
    out = np.empty_like(g)
    _check(lib().orc_unshift(_ptr(g), g.shape[0], float(fy), float(fx), _ptr(out)), "unshift")
    return out


class Model:
    """A multislice geometry: window N, periodic H x W object, M slices, S positions."""

    def __init__(self, n, obj_h, obj_w, n_slices, positions, dz, pixel_size, wavelength,
                 tilt_y=0.0, tilt_x=0.0, n_threads=0, objective=0):
        self.n, self.obj_h, self.obj_w, self.n_slices = int(n), int(obj_h), int(obj_w), int(n_slices)
        self.positions = _f64(np.asarray(positions).reshape(-1, 2))
        self.dz = _f64(np.asarray(dz).reshape(-1)) if n_slices > 1 else np.zeros(1)
        self.pb = Problem(self.n, self.obj_h, self.obj_w, self.n_slices, self.positions.shape[0],
                          self.positions.ctypes.data, self.dz.ctypes.data, float(pixel_size),
                          float(wavelength), float(tilt_y), float(tilt_x), int(n_threads), int(objective))

    @classmethod
    def from_geometry(cls, geo, positions=None, n_threads=0, objective=0):
        pos = geo.positions() if positions is None else positions
        return cls(geo.n, geo.obj_h, geo.obj_w, geo.n_slices, pos, geo.gaps(), geo.pixel_size,
                   geo.wavelength, n_threads=n_threads, objective=objective)

    @property
    def n_pos(self):
        return self.positions.shape[0]

    def forward(self, probe, slices, exit_waves=False):
        """Returns intensities (S, N, N) float64 and, if asked, exit waves E_M (S, N, N)."""
        pr, sl = _c128(probe), _c128(slices)
        inten = np.empty((self.n_pos, self.n, self.n), dtype=np.float64)
        ew = np.empty((self.n_pos, self.n, self.n), dtype=np.complex128) if exit_waves else None
        _check(lib().orc_forward(C.byref(self.pb), _ptr(pr), _ptr(sl), _ptr(inten), _ptr(ew)), "forward")
        return (inten, ew) if exit_waves else inten

    def loss_grad(self, probe, slices, measured, subset=None, layer=-1, want_slices=True,
                  want_probe=True, want_overlap=False):
        """Loss, slice gradient, probe gradient and (layer mode) overlap map."""
        pr, sl, ms = _c128(probe), _c128(slices), _f64(measured)
        sub = None if subset is None else np.ascontiguousarray(subset, dtype=np.int64)
        hw = (self.obj_h, self.obj_w)
        gs = None
        if want_slices:
            gs = np.empty(hw if layer >= 0 else (self.n_slices,) + hw, dtype=np.complex128)
        gp = np.empty((self.n, self.n), dtype=np.complex128) if want_probe else None
        ov = np.empty(hw, dtype=np.float64) if (want_overlap and layer >= 0) else None
        loss = np.zeros(1, dtype=np.float64)
        rc = lib().orc_loss_grad(C.byref(self.pb), _ptr(pr), _ptr(sl), _ptr(ms), _ptr(sub),
                                 0 if sub is None else len(sub), int(layer), _ptr(gs), _ptr(gp),
                                 _ptr(ov), _ptr(loss))
        _check(rc, "loss_grad")
        return float(loss[0]), gs, gp, ov

    def loss(self, probe, slices, measured, subset=None):
        return self.loss_grad(probe, slices, measured, subset, want_slices=False, want_probe=False)[0]

    def position_grad(self, probe, slices, measured):
        """Returns (loss, dL/dposition (S, 2), curvature bound (S, 2)), y then x."""
        pr, sl, ms = _c128(probe), _c128(slices), _f64(measured)
        g = np.empty((self.n_pos, 2))
        c = np.empty((self.n_pos, 2))
        loss = np.zeros(1)
        _check(lib().orc_position_grad(C.byref(self.pb), _ptr(pr), _ptr(sl), _ptr(ms), _ptr(g), _ptr(c), _ptr(loss)),
               "position_grad")
        return float(loss[0]), g, c

    def layer_step(self, probe, slices, measured, layer, k_steps=1):
        """Returns (new slices, loss before the last step, step size of the last step)."""
        pr, sl, ms = _c128(probe), _c128(slices).copy(), _f64(measured)
        loss = np.zeros(1)
        mu = np.zeros(1)
        _check(lib().orc_layer_step(C.byref(self.pb), _ptr(pr), _ptr(sl), _ptr(ms), int(layer),
                                    int(k_steps), _ptr(loss), _ptr(mu)), "layer_step")
        return sl, float(loss[0]), float(mu[0])

    def full_step(self, probe, slices, measured, k_steps=1, step_scale=1.0):
        """Returns (new slices, loss before the last step, the M step sizes of the last step)."""
        pr, sl, ms = _c128(probe), _c128(slices).copy(), _f64(measured)
        loss = np.zeros(1)
        mu = np.zeros(self.n_slices)
        _check(lib().orc_full_step(C.byref(self.pb), _ptr(pr), _ptr(sl), _ptr(ms), int(k_steps), float(step_scale),
                                   _ptr(loss), _ptr(mu)), "full_step")
        return sl, float(loss[0]), mu

    def probe_step(self, probe, slices, measured, subset=None, k_steps=1):
        """Returns (new probe, loss before the last step, step size of the last step)."""
        pr, sl, ms = _c128(probe).copy(), _c128(slices), _f64(measured)
        sub = None if subset is None else np.ascontiguousarray(subset, dtype=np.int64)
        loss = np.zeros(1)
        mu = np.zeros(1)
        _check(lib().orc_probe_step(C.byref(self.pb), _ptr(pr), _ptr(sl), _ptr(ms), _ptr(sub),
                                    0 if sub is None else len(sub), int(k_steps), _ptr(loss),
                                    _ptr(mu)), "probe_step")
        return pr, float(loss[0]), float(mu[0])


def layerwise(model: Model, probe, slices, measured, sweeps: int, k_steps: int = 1,
              probe_steps: int = 0, subset=None):
    """Algorithm 1 (layer-wise estimation): for each sweep, one gradient block per
    layer l = 1..M in order (Gauss-Seidel), optionally followed by probe steps.
    Returns (slices, probe, per-step loss list)."""
    sl = _c128(slices).copy()
    pr = _c128(probe).copy()
    hist = []
    for _ in range(sweeps):
        for layer in range(model.n_slices):
            sl, loss, _mu = model.layer_step(pr, sl, measured, layer, k_steps)
            hist.append(loss)
        if probe_steps:
            pr, loss, _mu = model.probe_step(pr, sl, measured, subset, probe_steps)
            hist.append(loss)
    return sl, pr, hist
