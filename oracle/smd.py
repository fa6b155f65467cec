"""FP64 reference of the sparse matrix decomposition (Algorithm 2, Sec. 3.4).

TEST INFRASTRUCTURE ONLY: used by the tests to check the device implementation; the
product path never imports it.  Plain dense numpy in the paper's order and notation:

  * the full-field model (object as large as the window, H = W = N, positions are
    integer shifts): the matrix of probes P in C^{N^2 x S} has the probe shifted to
    position s as column s, and A_M = O_M G_{M-1} ... G_1 O_1 is N^2 x N^2 with
    O_m = diag(t_m) and G_m = F_2D^{-1} diag(h_m) F_2D (eqs. Single_Multislice_Matrix,
    MultiSlice_FullMatrix);
  * step 1, eq. (Opt_Prob_Matrix): amplitude-flow steps on A,
      A <- A - mu F^H ((|F A P| - sqrt(I)) o F A P / |F A P|) P^H,  mu = 1 / (N^2 ||P||^2),
    with the phase taken as 0 where F A P = 0;
  * step 2, eq. (Prox_Min): for l = 1..M, with the prefix R_l = O_M G_{M-1} ... G_l and
    the suffix S_l = G_{l-1} O_{l-1} ... G_1 O_1 (R_M = S_1 = identity) of the slices of
    iteration t (the paper's R_l^t, S_l^t: every layer of a pass sees the same slices),
      O_l <- Proj(O_l - mu conj(lambda) diag(R_l^H (lambda R_l O_l S_l - A_hat) S_l^H)),
      mu = 1 / c,  c = (|lambda| prod_{m != l} max|o_m|)^2 >= (|lambda| ||R_l|| ||S_l||)^2
    (G_m is unitary, so each factor's norm is at most the largest entry of its diagonal),
    Proj keeping the diagonal scaled to unit Frobenius norm;
  * lambda = Tr(A_hat^H A~) / Tr(A~^H A~) (eq. Update Lambda), A~ = O_M prod G_m O_m;
  * the next A is lambda A~; the result is lambda^(1/M) O_m.

Readings: the paper's lambda is a complex scalar here, the least-squares value
Tr(A~^H A_hat) / Tr(A~^H A~) (its trace ratio with the conjugation on A~, which is real
lambda's formula when lambda is real); the matrix step uses the spectral norm of P;
F_2D is the unnormalised 2D DFT of the rest of the oracle, so ||F_2D||^2 = N^2.
"""
from __future__ import annotations

import numpy as np


def dft2_matrix(n: int) -> np.ndarray:
    """F_2D on row-major flattened N x N images: kron(F_N, F_N), F_N[k, j] = exp(-2 pi i j k / N)."""
    f = np.exp(-2j * np.pi * np.outer(np.arange(n), np.arange(n)) / n)
    return np.kron(f, f)


def propagator_matrix(h: np.ndarray) -> np.ndarray:
    """G = F^{-1} diag(h) F for an N x N propagator h (FFT order), F^{-1} = F^H / N^2."""
    n = h.shape[0]
    f2 = dft2_matrix(n)
    return (np.conj(f2).T / (n * n)) @ (h.reshape(-1)[:, None] * f2)


def probe_matrix(probe: np.ndarray, positions) -> np.ndarray:
    """Columns: the probe moved to each integer position (y, x) with periodic wrap."""
    cols = [np.roll(probe, (int(py), int(px)), axis=(0, 1)).reshape(-1) for py, px in positions]
    return np.stack(cols, axis=1)


def compose(slices: np.ndarray, gs) -> np.ndarray:
    """A = O_M G_{M-1} O_{M-1} ... G_1 O_1 (slices (M, N, N), gs the M-1 matrices G_m)."""
    a = np.diag(slices[0].reshape(-1))
    for m in range(1, slices.shape[0]):
        a = np.diag(slices[m].reshape(-1)) @ (gs[m - 1] @ a)
    return a


def matrix_loss(a: np.ndarray, p: np.ndarray, meas: np.ndarray) -> float:
    """1/2 || sqrt(I) - |F A P| ||_F^2, meas (N^2, S) in FFT order (columns = positions)."""
    n2 = a.shape[0]
    n = int(round(np.sqrt(n2)))
    z = dft2_matrix(n) @ a @ p
    return 0.5 * float(np.sum((np.sqrt(meas) - np.abs(z)) ** 2))


def estimate_a(a: np.ndarray, p: np.ndarray, meas: np.ndarray, steps: int):
    """Amplitude-flow steps on A; returns (A, loss before each step)."""
    n2 = a.shape[0]
    n = int(round(np.sqrt(n2)))
    f2 = dft2_matrix(n)
    mu = 1.0 / (n2 * np.linalg.norm(p, 2) ** 2)
    losses = []
    for _ in range(steps):
        z = f2 @ a @ p
        mag = np.abs(z)
        phase = np.where(mag == 0, 0, z / np.where(mag == 0, 1, mag))
        losses.append(0.5 * float(np.sum((np.sqrt(meas) - mag) ** 2)))
        r = (mag - np.sqrt(meas)) * phase
        a = a - mu * (np.conj(f2).T @ r) @ np.conj(p).T
    return a, losses


def prefix_suffix(slices: np.ndarray, gs, l: int):
    """R_l = O_M G_{M-1} ... O_{l+1} G_l and S_l = G_{l-1} O_{l-1} ... G_1 O_1 (0-based l)."""
    M = slices.shape[0]
    n2 = slices[0].size
    r = np.eye(n2, dtype=complex)
    for m in range(l + 1, M):
        r = np.diag(slices[m].reshape(-1)) @ gs[m - 1] @ r
    s = np.eye(n2, dtype=complex)
    for m in range(l):
        s = gs[m] @ np.diag(slices[m].reshape(-1)) @ s
    return r, s


def project(d: np.ndarray) -> np.ndarray:
    """The diagonal scaled to unit Frobenius norm."""
    return d / np.linalg.norm(d)


def decompose_pass(a_hat: np.ndarray, slices: np.ndarray, lam: complex, gs):
    """One pass over the layers l = 1..M (eq. Prox_Min) with the prefixes and suffixes of the
    incoming slices, then the lambda update.  Returns (slices, lambda, A~)."""
    old = slices.copy()
    new = slices.copy()
    M = slices.shape[0]
    peak = [np.abs(old[m]).max() for m in range(M)]
    for l in range(M):
        r, s = prefix_suffix(old, gs, l)
        o = old[l].reshape(-1)
        x = lam * (r @ (o[:, None] * s)) - a_hat
        grad = np.einsum("ik,ij,kj->k", np.conj(r), x, np.conj(s))      # diag(R^H X S^H)
        c = (abs(lam) * np.prod([peak[m] for m in range(M) if m != l])) ** 2
        o = project(o - (1.0 / c) * np.conj(lam) * grad)
        new[l] = o.reshape(old[l].shape)
    at = compose(new, gs)
    lam = np.vdot(at, a_hat) / np.vdot(at, at)        # Tr(A~^H A_hat) / Tr(A~^H A~)
    return new, lam, at


def algorithm2(probe, positions, meas, slices0, gs, iterations: int, a_steps: int):
    """Algorithm 2; returns (lambda^(1/M) O_m, lambda, history of the matrix loss)."""
    p = probe_matrix(probe, positions)
    slices = slices0.copy()
    M = slices.shape[0]
    lam = 1.0 + 0j
    a = compose(slices, gs)
    hist = []
    for _ in range(iterations):
        a_hat, losses = estimate_a(a, p, meas, a_steps)
        hist.append(losses[0])
        slices, lam, at = decompose_pass(a_hat, slices, lam, gs)
        a = lam * at
    return slices * lam ** (1.0 / M), lam, hist
