"""FP64 reference of the training-data generator: Philox4x32-10 and the lattice specimen.

TEST INFRASTRUCTURE ONLY: used by the tests to check the device generator; the
product path never imports it.  It shares no code with the GPU library: the
generator is written here from its published definition (Salmon, Moraes, Dror
and Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC 2011), and the
specimen is assembled the other way round from the device kernel (atom by atom,
each atom's Gaussian added to the pixels it reaches, instead of pixel by pixel).

Specimen definition (the same streams as the device): key (seed, specimen);
  counter (0xFFFFFFFF, 0, 0, 0): a = a_min + (a_max - a_min) u0, vacancy rate = vmax u1;
  counter (0xFFFFFFFE, m, 0, 0): origin of slice m = (a u0, a u1);
  counter (i, j, m, 1): site (i, j) at origin + (i a, j a) + jitter, for
      0 <= i < ceil((H dx - y0) / a), 0 <= j < ceil((W dx - x0) / a);
      jitter = clip(s sqrt(-2 ln((w0 + 1) / 2^32)) (cos, sin)(2 pi u1), -4 s, 4 s);
      amplitude 0.5 + u2, doubled if bit 31 of w3 is set (two species), zero if
      (w3 & 0xFFFFFF) / 2^24 < vacancy rate;
  u_k = w_k / 2^32.  V = sum of A exp(-d^2 / (2 sigma^2)) over sites, d the distance to
  the nearest periodic image, sites with |dy| or |dx| > 5 sigma left out.
"""
from __future__ import annotations

import math

import numpy as np

M0, M1 = 0xD2511F53, 0xCD9E8D57
W0, W1 = 0x9E3779B9, 0xBB67AE85
MASK = 0xFFFFFFFF


def philox4x32(counter, key, rounds: int = 10):
    """Philox4x32 on arrays: counter (..., 4) and key (2,) or (..., 2) of uint32 -> (..., 4) uint32."""
    c = [np.asarray(counter, dtype=np.uint64)[..., i] for i in range(4)]
    k = np.asarray(key, dtype=np.uint64)
    k0, k1 = k[..., 0].copy(), k[..., 1].copy()
    for r in range(rounds):
        if r > 0:
            k0 = (k0 + W0) & MASK
            k1 = (k1 + W1) & MASK
        p0 = np.uint64(M0) * c[0]
        p1 = np.uint64(M1) * c[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & np.uint64(MASK)
        hi1, lo1 = p1 >> np.uint64(32), p1 & np.uint64(MASK)
        c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
    return np.stack([x.astype(np.uint32) for x in c], axis=-1)


def _u(w):
    return np.asarray(w, dtype=np.float64) / 4294967296.0


def specimen(n_slices, obj_h, obj_w, dx, sigma, jitter, a_min, a_max, vacancy_max, two_species, seed, index):
    """Potentials V (M, H, W) float64 and the site lists [(y, x, amplitude) arrays per slice]."""
    key = np.array([seed, index], dtype=np.uint64)
    w = philox4x32([0xFFFFFFFF, 0, 0, 0], key)
    a = a_min + (a_max - a_min) * _u(w[0])
    vac = vacancy_max * _u(w[1])
    Ly, Lx = obj_h * dx, obj_w * dx
    V = np.zeros((n_slices, obj_h, obj_w))
    sites = []
    cut = 5.0 * sigma
    rad = int(math.ceil(cut / dx)) + 1
    for m in range(n_slices):
        o = philox4x32([0xFFFFFFFE, m, 0, 0], key)
        y0, x0 = a * _u(o[0]), a * _u(o[1])
        ny, nx = int(math.ceil((Ly - y0) / a)), int(math.ceil((Lx - x0) / a))
        ii, jj = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
        ctr = np.stack([ii.ravel(), jj.ravel(), np.full(ii.size, m), np.ones(ii.size)], axis=-1).astype(np.uint64)
        r = philox4x32(ctr, key)
        rho = np.sqrt(-2.0 * np.log((r[:, 0].astype(np.float64) + 1.0) / 4294967296.0))
        th = 2.0 * np.pi * _u(r[:, 1])
        jy = np.clip(jitter * rho * np.cos(th), -4 * jitter, 4 * jitter)
        jx = np.clip(jitter * rho * np.sin(th), -4 * jitter, 4 * jitter)
        py = y0 + ii.ravel() * a + jy
        px = x0 + jj.ravel() * a + jx
        amp = 0.5 + _u(r[:, 2])
        if two_species:
            amp = np.where(r[:, 3] >> np.uint32(31), 2.0 * amp, amp)
        amp = np.where((r[:, 3] & np.uint32(0xFFFFFF)).astype(np.float64) / 16777216.0 < vac, 0.0, amp)
        sites.append((py, px, amp))
        for ya, xa, am in zip(py, px, amp):
            if am == 0.0:
                continue
            cy, cx = int(math.floor(ya / dx)), int(math.floor(xa / dx))
            ys = np.arange(cy - rad, cy + rad + 1)
            xs = np.arange(cx - rad, cx + rad + 1)
            # nearest image of the site for every pixel of the window (pixel indices wrap)
            dyv = ya - ys * dx
            dxv = xa - xs * dx
            keep_y, keep_x = np.abs(dyv) <= cut, np.abs(dxv) <= cut
            g = np.exp(-(dyv[keep_y, None] ** 2 + dxv[None, keep_x] ** 2) / (2 * sigma * sigma))
            V[m][np.ix_(ys[keep_y] % obj_h, xs[keep_x] % obj_w)] += am * g
    return V, sites, a, vac
