"""Pins of the training-data reference (oracle/datagen.py): Philox4x32-10 known-answer vectors
(published with the Random123 library), closed forms of the Gaussian-atom potential, and the
statistics of the site draws."""
import math

import numpy as np
import pytest

from oracle import datagen as dg

# counter, key -> output (Random123 known-answer tests for philox4x32, 10 rounds)
KAT = [
    ([0, 0, 0, 0], [0, 0], [0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8]),
    ([0xFFFFFFFF] * 4, [0xFFFFFFFF, 0xFFFFFFFF], [0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD]),
    ([0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344], [0xA4093822, 0x299F31D0],
     [0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1]),
]


@pytest.mark.parametrize("ctr,key,want", KAT)
def test_philox_known_answers(ctr, key, want):
    got = dg.philox4x32(np.array(ctr, dtype=np.uint64), np.array(key, dtype=np.uint64))
    assert [int(v) for v in got] == want


def test_philox_vectorised_matches_one_by_one():
    ctr = np.array([[i, 7 * i, 3, 1] for i in range(5)], dtype=np.uint64)
    key = np.array([11, 12], dtype=np.uint64)
    many = dg.philox4x32(ctr, key)
    for i in range(5):
        assert np.array_equal(many[i], dg.philox4x32(ctr[i], key))


SPEC = dict(n_slices=2, obj_h=96, obj_w=128, dx=0.2, sigma=0.3, jitter=0.1, a_min=3.5, a_max=4.2,
            vacancy_max=0.05, two_species=True, seed=30, index=7)


def test_each_pixel_sees_at_most_one_site_so_the_value_is_closed_form():
    V, sites, a, vac = dg.specimen(**SPEC)
    dx, s = SPEC["dx"], SPEC["sigma"]
    H, W = SPEC["obj_h"], SPEC["obj_w"]
    checked = 0
    for m, (py, px, amp) in enumerate(sites):
        for ya, xa, am in zip(py, px, amp):
            iy, ix = int(round(ya / dx)), int(round(xa / dx))
            d2 = (ya - iy * dx) ** 2 + (xa - ix * dx) ** 2
            assert abs(V[m, iy % H, ix % W] - am * math.exp(-d2 / (2 * s * s))) < 1e-12
            checked += 1
    assert checked == sum(len(p[0]) for p in sites)


def test_integral_of_the_potential_is_the_sum_of_the_gaussian_masses():
    V, sites, a, vac = dg.specimen(**SPEC)
    s, dx = SPEC["sigma"], SPEC["dx"]
    for m in range(SPEC["n_slices"]):
        mass = 2 * math.pi * s * s * sites[m][2].sum()
        # the square 5-sigma cut drops 1 - erf(5/sqrt 2)^2 = 1.1e-6 of each atom
        assert abs(V[m].sum() * dx * dx / mass - 1.0) < 3e-6


def test_lattice_and_site_statistics():
    spec = dict(SPEC, obj_h=512, obj_w=512, n_slices=4, vacancy_max=1.0, index=3)
    V, sites, a, vac = dg.specimen(**spec)
    assert spec["a_min"] <= a <= spec["a_max"] and 0 <= vac <= 1
    amp = np.concatenate([p[2] for p in sites])
    n = amp.size
    ny = [int(math.ceil((512 * 0.2 - 0.0) / a))]
    assert n >= 4 * (ny[0] - 1) ** 2
    empty = np.mean(amp == 0)
    assert abs(empty - vac) < 5 * math.sqrt(vac * (1 - vac) / n) + 1e-3
    alive = amp[amp > 0]
    # light amplitudes lie in [0.5, 1.5), heavy ones in [1, 3): P(A > 1.5) = 1/2 * 3/4
    heavy = np.mean(alive > 1.5)
    assert abs(heavy - 0.375) < 5 * math.sqrt(0.375 * 0.625 / alive.size)
    # jitter: the site positions minus the lattice, standard deviation 0.1 A
    for m in range(4):
        py = sites[m][0]
        resid = (py - py.min()) % a
        resid = np.where(resid > a / 2, resid - a, resid)
        resid -= resid.mean()
        assert abs(resid.std() - 0.1) < 0.01
