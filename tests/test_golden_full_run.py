"""The stored oracle reconstruction of config 1 (tests/golden/config1_full_run.txt) against the
oracle as it stands: the file's first loss is the oracle's loss at the run's start, its losses
never rise (the step rule of Sec. 3.2 is a majorised descent, Algorithm 1 and the probe step of
Sec. 3.5 take one such step at a time), and its samples have the shapes the GPU test reads."""
import os

import numpy as np
import pytest

from parity_cases import make_case, read_full_run

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def run():
    from paper_2205_03902_amd import configs
    return read_full_run(os.path.join(GOLDEN, "config1_full_run.txt"), configs.CFG1.n_slices)


def test_stored_run_has_every_step(run):
    from paper_2205_03902_amd import configs
    geo = configs.CFG1
    assert run.sweeps == 20 and len(run.losses) == run.sweeps * (geo.n_slices + 1)
    assert run.slices.shape == (geo.n_slices, len(run.rows), len(run.cols))
    assert run.probe.shape == (geo.n // run.probe_stride,) * 2
    assert np.isfinite(run.slices).all() and np.isfinite(run.probe).all()


def test_stored_spread_is_the_rounding_of_the_probe(run):
    # the second oracle run starts from the probe before its rounding to single precision: a
    # relative change below the unit roundoff 2^-24 (6e-8), and its end differs but stays close
    assert 0 < run.spread_probe_change < 2.0 ** -24
    assert 0 < abs(run.spread_final_loss - run.final_loss) / run.final_loss < 1e-2
    assert 0 < run.spread_slice_error < 5e-2 and 0 < run.spread_probe_error < 5e-2


def test_stored_losses_never_rise(run):
    assert (np.diff(run.losses) <= 1e-9 * run.losses[0]).all()
    assert run.final_loss <= run.losses[-1] * (1 + 1e-9)
    assert run.final_loss < 0.5 * run.losses[0]


def test_stored_start_is_the_oracles_loss_at_the_start(orc, run):
    from paper_2205_03902_amd import configs
    geo = configs.CFG1
    c = make_case(geo)
    p0 = orc.probe(geo.n, geo.pixel_size, geo.wavelength, geo.alpha,
                   run.defocus_factor * geo.defocus).astype(np.complex64)
    l0 = c.model.loss(p0, np.ones_like(c.truth), c.measured)
    assert abs(l0 - run.losses[0]) <= 1e-12 * l0
