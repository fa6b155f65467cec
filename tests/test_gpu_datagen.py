"""GPU checks of the training-data generator.

* Specimens: the device kernel (pixel by pixel, FP64 sums, FP32 output) against the FP64
  reference built atom by atom from the same Philox4x32-10 counters.  Bar: the FP32 rounding of
  V plus the few pixels where a site sits exactly at the 5-sigma cut on one side and not the
  other (each worth at most 3 exp(-12.5) = 1.1e-5): max |difference| <= 3e-5.
* Poisson noise: a different generator from numpy's, so not comparable value by value; its
  mean and variance are checked within 5 standard errors and its histogram by a chi-square
  test, below and above the switch from inversion to transformed rejection (mean 10).
* Crops and the learned initialisation: exact index maps, FP32 transcendental accuracy.
"""
import numpy as np
import pytest
import scipy.stats

from oracle import datagen as ref

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


@pytest.mark.parametrize("shape,index,vmax", [((2, 96, 128), 7, 0.05), ((6, 320, 320), 30001, 0.05),
                                              ((3, 64, 80), 5, 0.5)])
def test_specimen_matches_the_reference(dev, shape, index, vmax):
    from paper_2205_03902_amd import datagen
    M, H, W = shape
    print(f"[case] specimen {shape} index {index}", flush=True)
    fam = datagen.SpecimenFamily(M, H, W, vacancy_max=vmax, seed=30)
    pot = torch.empty(shape, dtype=torch.float32, device=dev)
    sl = torch.empty(shape, dtype=torch.complex64, device=dev)
    datagen.make_specimen(fam, index, 0.5, potential=pot, slices=sl)
    V, _, _, _ = ref.specimen(M, H, W, 0.2, 0.3, 0.1, 3.5, 4.2, vmax, True, 30, index)
    got = pot.cpu().numpy()
    assert np.abs(got - V).max() <= 3e-5
    t = sl.cpu().numpy()
    assert np.abs(t - np.exp(0.5j * V)).max() <= 2e-5


@pytest.mark.parametrize("lam", [0.3, 4.0, 9.99, 10.0, 37.5, 300.0])
def test_poisson_statistics(dev, lam):
    from paper_2205_03902_amd import datagen
    n_pix = 64 * 64
    dose = 1e5
    count = 1 << 20
    inten = torch.full((count // n_pix, 64, 64), lam * n_pix / dose, dtype=torch.float32, device=dev)
    out = datagen.poisson(inten, dose, seed=99, stream_id=int(lam * 100))
    k = np.rint(out.double().cpu().numpy().ravel() * dose / n_pix).astype(np.int64)
    assert np.allclose(k, out.double().cpu().numpy().ravel() * dose / n_pix, atol=1e-3 * max(1.0, lam))
    se = np.sqrt(lam / count)
    assert abs(k.mean() - lam) < 5 * se
    # variance: its standard error is about lam sqrt(2 / count) for large lam
    assert abs(k.var() - lam) < 5 * np.sqrt((2 * lam * lam + lam) / count)
    lo, hi = int(scipy.stats.poisson.ppf(1e-4, lam)), int(scipy.stats.poisson.ppf(1 - 1e-4, lam))
    edges = np.arange(lo, hi + 2)
    obs, _ = np.histogram(np.clip(k, lo, hi), bins=edges)
    p = scipy.stats.poisson.pmf(np.arange(lo, hi + 1), lam)
    p[0] += scipy.stats.poisson.cdf(lo - 1, lam)
    p[-1] += scipy.stats.poisson.sf(hi, lam)
    exp = p * count
    keep = exp >= 5
    chi2 = ((obs[keep] - exp[keep]) ** 2 / exp[keep]).sum() + 0.0
    dof = keep.sum() - 1
    assert scipy.stats.chi2.sf(chi2, dof) > 1e-4, (chi2, dof)


def test_poisson_is_deterministic_per_seed_and_independent_across_streams(dev):
    from paper_2205_03902_amd import datagen
    inten = torch.full((4, 32, 32), 50.0 * 1024 / 1e5, dtype=torch.float32, device=dev)
    a = datagen.poisson(inten, 1e5, 5, 1)
    b = datagen.poisson(inten, 1e5, 5, 1)
    c = datagen.poisson(inten, 1e5, 5, 2)
    assert torch.equal(a, b) and not torch.equal(a, c)
    zero = datagen.poisson(torch.zeros_like(inten), 1e5, 5, 1)
    assert torch.count_nonzero(zero).item() == 0


def test_crops_and_initialisation(dev):
    from paper_2205_03902_amd import datagen, synth
    M, H, W = 6, 40, 48
    t = synth.unit_phase_field((M, H, W), 3, 3.0)
    pot = np.random.Generator(np.random.PCG64(4)).standard_normal((M, H, W)).astype(np.float32)
    tg = torch.from_numpy(t).to(dev)
    pg = torch.from_numpy(pot).to(dev)
    y0, x0, h, w = 30, 20, 16, 32            # wraps in y and x
    x = datagen.crop_phase(tg, y0, x0, h, w, 8).float().cpu().numpy()
    ys, xs = (y0 + np.arange(h)) % H, (x0 + np.arange(w)) % W
    want = np.angle(t[:, ys][:, :, xs]).transpose(1, 2, 0)
    assert np.abs(x[..., :M] - want).max() <= 2.0 ** -8 * np.pi + 1e-6
    assert np.all(x[..., M:] == 0)
    c = datagen.crop_potential(pg, y0, x0, h, w).cpu().numpy()
    assert np.array_equal(c, pot[:, ys][:, :, xs].transpose(1, 2, 0))
    vh = torch.from_numpy(c * 0.5).to(dev)
    datagen.apply_init(vh, tg, y0, x0, 0.7)
    out = tg.cpu().numpy()
    inside = np.exp(0.7j * (c * 0.5)).transpose(2, 0, 1)
    assert np.abs(out[:, ys][:, :, xs] - inside).max() <= 1e-6
    mask = np.ones((H, W), bool)
    mask[np.ix_(ys, xs)] = False
    assert np.array_equal(out[:, mask], t[:, mask])
