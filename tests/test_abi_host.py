"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every entry point include/ms.h declares, and rejects bad problems before
anything is enqueued."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2205_03902_amd import abi, configs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "ms.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ms_[a-z_]+)\s*\(", text)))


def test_header_declares_the_abi():
    assert set(_declared()) == set(abi.SYMBOLS)


def test_library_exports_every_declared_symbol():
    lib = abi.lib()
    for name in _declared():
        assert hasattr(lib, name), name


def _pb(**kw):
    geo = configs.small()
    args = dict(n=geo.n, obj_h=geo.obj_h, obj_w=geo.obj_w, n_slices=geo.n_slices, positions=geo.positions(),
                dz=geo.gaps(), pixel_size=geo.pixel_size, wavelength=geo.wavelength)
    args.update(kw)
    return abi.make_problem(**args)


def test_workspace_size_accepts_a_valid_problem():
    pb, keep = _pb()
    ws = abi.workspace_size(pb)
    assert ws > 0
    # a budget smaller than one batch of everything forces batching but still fits
    ws_small = abi.workspace_size(pb, budget_bytes=ws // 2)
    assert 0 < ws_small <= ws // 2


def test_checkpoint_interval_sets_the_wave_storage():
    """checkpoint_every = k keeps floor((M - 1) / k) stored waves and one work slot a position instead
    of M; k = 0 takes the smallest k whose waves fit the budget with every position in one batch,
    and only below the k = M footprint cuts the positions into batches."""
    geo = configs.CFG4
    args = dict(n=geo.n, obj_h=geo.obj_h, obj_w=geo.obj_w, n_slices=geo.n_slices, positions=geo.positions(),
                dz=geo.gaps(), pixel_size=geo.pixel_size, wavelength=geo.wavelength)
    ws = {}
    for k in (1, 2, 3, 4, 12, 40):
        pb, keep = abi.make_problem(checkpoint_every=k, **args)
        ws[k] = abi.workspace_size(pb)
    assert ws[1] > ws[2] > ws[3] > ws[4] > ws[12] == ws[40]
    # one position's waves: 12 slots of 256^2 complex64 against 1 slot (+ the recomputation buffers)
    per_slot = geo.n_pos * geo.n * geo.n * 8
    assert ws[1] - ws[12] > 9 * per_slot
    pb, keep = abi.make_problem(checkpoint_every=0, **args)
    assert abi.workspace_size(pb) == ws[1]                      # no budget: every wave
    assert abi.workspace_size(pb, budget_bytes=ws[1]) == ws[1]
    assert abi.workspace_size(pb, budget_bytes=ws[3]) == ws[3]   # k = 2 does not fit, k = 3 does
    assert abi.workspace_size(pb, budget_bytes=ws[3] - 1) == ws[4]
    small = abi.workspace_size(pb, budget_bytes=ws[12] // 2)     # batches, no wave stored
    assert small <= ws[12] // 2
    pb, keep = abi.make_problem(checkpoint_every=-1, **args)
    with pytest.raises(abi.MsError) as e:
        abi.workspace_size(pb)
    assert e.value.status == abi.MS_ERR_INVALID_ARG


@pytest.mark.parametrize("kw, status", [
    (dict(n=24), abi.MS_ERR_INVALID_ARG),
    (dict(n=8), abi.MS_ERR_INVALID_ARG),
    (dict(n=512, obj_h=512, obj_w=512), abi.MS_ERR_INVALID_ARG),
    # more distinct sub-pixel offsets than the plan keeps shifted probes for
    (dict(positions=np.stack([np.arange(4100) * 1e-4, np.zeros(4100)], axis=1)), abi.MS_ERR_UNSUPPORTED),
    # more distinct slice distances than the fused kernel keeps in LDS at this window size
    (dict(n_slices=6, dz=np.array([1.0, 2.0, 3.0, 4.0, 5.0])), abi.MS_ERR_UNSUPPORTED),
    (dict(obj_h=16), abi.MS_ERR_INVALID_ARG),
    (dict(n_slices=0), abi.MS_ERR_INVALID_ARG),
    (dict(pixel_size=0.0), abi.MS_ERR_INVALID_ARG),
    (dict(wavelength=float("nan")), abi.MS_ERR_INVALID_ARG),
    (dict(positions=np.array([[0.0, float("inf")]])), abi.MS_ERR_INVALID_ARG),
])
def test_invalid_problems_are_rejected(kw, status):
    pb, keep = _pb(**kw)
    with pytest.raises(abi.MsError) as e:
        abi.workspace_size(pb)
    assert e.value.status == status
    assert abi.lib().ms_last_error().decode() != ""


def test_budget_too_small_is_reported():
    pb, keep = _pb()
    with pytest.raises(abi.MsError) as e:
        abi.workspace_size(pb, budget_bytes=1024)
    assert e.value.status == abi.MS_ERR_BUDGET


def test_null_arguments_are_rejected_without_a_device():
    lib = abi.lib()
    assert lib.ms_workspace_size(None, 0, None) == abi.MS_ERR_INVALID_ARG
    pb, keep = _pb()
    assert lib.ms_workspace_size(C.byref(pb), 0, None) == abi.MS_ERR_INVALID_ARG
    h = C.c_void_p()
    assert lib.ms_plan_create(C.byref(pb), None, 0, C.byref(h)) == abi.MS_ERR_INVALID_ARG
    # the compute calls validate their plan before touching the stream
    assert lib.ms_forward(None, None, None, None, None, None) == abi.MS_ERR_INVALID_ARG
    assert lib.ms_adjoint(None, None, None, None, None, None, None, None) == abi.MS_ERR_INVALID_ARG
    assert lib.ms_layer_step(None, None, 0, 1, None, None, None, None, None) == abi.MS_ERR_INVALID_ARG
    assert lib.ms_probe_step(None, None, 1, None, None, None, None, 0, None, None) == abi.MS_ERR_INVALID_ARG
    # the plan's switches reject a missing plan; its queries answer 0
    for setter in (lib.ms_plan_set_path, lib.ms_plan_set_bands, lib.ms_plan_set_kept_windows,
                   lib.ms_plan_set_layer_carry, lib.ms_plan_set_objective):
        assert setter(None, 1) == abi.MS_ERR_INVALID_ARG
        assert "NULL" in lib.ms_last_error().decode()
    assert lib.ms_plan_kept_windows(None) == 0 and lib.ms_plan_has_bands(None) == 0


def _unet_declared():
    text = open(os.path.join(ROOT, "include", "unet.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(un_[a-z_]+)\s*\(", text)))


def test_unet_header_declares_the_binding_and_the_library_exports_it():
    from paper_2205_03902_amd import unet
    assert set(_unet_declared()) == set(unet.SYMBOLS)
    L = unet.lib()
    for name in _unet_declared():
        assert hasattr(L, name), name


@pytest.mark.parametrize("kw", [dict(in_ch=0), dict(out_ch=17), dict(in_ch=17), dict(levels=0), dict(levels=6), dict(base=12),
                                dict(base=64, levels=4), dict(height=48), dict(width=4), dict(max_batch=0),
                                dict(height=8, levels=5, base=8)])
def test_unet_invalid_configs_are_rejected(kw):
    from paper_2205_03902_amd import unet
    args = dict(in_ch=6, out_ch=6, base=32, levels=4, height=256, width=256, max_batch=2)
    args.update(kw)
    cfg = unet.UnConfig(*[args[k] for k in ("in_ch", "out_ch", "base", "levels", "height", "width", "max_batch")])
    with pytest.raises(abi.MsError) as e:
        unet.workspace_size(cfg)
    assert e.value.status == abi.MS_ERR_INVALID_ARG
    assert unet.lib().un_last_error().decode() != ""


def test_unet_workspace_and_layer_table():
    from paper_2205_03902_amd import unet
    cfg = unet.UnConfig(6, 6, 32, 4, 256, 256, 4)
    ws = unet.workspace_size(cfg)
    assert 100e6 < ws < 4e9
    assert unet.workspace_size(unet.UnConfig(6, 6, 32, 4, 256, 256, 8)) > ws


def test_datagen_header_declares_the_binding_and_the_library_exports_it():
    from paper_2205_03902_amd import datagen
    text = open(os.path.join(ROOT, "include", "datagen.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    declared = set(re.findall(r"\b(dg_[a-z_]+)\s*\(", text))
    assert declared == set(datagen.SYMBOLS)
    L = datagen.lib()
    for name in declared:
        assert hasattr(L, name), name


def test_datagen_rejects_bad_arguments_without_a_device():
    from paper_2205_03902_amd import datagen
    L = datagen.lib()
    s = datagen.SpecimenFamily(2, 16, 16).struct(0)          # 3.2 A: smaller than two atom reaches
    assert L.dg_make_specimen(None, C.byref(s), 0.5, 1, None) == abi.MS_ERR_INVALID_ARG
    assert L.dg_poisson(None, None, 10, 64, 1e5, 1, 1, None) == abi.MS_ERR_INVALID_ARG
    assert L.dg_crop_phase(None, 1, 6, 32, 32, 0, 0, 64, 16, 8, 1) == abi.MS_ERR_INVALID_ARG
    assert L.dg_last_error().decode() != ""


def test_smd_header_declares_the_binding_and_the_library_exports_it():
    from paper_2205_03902_amd import smd
    text = open(os.path.join(ROOT, "include", "smd.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    declared = set(re.findall(r"\b(smd_[a-z_0-9]+)\s*\(", text))
    assert declared == set(smd.SYMBOLS)
    L = smd.lib()
    for name in declared:
        assert hasattr(L, name), name


@pytest.mark.parametrize("kw", [dict(n=12), dict(n=8), dict(n=128), dict(n_slices=0), dict(positions=[[0.5, 1.0]]),
                                dict(positions=[[0, 0]] * 257), dict(wavelength=0.0), dict(dz=[float("nan")])])
def test_smd_rejects_invalid_problems_without_a_device(kw):
    from paper_2205_03902_amd import smd
    args = dict(n=16, n_slices=2, positions=[[0, 0], [3, 5]], dz=[2.0], pixel_size=0.2, wavelength=0.0487)
    args.update(kw)
    pb, keep = smd.make_problem(**args)
    out = C.c_size_t(0)
    assert smd.lib().smd_workspace_size(C.byref(pb), C.byref(out)) == abi.MS_ERR_INVALID_ARG
    assert smd.lib().smd_last_error().decode() != ""


def test_smd_workspace_holds_the_dense_matrices():
    from paper_2205_03902_amd import smd
    pb, keep = smd.make_problem(32, 3, [[0, 0]] * 40, [2.0, 2.0], 0.2, 0.0487)
    ws = smd.workspace_size(pb)
    n2 = 32 * 32
    # one working matrix and the three suffixes; no F or G_m is ever formed
    assert ws >= (1 + 3) * n2 * n2 * 8
    assert ws < (1 + 3) * n2 * n2 * 8 + (64 << 20)
    handle = C.c_void_p()
    assert smd.lib().smd_plan_create(C.byref(pb), None, ws, C.byref(handle)) == abi.MS_ERR_INVALID_ARG
    assert smd.lib().smd_set_probe(None, None, None) == abi.MS_ERR_INVALID_ARG


def test_non_finite_losses_are_reported_with_their_status():
    abi.check_finite([1.0, 2.5e3], "ok")
    with pytest.raises(abi.MsError) as e:
        abi.check_finite([1.0, float("nan"), 3.0], "reconstruct")
    assert e.value.status == abi.MS_ERR_NOT_FINITE and "entry 1" in str(e.value)
    with pytest.raises(abi.MsError):
        abi.check_finite(float("inf"), "refine_positions")
    text = open(os.path.join(ROOT, "include", "ms.h")).read()
    assert re.search(r"MS_ERR_NOT_FINITE\s*=\s*-5", text)
