"""Pins of the FP64 U-Net reference (oracle/unet.py) against independent
implementations of the same definitions: scipy's 2-D correlation, torch's CPU
float64 convolution / transposed convolution / pooling and its autograd,
torch's Adam, adjoint (dot-product) identities and finite differences."""
import numpy as np
import pytest
import scipy.signal

from oracle import unet

torch = pytest.importorskip("torch")
F = torch.nn.functional


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def test_single_channel_conv_is_scipy_correlate_same():
    r = _rng(1)
    x = r.standard_normal((1, 1, 11, 9))
    w = r.standard_normal((1, 1, 3, 3))
    y = unet.conv2d(x, w)
    ref = scipy.signal.correlate2d(x[0, 0], w[0, 0], mode="same", boundary="fill")
    assert np.abs(y[0, 0] - ref).max() < 1e-12


@pytest.mark.parametrize("pad,k", [(1, 3), (0, 1)])
def test_conv_matches_torch(pad, k):
    r = _rng(2)
    x = r.standard_normal((2, 5, 8, 6))
    w = r.standard_normal((7, 5, k, k))
    b = r.standard_normal(7)
    y = unet.conv2d(x, w, b, pad=pad)
    ref = F.conv2d(torch.from_numpy(x), torch.from_numpy(w), torch.from_numpy(b), padding=pad).numpy()
    assert np.abs(y - ref).max() < 1e-12


def test_transposed_conv_and_pool_match_torch():
    r = _rng(3)
    x = r.standard_normal((2, 6, 5, 4))
    w = r.standard_normal((6, 3, 2, 2))
    b = r.standard_normal(3)
    y = unet.conv_transpose2(x, w, b)
    ref = F.conv_transpose2d(torch.from_numpy(x), torch.from_numpy(w), torch.from_numpy(b), stride=2).numpy()
    assert np.abs(y - ref).max() < 1e-12
    z = r.standard_normal((2, 3, 8, 6))
    assert np.array_equal(unet.maxpool2(z), F.max_pool2d(torch.from_numpy(z), 2).numpy())


def test_transposed_conv_is_the_adjoint_of_the_strided_conv():
    """<convT(x), y> = <x, S(y)> with S(y)[c,i,j] = sum_{o,u,v} w[c,o,u,v] y[o,2i+u,2j+v]."""
    r = _rng(4)
    x = r.standard_normal((1, 4, 3, 5))
    w = r.standard_normal((4, 2, 2, 2))
    y = r.standard_normal((1, 2, 6, 10))
    s = F.conv2d(torch.from_numpy(y), torch.from_numpy(w), stride=2).numpy()
    assert abs(np.vdot(unet.conv_transpose2(x, w), y) - np.vdot(x, s)) < 1e-10


def test_conv_backward_adjoint_identities_and_finite_differences():
    r = _rng(5)
    x = r.standard_normal((2, 3, 6, 7))
    w = r.standard_normal((4, 3, 3, 3))
    dy = r.standard_normal((2, 4, 6, 7))
    dx, dw, db = unet.conv2d_backward(x, w, dy)
    # dx is the adjoint of x -> conv(x, w); dw the adjoint of w -> conv(x, w)
    assert abs(np.vdot(unet.conv2d(x, w), dy) - np.vdot(x, dx)) < 1e-10
    assert abs(np.vdot(unet.conv2d(x, w), dy) - np.vdot(w, dw)) < 1e-10
    assert np.allclose(db, dy.sum(axis=(0, 2, 3)))
    d = r.standard_normal(w.shape)
    eps = 1e-6
    fd = (np.vdot(unet.conv2d(x, w + eps * d), dy) - np.vdot(unet.conv2d(x, w - eps * d), dy)) / (2 * eps)
    assert abs(fd - np.vdot(d, dw)) < 1e-6 * abs(fd)


def test_transposed_conv_backward_adjoint_identities():
    r = _rng(6)
    x = r.standard_normal((2, 5, 4, 3))
    w = r.standard_normal((5, 3, 2, 2))
    dy = r.standard_normal((2, 3, 8, 6))
    dx, dw, db = unet.conv_transpose2_backward(x, w, dy)
    ip = np.vdot(unet.conv_transpose2(x, w), dy)
    assert abs(ip - np.vdot(x, dx)) < 1e-10 and abs(ip - np.vdot(w, dw)) < 1e-10
    assert np.allclose(db, dy.sum(axis=(0, 2, 3)))


def test_maxpool_backward_routes_to_the_first_maximum():
    x = np.zeros((1, 1, 4, 4))
    x[0, 0, 0, 1] = x[0, 0, 1, 0] = 2.0      # tie in the top-left window: (0,1) comes first
    x[0, 0, 3, 3] = 1.0
    x[0, 0, 2:4, 0:2] = -1.0                 # all equal: (0,0) of the window takes it
    dy = np.array([[[[1.0, 2.0], [3.0, 4.0]]]])
    dx = unet.maxpool2_backward(x, dy)
    want = np.zeros_like(x)
    want[0, 0, 0, 1] = 1.0
    want[0, 0, 0, 2] = 2.0                   # top-right window is all zero: its (0,0)
    want[0, 0, 2, 0] = 3.0
    want[0, 0, 3, 3] = 4.0
    assert np.array_equal(dx, want)


def test_centered_mse_ignores_a_constant_per_channel_and_has_the_right_gradient():
    r = _rng(7)
    p = r.standard_normal((2, 3, 5, 4))
    t = r.standard_normal((2, 3, 5, 4))
    l0, g = unet.centered_mse(p, t)
    shift = r.standard_normal((2, 3, 1, 1))
    l1, _ = unet.centered_mse(p + shift, t)
    assert abs(l0 - l1) < 1e-12
    assert unet.centered_mse(t + shift, t)[0] < 1e-28
    assert np.abs(g.sum(axis=(2, 3))).max() < 1e-14
    d = r.standard_normal(p.shape)
    eps = 1e-6
    fd = (unet.centered_mse(p + eps * d, t)[0] - unet.centered_mse(p - eps * d, t)[0]) / (2 * eps)
    assert abs(fd - np.vdot(g, d)) < 1e-7 * abs(fd)


def test_adam_matches_torch_and_the_first_step_closed_form():
    r = _rng(8)
    p0 = r.standard_normal(10)
    gs = [r.standard_normal(10) for _ in range(4)]
    tp = torch.tensor(p0, requires_grad=True)
    opt = torch.optim.Adam([tp], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    p, m, v = p0.copy(), np.zeros(10), np.zeros(10)
    for t, g in enumerate(gs, start=1):
        p, m, v = unet.adam_step(p, g, m, v, t)
        opt.zero_grad()
        tp.grad = torch.from_numpy(g.copy())
        opt.step()
        if t == 1:
            assert np.allclose(p, p0 - 1e-3 * gs[0] / (np.abs(gs[0]) + 1e-8), rtol=0, atol=1e-15)
    assert np.abs(p - tp.detach().numpy()).max() < 1e-15


def _torch_unet(params, x, levels):
    h = x
    skips = []
    for l in range(levels):
        w0, b0 = params[f"enc{l}.conv0"]
        w1, b1 = params[f"enc{l}.conv1"]
        h = F.relu(F.conv2d(F.relu(F.conv2d(h, w0, b0, padding=1)), w1, b1, padding=1))
        skips.append(h)
        if l < levels - 1:
            h = F.max_pool2d(h, 2)
    for l in reversed(range(levels - 1)):
        wu, bu = params[f"dec{l}.up"]
        w0, b0 = params[f"dec{l}.conv0"]
        w1, b1 = params[f"dec{l}.conv1"]
        h = torch.cat([F.conv_transpose2d(h, wu, bu, stride=2), skips[l]], dim=1)
        h = F.relu(F.conv2d(F.relu(F.conv2d(h, w0, b0, padding=1)), w1, b1, padding=1))
    wh, bh = params["head"]
    return F.conv2d(h, wh, bh)


def test_network_forward_and_gradients_match_torch_autograd():
    levels, base = 3, 4
    params = unet.init_params(in_ch=3, out_ch=2, seed=9, base=base, levels=levels)
    r = _rng(10)
    params = {k: (w, r.standard_normal(b.shape) * 0.1) for k, (w, b) in params.items()}
    x = r.standard_normal((2, 3, 16, 16))
    target = r.standard_normal((2, 2, 16, 16))
    y, cache = unet.unet_forward(params, x, levels)
    loss, dy = unet.centered_mse(y, target)
    grads = unet.unet_backward(params, cache, dy, levels)
    tparams = {k: (torch.tensor(w, requires_grad=True), torch.tensor(b, requires_grad=True))
               for k, (w, b) in params.items()}
    ty = _torch_unet(tparams, torch.from_numpy(x), levels)
    e = ty - torch.from_numpy(target)
    e = e - e.mean(dim=(2, 3), keepdim=True)
    tl = (e * e).mean()
    tl.backward()
    assert np.abs(y - ty.detach().numpy()).max() < 1e-10
    assert abs(loss - tl.item()) < 1e-12 * max(1.0, loss)
    assert set(grads) == set(params) == set(unet.layer_names(levels))
    for k, (tw, tb) in tparams.items():
        dw, db = grads[k]
        assert np.abs(dw - tw.grad.numpy()).max() < 1e-10 * max(1.0, np.abs(dw).max()), k
        assert np.abs(db - tb.grad.numpy()).max() < 1e-10 * max(1.0, np.abs(db).max()), k


def test_layer_shapes_of_the_full_network():
    s = unet.layer_shapes(6, 6)
    assert s["enc0.conv0"][0] == (32, 6, 3, 3) and s["enc3.conv1"][0] == (256, 256, 3, 3)
    assert s["dec2.up"][0] == (256, 128, 2, 2) and s["dec2.conv0"][0] == (128, 256, 3, 3)
    assert s["dec0.conv0"][0] == (32, 64, 3, 3) and s["head"][0] == (6, 32, 1, 1)
    assert len(unet.layer_names()) == 18
