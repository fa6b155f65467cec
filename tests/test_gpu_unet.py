"""GPU parity of the learned-initialisation network against the FP64 reference (oracle/unet.py).

Both sides get the same weights, rounded once to bfloat16 (what the matrix cores read), and
the same bfloat16 input.  Bars, from the arithmetic:
  * one operation on the GPU's own input activations: FP32 accumulation plus one bfloat16
    rounding of the output (relative 2^-9 per element): relative L2 <= 4e-3; the pooling is
    exact; the FP32 head output <= 1e-5;
  * the whole network: every stored activation and activation gradient is rounded to
    bfloat16, about 20 roundings deep: relative L2 <= 3e-2 for the output and <= 5e-2 for
    each layer's weight gradient;
  * Adam (FP32) against the FP64 update applied to the GPU's gradient: 1e-6.
"""
import numpy as np
import pytest

from oracle import unet as ref

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _bf16(a):
    return torch.from_numpy(np.asarray(a, dtype=np.float32)).to(torch.bfloat16).to(torch.float64).numpy()


def _rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _setup(dev, in_ch, out_ch, base, levels, h, w, batch, seed):
    from paper_2205_03902_amd import unet
    print(f"[case] unet in={in_ch} out={out_ch} base={base} levels={levels} {h}x{w} batch={batch}", flush=True)
    rng = np.random.Generator(np.random.PCG64(seed))
    params = ref.init_params(in_ch, out_ch, seed, base=base, levels=levels)
    params = {k: (_bf16(wt), rng.standard_normal(b.shape) * 0.05) for k, (wt, b) in params.items()}
    params = {k: (wt, b.astype(np.float32).astype(np.float64)) for k, (wt, b) in params.items()}
    x = _bf16(rng.standard_normal((batch, in_ch, h, w)))
    target = rng.standard_normal((batch, out_ch, h, w)).astype(np.float32).astype(np.float64)
    net = unet.UNet(in_ch, out_ch, base=base, levels=levels, height=h, width=w, max_batch=batch, device=dev)
    net.set_params(params)
    xg = unet.to_nhwc_bf16(torch.from_numpy(x).to(dev), net.in_pad)
    tg = torch.from_numpy(target).permute(0, 2, 3, 1).contiguous().float().to(dev)
    return net, params, x, target, xg, tg


def _nchw(t):
    return t.permute(0, 3, 1, 2).double().cpu().numpy()


# (in, out, base, levels, height, width, batch, seed). The fourth and fifth cases reach the
# direct 3x3 convolution, which takes images of 64 rows and more: 32 channels at 128 x 64 (two
# row tiles, the concatenation's 64 input channels, its gradient split 32 / 32 over the two
# sources) and 64 channels at 128 x 128 (two 32-channel launches a layer, the gradient split
# 64 / 64).  The sixth has 12 input channels, padded to 16, as the network of the 12-slice
# workload has (its input layer on the implicit GEMM), over 4 levels of a non-square image.
# The last case is the deployed network (4 levels, 32 base channels, 256 x 256 crops of 6 slices,
# the only shape with 256-channel layers), at batch 1.
CASES = [(3, 2, 8, 3, 16, 32, 2, 1), (6, 6, 16, 4, 32, 32, 2, 2), (8, 1, 8, 1, 8, 16, 3, 3),
         (6, 6, 32, 2, 128, 64, 2, 4), (4, 3, 64, 2, 128, 128, 1, 6), (12, 12, 16, 4, 64, 128, 2, 7),
         (6, 6, 32, 4, 256, 256, 1, 5)]


@pytest.mark.parametrize("case", CASES)
def test_each_operation_on_the_gpus_own_activations(dev, case):
    in_ch, out_ch, base, levels, h, w, batch, seed = case
    net, params, x, _, xg, _ = _setup(dev, *case)
    y = _nchw(net.forward(xg))
    torch.cuda.synchronize()
    act = lambda i: _nchw(net.activation(i)[:batch])
    L = levels
    h_in = x
    for l in range(L):
        (w0, b0), (w1, b1) = params[f"enc{l}.conv0"], params[f"enc{l}.conv1"]
        a0, a1 = act(3 * l), act(3 * l + 1)
        e0 = _rel(a0, ref.relu(ref.conv2d(h_in, w0, b0)))
        e1 = _rel(a1, ref.relu(ref.conv2d(a0, w1, b1)))
        assert e0 < 4e-3 and e1 < 4e-3, (l, e0, e1)
        if l < L - 1:
            p = act(3 * l + 2)
            assert np.array_equal(p, ref.maxpool2(a1)), l
            h_in = p
        else:
            h_in = a1
    for l in reversed(range(L - 1)):
        (wu, bu), (w0, b0), (w1, b1) = params[f"dec{l}.up"], params[f"dec{l}.conv0"], params[f"dec{l}.conv1"]
        up, a0, a1 = act(3 * L + 3 * l), act(3 * L + 3 * l + 1), act(3 * L + 3 * l + 2)
        eu = _rel(up, ref.conv_transpose2(h_in, wu, bu))
        e0 = _rel(a0, ref.relu(ref.conv2d(np.concatenate([up, act(3 * l + 1)], axis=1), w0, b0)))
        e1 = _rel(a1, ref.relu(ref.conv2d(a0, w1, b1)))
        assert eu < 4e-3 and e0 < 4e-3 and e1 < 4e-3, (l, eu, e0, e1)
        h_in = a1
    wh, bh = params["head"]
    assert _rel(y, ref.conv2d(h_in, wh, bh, pad=0)) < 1e-5


def _gpu_cache(net, x, levels, batch):
    """The reference's backward cache filled with the GPU's own (bfloat16) activations, so that
    both sides take the ReLU-mask and pooling-argmax decisions on the same values."""
    act = lambda i: _nchw(net.activation(i)[:batch])
    L = levels
    cache, h = {"x": x}, x
    for l in range(L):
        cache[f"enc{l}.in"], cache[f"enc{l}.a0"], cache[f"enc{l}.a1"] = h, act(3 * l), act(3 * l + 1)
        h = act(3 * l + 2) if l < L - 1 else cache[f"enc{l}.a1"]
    for l in reversed(range(L - 1)):
        cache[f"dec{l}.in"] = h
        cache[f"dec{l}.cat"] = np.concatenate([act(3 * L + 3 * l), act(3 * l + 1)], axis=1)
        cache[f"dec{l}.a0"], cache[f"dec{l}.a1"] = act(3 * L + 3 * l + 1), act(3 * L + 3 * l + 2)
        h = cache[f"dec{l}.a1"]
    cache["head.in"] = h
    return cache


@pytest.mark.parametrize("case", CASES)
def test_network_output_and_gradients_match_the_reference(dev, case):
    in_ch, out_ch, base, levels, h, w, batch, seed = case
    net, params, x, target, xg, tg = _setup(dev, *case)
    y, loss = net.backward(xg, tg)
    torch.cuda.synchronize()
    y_gpu = _nchw(y)
    # forward: the FP64 network from scratch
    y_ref, _ = ref.unet_forward(params, x, levels)
    ey = _rel(y_gpu, y_ref)
    # backward: the FP64 backward pass through the GPU's activations and output
    l_ref, dy = ref.centered_mse(y_gpu, target)
    g_ref = ref.unet_backward(params, _gpu_cache(net, x, levels, batch), dy, levels)
    el = abs(loss.item() - l_ref) / l_ref
    shapes = {k: v[0].shape for k, v in params.items()}
    grads = net.get_grads(shapes)
    worst = max((_rel(grads[k][0], g_ref[k][0]), k) for k in g_ref)
    worst_b = max((_rel(grads[k][1], g_ref[k][1]), k) for k in g_ref if k != "head")
    print(f"unet {case}: output {ey:.2e} loss {el:.2e} worst dW {worst} worst db {worst_b}")
    assert ey < 3e-2 and el < 1e-9
    assert worst[0] < 2e-2 and worst_b[0] < 2e-2
    # the head bias gradient is sum(d loss / d y) over pixels, zero for the centred loss: it
    # is only the sum of the rounding errors of the bfloat16 output gradient
    assert np.abs(grads["head"][1]).max() <= 1e-2 * np.abs(dy).sum(axis=(0, 2, 3)).max()


def test_loss_and_its_gradient_on_the_gpus_own_output(dev):
    """The loss kernel alone: FP64 statistics of the GPU output against the reference formula."""
    net, params, x, target, xg, tg = _setup(dev, *CASES[0])
    y, loss = net.backward(xg, tg)
    l_ref, _ = ref.centered_mse(_nchw(y), target)
    assert abs(loss.item() - l_ref) <= 1e-9 * l_ref


def test_adam_step_matches_the_reference_update(dev):
    net, params, x, target, xg, tg = _setup(dev, *CASES[1])
    shapes = {k: v[0].shape for k, v in params.items()}
    m, v = {}, {}
    for t in range(1, 4):
        net.backward(xg, tg)
        before, g = net.get_params(shapes), net.get_grads(shapes)
        net.adam_step(lr=1e-3)
        after = net.get_params(shapes)
        for k in g:
            for j in range(2):
                key = (k, j)
                m.setdefault(key, np.zeros_like(g[k][j], dtype=np.float64))
                v.setdefault(key, np.zeros_like(g[k][j], dtype=np.float64))
                p, m[key], v[key] = ref.adam_step(before[k][j].astype(np.float64), g[k][j].astype(np.float64),
                                                  m[key], v[key], t)
                assert np.abs(after[k][j] - p).max() <= 1e-6 * max(1.0, np.abs(p).max()), (t, k, j)


def test_training_steps_reduce_the_loss(dev):
    net, params, x, target, xg, tg = _setup(dev, *CASES[1])
    losses = []
    for _ in range(30):
        _, loss = net.backward(xg, tg)
        losses.append(loss.item())
        net.adam_step(lr=1e-3)
    assert losses[-1] < 0.8 * losses[0], losses


def test_full_size_network_first_layers_and_finite_output(dev):
    """The 4-level, 32-wide network on 256 x 256 crops of 6 slices (the deployed shape)."""
    net, params, x, target, xg, tg = _setup(dev, 6, 6, 32, 4, 256, 256, 2, 5)
    y, loss = net.backward(xg, tg)
    assert torch.isfinite(y).all() and np.isfinite(loss.item())
    a0 = _nchw(net.activation(0)[:1])
    w0, b0 = params["enc0.conv0"]
    assert _rel(a0, ref.relu(ref.conv2d(x[:1], w0, b0))) < 4e-3
    p = _nchw(net.activation(2)[:1])
    assert np.array_equal(p, ref.maxpool2(_nchw(net.activation(1)[:1])))


def test_whole_object_network_of_the_12_slice_workload(dev):
    """The instance that initialises the whole 1024^2 object of the 12-slice workload (12 channels,
    padded to 16; the trained weights of the 256^2 network): its first layer on an interior patch
    against the FP64 convolution, the first pooling exactly, and a finite output."""
    net, params, x, target, xg, tg = _setup(dev, 12, 12, 32, 4, 1024, 1024, 1, 9)
    y = net.forward(xg)
    torch.cuda.synchronize()
    assert torch.isfinite(y).all()
    y0, x0 = 500, 300
    a0 = _nchw(net.activation(0)[:, y0:y0 + 64, x0:x0 + 64].contiguous())
    w0, b0 = params["enc0.conv0"]
    ref0 = ref.relu(ref.conv2d(x[:, :, y0 - 1:y0 + 65, x0 - 1:x0 + 65], w0, b0))[:, :, 1:65, 1:65]
    assert _rel(a0, ref0) < 4e-3
    p = _nchw(net.activation(2)[:, 250:282, 150:182].contiguous())
    assert np.array_equal(p, ref.maxpool2(_nchw(net.activation(1)[:, 500:564, 300:364].contiguous())))
