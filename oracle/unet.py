"""FP64 reference of the learned-initialisation network (a 4-level U-Net).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark use it; the product path never imports it.  It shares no
code with the GPU library (which stores activations NHWC in bfloat16; this
module is NCHW in float64).

The network is not part of the paper; it follows the usual U-Net definition
(Ronneberger, Fischer and Brox, 2015): per level two 3x3 convolutions with
zero padding 1, each followed by ReLU; 2x2 max pooling between levels; on the
way up a 2x2 stride-2 transposed convolution (no activation), concatenated
with the encoder output of the same level ([upsampled, skip] channel order),
then two 3x3 convolution + ReLU; a final 1x1 convolution without activation.
Adam is Kingma and Ba (2015), Algorithm 1, with bias correction.

Every function writes out the definition with numpy primitives (padding,
tensordot over channels, one tap at a time); nothing is blocked or fused.
"""
from __future__ import annotations

import numpy as np


def relu(x):
    return np.maximum(x, 0.0)


def conv2d(x, w, b=None, pad=1):
    """Cross-correlation y[n,o,i,j] = b[o] + sum_{c,u,v} w[o,c,u,v] x[n,c,i+u-pad,j+v-pad], zeros outside."""
    n, cin, h, wd = x.shape
    cout, cin2, kh, kw = w.shape
    assert cin == cin2
    xp = np.pad(x, ((0, 0), (0, 0), (pad, pad), (pad, pad)))
    ho, wo = h + 2 * pad - kh + 1, wd + 2 * pad - kw + 1
    y = np.zeros((n, cout, ho, wo))
    for u in range(kh):
        for v in range(kw):
            patch = xp[:, :, u:u + ho, v:v + wo]                       # (n, c, ho, wo)
            y += np.einsum("oc,ncij->noij", w[:, :, u, v], patch, optimize=True)
    if b is not None:
        y += b[None, :, None, None]
    return y


def conv2d_backward(x, w, dy, pad=1):
    """Gradients of conv2d with respect to x, w and b, given dL/dy."""
    n, cin, h, wd = x.shape
    cout, _, kh, kw = w.shape
    ho, wo = dy.shape[2], dy.shape[3]
    xp = np.pad(x, ((0, 0), (0, 0), (pad, pad), (pad, pad)))
    dxp = np.zeros_like(xp)
    dw = np.zeros_like(w)
    for u in range(kh):
        for v in range(kw):
            patch = xp[:, :, u:u + ho, v:v + wo]
            dw[:, :, u, v] = np.einsum("noij,ncij->oc", dy, patch, optimize=True)
            dxp[:, :, u:u + ho, v:v + wo] += np.einsum("oc,noij->ncij", w[:, :, u, v], dy, optimize=True)
    dx = dxp[:, :, pad:pad + h, pad:pad + wd]
    db = dy.sum(axis=(0, 2, 3))
    return dx, dw, db


def maxpool2(x):
    """2x2 max pooling, stride 2 (H and W even)."""
    n, c, h, w = x.shape
    return x.reshape(n, c, h // 2, 2, w // 2, 2).max(axis=(3, 5))


def maxpool2_backward(x, dy):
    """Routes each pooled gradient to the first maximum of its 2x2 window, in the
    order (0,0), (0,1), (1,0), (1,1)."""
    n, c, h, w = x.shape
    dx = np.zeros_like(x)
    taken = np.zeros(dy.shape, dtype=bool)
    m = maxpool2(x)
    for u in range(2):
        for v in range(2):
            hit = (x[:, :, u::2, v::2] == m) & ~taken
            dx[:, :, u::2, v::2] = np.where(hit, dy, 0.0)
            taken |= hit
    return dx


def conv_transpose2(x, w, b=None):
    """2x2 stride-2 transposed convolution: y[n,o,2i+u,2j+v] = b[o] + sum_c x[n,c,i,j] w[c,o,u,v]."""
    n, cin, h, wd = x.shape
    cin2, cout, _, _ = w.shape
    assert cin == cin2
    y = np.zeros((n, cout, 2 * h, 2 * wd))
    for u in range(2):
        for v in range(2):
            y[:, :, u::2, v::2] = np.einsum("co,ncij->noij", w[:, :, u, v], x, optimize=True)
    if b is not None:
        y += b[None, :, None, None]
    return y


def conv_transpose2_backward(x, w, dy):
    dx = np.zeros_like(x)
    dw = np.zeros_like(w)
    for u in range(2):
        for v in range(2):
            g = dy[:, :, u::2, v::2]
            dx += np.einsum("co,noij->ncij", w[:, :, u, v], g, optimize=True)
            dw[:, :, u, v] = np.einsum("ncij,noij->co", x, g, optimize=True)
    return dx, dw, dy.sum(axis=(0, 2, 3))


def centered_mse(pred, target):
    """Mean squared error after removing each (sample, channel) mean over pixels,
    so that a constant phase offset per slice costs nothing.  Returns (loss, dL/dpred)."""
    e = pred - target
    e = e - e.mean(axis=(2, 3), keepdims=True)
    count = e.size
    return float((e * e).sum() / count), 2.0 * e / count


def adam_step(p, g, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step number t >= 1); returns (p, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v


def layer_names(levels: int = 4):
    """Parameter order of the network (the GPU library uses the same order)."""
    names = []
    for l in range(levels):
        names += [f"enc{l}.conv0", f"enc{l}.conv1"]
    for l in reversed(range(levels - 1)):
        names += [f"dec{l}.up", f"dec{l}.conv0", f"dec{l}.conv1"]
    names.append("head")
    return names


def layer_shapes(in_ch: int, out_ch: int, base: int = 32, levels: int = 4):
    """{name: (weight shape, bias length)}; 3x3 weights (Cout, Cin, 3, 3), transposed
    convolutions (Cin, Cout, 2, 2), head (out_ch, base, 1, 1)."""
    width = [base << l for l in range(levels)]
    shapes = {}
    cin = in_ch
    for l in range(levels):
        shapes[f"enc{l}.conv0"] = ((width[l], cin, 3, 3), width[l])
        shapes[f"enc{l}.conv1"] = ((width[l], width[l], 3, 3), width[l])
        cin = width[l]
    for l in reversed(range(levels - 1)):
        shapes[f"dec{l}.up"] = ((width[l + 1], width[l], 2, 2), width[l])
        shapes[f"dec{l}.conv0"] = ((width[l], 2 * width[l], 3, 3), width[l])
        shapes[f"dec{l}.conv1"] = ((width[l], width[l], 3, 3), width[l])
    shapes["head"] = ((out_ch, base, 1, 1), out_ch)
    return shapes


def init_params(in_ch: int, out_ch: int, seed: int, base: int = 32, levels: int = 4):
    """He-normal weights (std sqrt(2 / fan_in)) and zero biases, from a PCG64 stream."""
    rng = np.random.Generator(np.random.PCG64(seed))
    params = {}
    for name, (ws, nb) in layer_shapes(in_ch, out_ch, base, levels).items():
        fan_in = ws[0] * ws[2] * ws[3] if name.endswith(".up") else ws[1] * ws[2] * ws[3]
        params[name] = (rng.standard_normal(ws) * np.sqrt(2.0 / fan_in), np.zeros(nb))
    return params


def unet_forward(params, x, levels: int = 4):
    """Returns (output, cache) with every intermediate the backward pass needs."""
    cache = {"x": x}
    skips = []
    h = x
    for l in range(levels):
        w0, b0 = params[f"enc{l}.conv0"]
        w1, b1 = params[f"enc{l}.conv1"]
        a0 = relu(conv2d(h, w0, b0))
        a1 = relu(conv2d(a0, w1, b1))
        cache[f"enc{l}.in"], cache[f"enc{l}.a0"], cache[f"enc{l}.a1"] = h, a0, a1
        skips.append(a1)
        h = maxpool2(a1) if l < levels - 1 else a1
    for l in reversed(range(levels - 1)):
        wu, bu = params[f"dec{l}.up"]
        w0, b0 = params[f"dec{l}.conv0"]
        w1, b1 = params[f"dec{l}.conv1"]
        up = conv_transpose2(h, wu, bu)
        cat = np.concatenate([up, skips[l]], axis=1)
        a0 = relu(conv2d(cat, w0, b0))
        a1 = relu(conv2d(a0, w1, b1))
        cache[f"dec{l}.in"], cache[f"dec{l}.cat"], cache[f"dec{l}.a0"], cache[f"dec{l}.a1"] = h, cat, a0, a1
        h = a1
    wh, bh = params["head"]
    cache["head.in"] = h
    return conv2d(h, wh, bh, pad=0), cache


def unet_backward(params, cache, dy, levels: int = 4):
    """Gradients {name: (dW, db)} of the network, given dL/d(output)."""
    grads = {}
    wh, _ = params["head"]
    g, dw, db = conv2d_backward(cache["head.in"], wh, dy, pad=0)
    grads["head"] = (dw, db)
    dskip = [None] * levels
    # the forward pass met decoder levels deepest first, so the backward pass starts at level 0
    for l in range(levels - 1):
        w0, _ = params[f"dec{l}.conv0"]
        w1, _ = params[f"dec{l}.conv1"]
        wu, _ = params[f"dec{l}.up"]
        da1 = g * (cache[f"dec{l}.a1"] > 0)
        da0, dw1, db1 = conv2d_backward(cache[f"dec{l}.a0"], w1, da1)
        da0 = da0 * (cache[f"dec{l}.a0"] > 0)
        dcat, dw0, db0 = conv2d_backward(cache[f"dec{l}.cat"], w0, da0)
        cu = wu.shape[1]
        dup, dskip[l] = dcat[:, :cu], dcat[:, cu:]
        g, dwu, dbu = conv_transpose2_backward(cache[f"dec{l}.in"], wu, dup)
        grads[f"dec{l}.up"], grads[f"dec{l}.conv0"], grads[f"dec{l}.conv1"] = (dwu, dbu), (dw0, db0), (dw1, db1)
    # g is now dL/d(output of the deepest encoder level)
    for l in reversed(range(levels)):
        w0, _ = params[f"enc{l}.conv0"]
        w1, _ = params[f"enc{l}.conv1"]
        a1 = cache[f"enc{l}.a1"]
        if l < levels - 1:
            g = maxpool2_backward(a1, g) + dskip[l]
        da1 = g * (a1 > 0)
        da0, dw1, db1 = conv2d_backward(cache[f"enc{l}.a0"], w1, da1)
        da0 = da0 * (cache[f"enc{l}.a0"] > 0)
        g, dw0, db0 = conv2d_backward(cache[f"enc{l}.in"], w0, da0)
        grads[f"enc{l}.conv0"], grads[f"enc{l}.conv1"] = (dw0, db0), (dw1, db1)
    return grads
