"""ctypes binding of the learned-initialisation network (include/unet.h).

Argument marshalling only: convolutions, pooling, loss, gradients and Adam run
in the HIP kernels behind the C ABI.  Weights are exchanged in the usual
(Cout, Cin, kh, kw) / (Cin, Cout, 2, 2) shapes and laid out here into the
library's GEMM matrices; images are exchanged NCHW and laid out NHWC.
"""
from __future__ import annotations

import ctypes as C
from typing import Dict, List, Tuple

import numpy as np

from . import abi
from .abi import _indexed

UN_CONV3X3, UN_UPCONV2X2, UN_CONV1X1 = 0, 1, 2

SYMBOLS = ("un_workspace_size", "un_net_create", "un_net_destroy", "un_layer_count", "un_layer_info", "un_params",
           "un_sync_weights", "un_forward", "un_backward", "un_adam_step", "un_activation", "un_last_error")


class UnConfig(C.Structure):
    _fields_ = [("in_ch", C.c_int32), ("out_ch", C.c_int32), ("base", C.c_int32), ("levels", C.c_int32),
                ("height", C.c_int32), ("width", C.c_int32), ("max_batch", C.c_int32)]


class UnLayer(C.Structure):
    _fields_ = [("kind", C.c_int32), ("cin", C.c_int32), ("cout", C.c_int32), ("taps", C.c_int32),
                ("n_rows", C.c_int32), ("kpad", C.c_int32), ("w_offset", C.c_int64), ("b_offset", C.c_int64)]


_bound = False


def lib():
    global _bound
    L = abi.lib()
    if not _bound:
        P, I32, I64 = C.c_void_p, C.c_int32, C.c_int64
        L.un_workspace_size.restype = I32
        L.un_workspace_size.argtypes = [C.POINTER(UnConfig), C.POINTER(C.c_size_t)]
        L.un_net_create.restype = I32
        L.un_net_create.argtypes = [C.POINTER(UnConfig), P, C.c_size_t, C.POINTER(P)]
        L.un_net_destroy.restype = None
        L.un_net_destroy.argtypes = [P]
        L.un_layer_count.restype = I32
        L.un_layer_count.argtypes = [P]
        L.un_layer_info.restype = I32
        L.un_layer_info.argtypes = [P, I32, C.POINTER(UnLayer)]
        L.un_params.restype = I32
        L.un_params.argtypes = [P, C.POINTER(P), C.POINTER(P), C.POINTER(I64)]
        L.un_sync_weights.restype = I32
        L.un_sync_weights.argtypes = [P, P]
        L.un_forward.restype = I32
        L.un_forward.argtypes = [P, P, I32, P, P]
        L.un_backward.restype = I32
        L.un_backward.argtypes = [P, P, I32, P, P, P, P]
        L.un_adam_step.restype = I32
        L.un_adam_step.argtypes = [P, P, C.c_float, C.c_float, C.c_float, C.c_float]
        L.un_activation.restype = I32
        L.un_activation.argtypes = [P, I32, C.POINTER(P), C.POINTER(I32), C.POINTER(I32), C.POINTER(I32)]
        L.un_last_error.restype = C.c_char_p
        L.un_last_error.argtypes = []
        _bound = True
    return L


def _check(status: int, what: str):
    if status != 0:
        raise abi.MsError(status, what, lib().un_last_error().decode())


def layer_names(levels: int) -> List[str]:
    """Parameter order of the library: encoder levels, decoder levels deepest first, head."""
    names = []
    for l in range(levels):
        names += [f"enc{l}.conv0", f"enc{l}.conv1"]
    for l in reversed(range(levels - 1)):
        names += [f"dec{l}.up", f"dec{l}.conv0", f"dec{l}.conv1"]
    return names + ["head"]


def workspace_size(cfg: UnConfig) -> int:
    out = C.c_size_t(0)
    _check(lib().un_workspace_size(C.byref(cfg), C.byref(out)), "un_workspace_size")
    return out.value


def to_nhwc_bf16(x, in_pad: int):
    """(B, C, H, W) float tensor -> (B, H, W, in_pad) bfloat16, zero pad channels."""
    import torch
    b, c, h, w = x.shape
    out = torch.zeros((b, h, w, in_pad), dtype=torch.bfloat16, device=x.device)
    out[..., :c] = x.permute(0, 2, 3, 1).to(torch.bfloat16)
    return out


class UNet:
    """The network on one device, in a workspace tensor it owns.  Calls enqueue on torch's
    current stream of that device."""

    def __init__(self, in_ch: int, out_ch: int, base: int = 32, levels: int = 4, height: int = 256,
                 width: int = 256, max_batch: int = 8, device=None):
        import torch
        self.device = _indexed(torch.device(device if device is not None else "cuda"))
        self.cfg = UnConfig(in_ch, out_ch, base, levels, height, width, max_batch)
        self.in_pad = (in_ch + 7) // 8 * 8
        ws = workspace_size(self.cfg)
        self._ws = torch.empty(ws, dtype=torch.uint8, device=self.device)
        h = C.c_void_p()
        _check(lib().un_net_create(C.byref(self.cfg), self._ws.data_ptr(), ws, C.byref(h)), "un_net_create")
        self._h = h
        self.names = layer_names(levels)
        self.layers: Dict[str, UnLayer] = {}
        for i, name in enumerate(self.names):
            li = UnLayer()
            _check(lib().un_layer_info(h, i, C.byref(li)), "un_layer_info")
            self.layers[name] = li
        pp, gp, cnt = C.c_void_p(), C.c_void_p(), C.c_int64()
        _check(lib().un_params(h, C.byref(pp), C.byref(gp), C.byref(cnt)), "un_params")
        base_ptr = self._ws.data_ptr()
        self.n_params = cnt.value
        self.params = self._ws[pp.value - base_ptr: pp.value - base_ptr + 4 * cnt.value].view(torch.float32)
        self.grads = self._ws[gp.value - base_ptr: gp.value - base_ptr + 4 * cnt.value].view(torch.float32)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().un_net_destroy(h)
            self._h = None

    def _stream(self):
        import torch
        return torch.cuda.current_stream(self.device).cuda_stream

    # -- parameters -------------------------------------------------------------------------
    def _to_matrix(self, li: UnLayer, w: np.ndarray) -> np.ndarray:
        m = np.zeros((li.n_rows, li.kpad), dtype=np.float32)
        if li.kind == UN_UPCONV2X2:                    # (Cin, Cout, 2, 2) -> [(2u+v) Cout + co][ci]
            cin, cout = w.shape[0], w.shape[1]
            m[:, :cin] = np.transpose(w, (2, 3, 1, 0)).reshape(4 * cout, cin)
        else:                                          # (Cout, Cin, k, k) -> [co][(k u + v) cin_pad + ci]
            cout, cin, k, _ = w.shape
            blk = np.zeros((cout, k * k, li.cin), dtype=np.float32)
            blk[:, :, :cin] = np.transpose(w, (0, 2, 3, 1)).reshape(cout, k * k, cin)
            m[:, :k * k * li.cin] = blk.reshape(cout, -1)
        return m

    def _from_matrix(self, li: UnLayer, m: np.ndarray, shape) -> np.ndarray:
        if li.kind == UN_UPCONV2X2:
            cin, cout = shape[0], shape[1]
            return np.transpose(m[:, :cin].reshape(2, 2, cout, cin), (3, 2, 0, 1))
        cout, cin, k, _ = shape
        blk = m[:, :k * k * li.cin].reshape(cout, k, k, li.cin)[..., :cin]
        return np.transpose(blk, (0, 3, 1, 2))

    def set_params(self, params: Dict[str, Tuple[np.ndarray, np.ndarray]]):
        """Writes weights {name: (W, b)} and makes the bf16 copies; clears the Adam state."""
        import torch
        flat = np.zeros(self.n_params, dtype=np.float32)
        for name, li in self.layers.items():
            w, b = params[name]
            m = self._to_matrix(li, np.asarray(w, dtype=np.float32))
            flat[li.w_offset: li.w_offset + m.size] = m.reshape(-1)
            flat[li.b_offset: li.b_offset + li.cout] = np.asarray(b, dtype=np.float32)
        self.params.copy_(torch.from_numpy(flat))
        _check(lib().un_sync_weights(self._h, self._stream()), "un_sync_weights")

    def shapes(self) -> Dict[str, tuple]:
        """Weight shapes {name: (Cout, Cin, k, k) or (Cin, Cout, 2, 2)} with the real input channels."""
        out = {}
        for name, li in self.layers.items():
            cin = self.cfg.in_ch if name == "enc0.conv0" else li.cin
            if li.kind == UN_UPCONV2X2:
                out[name] = (cin, li.cout, 2, 2)
            else:
                k = 3 if li.kind == UN_CONV3X3 else 1
                out[name] = (li.cout, cin, k, k)
        return out

    def init_he(self, seed: int):
        """He-normal weights (standard deviation sqrt(2 / fan_in)) and zero biases."""
        rng = np.random.Generator(np.random.PCG64(seed))
        params = {}
        for name, shp in self.shapes().items():
            fan_in = shp[0] * shp[2] * shp[3] if self.layers[name].kind == UN_UPCONV2X2 else shp[1] * shp[2] * shp[3]
            params[name] = (rng.standard_normal(shp) * np.sqrt(2.0 / fan_in), np.zeros(shp[1] if
                            self.layers[name].kind == UN_UPCONV2X2 else shp[0]))
        self.set_params(params)

    def flops_per_sample(self) -> float:
        """Forward multiply-adds x 2 of one image (real channels, no padding); the training step
        (forward, data and weight gradients) is about three times this."""
        total = 0.0
        h, w = self.cfg.height, self.cfg.width
        for name, shp in self.shapes().items():
            level = int(name[3]) if name.startswith(("enc", "dec")) else 0
            px = (h >> level) * (w >> level)
            if self.layers[name].kind == UN_UPCONV2X2:
                total += 2.0 * px * shp[0] * shp[1]          # every output pixel: Cin x Cout
            else:
                total += 2.0 * px * shp[0] * shp[1] * shp[2] * shp[3]
        return total

    def _unflatten(self, flat: np.ndarray, shapes) -> Dict[str, Tuple[np.ndarray, np.ndarray]]:
        out = {}
        for name, li in self.layers.items():
            m = flat[li.w_offset: li.w_offset + li.n_rows * li.kpad].reshape(li.n_rows, li.kpad)
            out[name] = (self._from_matrix(li, m, shapes[name]), flat[li.b_offset: li.b_offset + li.cout].copy())
        return out

    def get_params(self, shapes):
        return self._unflatten(self.params.cpu().numpy(), shapes)

    def get_grads(self, shapes):
        return self._unflatten(self.grads.cpu().numpy(), shapes)

    # -- compute ----------------------------------------------------------------------------
    def forward(self, x_nhwc, out=None):
        """x: (B, H, W, in_pad) bfloat16 on the device -> (B, H, W, out_ch) float32."""
        import torch
        b = x_nhwc.shape[0]
        self._expect(x_nhwc, torch.bfloat16, (b, self.cfg.height, self.cfg.width, self.in_pad))
        y = out if out is not None else torch.empty((b, self.cfg.height, self.cfg.width, self.cfg.out_ch),
                                                   dtype=torch.float32, device=self.device)
        _check(lib().un_forward(self._h, self._stream(), b, x_nhwc.data_ptr(), y.data_ptr()), "un_forward")
        return y

    def backward(self, x_nhwc, target_nhwc, out=None, loss=None):
        """Forward, centred MSE against the target and parameter gradients (into self.grads).
        Returns (y, loss) with loss a one-element float64 device tensor."""
        import torch
        b = x_nhwc.shape[0]
        self._expect(x_nhwc, torch.bfloat16, (b, self.cfg.height, self.cfg.width, self.in_pad))
        self._expect(target_nhwc, torch.float32, (b, self.cfg.height, self.cfg.width, self.cfg.out_ch))
        y = out if out is not None else torch.empty_like(target_nhwc)
        loss = loss if loss is not None else torch.zeros(1, dtype=torch.float64, device=self.device)
        _check(lib().un_backward(self._h, self._stream(), b, x_nhwc.data_ptr(), target_nhwc.data_ptr(),
                                 y.data_ptr(), loss.data_ptr()), "un_backward")
        return y, loss

    def adam_step(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        _check(lib().un_adam_step(self._h, self._stream(), lr, beta1, beta2, eps), "un_adam_step")

    def activation(self, index: int):
        """(B, h, w, c) bfloat16 view of activation `index` of the last forward pass."""
        import torch
        p, hh, ww, cc = C.c_void_p(), C.c_int32(), C.c_int32(), C.c_int32()
        _check(lib().un_activation(self._h, index, C.byref(p), C.byref(hh), C.byref(ww), C.byref(cc)),
               "un_activation")
        off = p.value - self._ws.data_ptr()
        n = self.cfg.max_batch * hh.value * ww.value * cc.value
        return self._ws[off: off + 2 * n].view(torch.bfloat16).view(self.cfg.max_batch, hh.value, ww.value,
                                                                    cc.value)

    def _expect(self, t, dtype, shape):
        if t.device != self.device or t.dtype != dtype or tuple(t.shape) != tuple(shape) or not t.is_contiguous():
            raise ValueError(f"expected a contiguous {dtype} tensor of shape {tuple(shape)} on {self.device}, "
                             f"got {t.dtype} {tuple(t.shape)} on {t.device}")
        if shape[0] > self.cfg.max_batch:
            raise ValueError(f"batch {shape[0]} exceeds max_batch {self.cfg.max_batch}")
