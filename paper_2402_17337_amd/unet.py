"""Thin ctypes binding of the warm-start network (``include/ibm_unet.h``).

Argument marshalling only: the network's forward and backward passes, loss and
Adam update run in the HIP kernels of ``libibm_hip.so``.  PyTorch provides the
device workspace, the tensors handed across and the HIP stream.  There is no
CPU fallback.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import ibm

CONV_FORWARD, CONV_DGRAD, CONV_WGRAD = 0, 1, 2
IN_CHANNELS = 3
LAYERS = [  # (name, in, out, ReLU after), the order of the parameter vector
    ("enc0a", 3, 16, True), ("enc0b", 16, 16, True), ("enc1a", 16, 32, True), ("enc1b", 32, 32, True),
    ("enc2a", 32, 64, True), ("enc2b", 64, 64, True), ("mid_a", 64, 128, True), ("mid_b", 128, 128, True),
    ("dec2a", 192, 64, True), ("dec2b", 64, 64, True), ("dec1a", 96, 32, True), ("dec1b", 32, 32, True),
    ("dec0a", 48, 16, True), ("dec0b", 16, 16, True), ("out", 16, 1, False),
]

EXPORTED = ("ibm_unet_param_count", "ibm_unet_workspace_bytes", "ibm_unet_create", "ibm_unet_set_params",
            "ibm_unet_get_params", "ibm_unet_get_grads", "ibm_unet_forward", "ibm_unet_loss_grad",
            "ibm_unet_adam_step", "ibm_unet_train_step", "ibm_unet_destroy", "ibm_unet_last_error",
            "ibm_unet_conv_workspace_bytes", "ibm_unet_conv3x3")

_bound = False


def lib():
    """The solver library with the network's entry points typed."""
    global _bound
    L = ibm.lib()
    if not _bound:
        vp, fp, i32, sz = C.c_void_p, C.POINTER(C.c_float), C.c_int32, C.c_size_t
        L.ibm_unet_param_count.argtypes = []
        L.ibm_unet_param_count.restype = sz
        L.ibm_unet_workspace_bytes.argtypes = [i32, i32, i32]
        L.ibm_unet_workspace_bytes.restype = sz
        L.ibm_unet_create.argtypes = [i32, i32, i32, vp, sz, vp, C.POINTER(vp)]
        L.ibm_unet_create.restype = i32
        for f in ("ibm_unet_set_params", "ibm_unet_get_params", "ibm_unet_get_grads"):
            getattr(L, f).argtypes = [vp, fp, sz]
            getattr(L, f).restype = i32
        L.ibm_unet_forward.argtypes = [vp, vp, vp, i32]
        L.ibm_unet_forward.restype = i32
        L.ibm_unet_loss_grad.argtypes = [vp, vp, vp, vp, i32, fp]
        L.ibm_unet_loss_grad.restype = i32
        L.ibm_unet_adam_step.argtypes = [vp, C.c_float, C.c_float, C.c_float, C.c_float]
        L.ibm_unet_adam_step.restype = i32
        L.ibm_unet_train_step.argtypes = [vp, vp, vp, vp, i32, C.c_float, fp]
        L.ibm_unet_train_step.restype = i32
        L.ibm_unet_destroy.argtypes = [vp]
        L.ibm_unet_destroy.restype = None
        L.ibm_unet_last_error.argtypes = [vp]
        L.ibm_unet_last_error.restype = C.c_char_p
        L.ibm_unet_conv_workspace_bytes.argtypes = [i32, i32, i32, i32, i32]
        L.ibm_unet_conv_workspace_bytes.restype = sz
        L.ibm_unet_conv3x3.argtypes = [i32, i32, i32, i32, i32, i32, vp, vp, vp, vp, vp, vp, sz, vp]
        L.ibm_unet_conv3x3.restype = i32
        _bound = True
    return L


def param_count() -> int:
    return int(lib().ibm_unet_param_count())


def forward_flops(batch: int, h: int, w: int) -> float:
    """Multiply-add FLOPs (2 per product) of the network's convolutions for
    one forward pass over batch images h x w (unpadded channel counts)."""
    lvl = {"enc0": 0, "enc1": 1, "enc2": 2, "mid_": 3, "dec2": 2, "dec1": 1, "dec0": 0, "out": 0}
    total = 0.0
    for name, ci, co, _ in LAYERS:
        l = lvl[name[:4] if name != "out" else "out"]
        total += 2.0 * 9 * ci * co * batch * (h >> l) * (w >> l)
    return total


def flatten_params(params: dict) -> np.ndarray:
    """Parameter dict {name.w: (co, ci, 3, 3), name.b: (co,)} -> float32 vector."""
    parts = []
    for name, ci, co, _ in LAYERS:
        parts.append(np.asarray(params[name + ".w"], dtype=np.float32).reshape(-1))
        parts.append(np.asarray(params[name + ".b"], dtype=np.float32).reshape(-1))
    return np.ascontiguousarray(np.concatenate(parts))


def unflatten_params(vec: np.ndarray) -> dict:
    out, k = {}, 0
    for name, ci, co, _ in LAYERS:
        n = co * ci * 9
        out[name + ".w"] = vec[k:k + n].reshape(co, ci, 3, 3)
        k += n
        out[name + ".b"] = vec[k:k + co]
        k += co
    return out


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _check_f32_cuda(t, shape, what):
    import torch
    if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous() or tuple(t.shape) != tuple(shape):
        raise ValueError(f"{what}: expected a contiguous float32 device tensor of shape {shape}, "
                         f"got {t.dtype} {tuple(t.shape)} on {t.device}")


class UNet:
    """A warm-start network for batches of up to max_batch images h x w."""

    def __init__(self, max_batch: int, h: int, w: int, device="cuda:0", stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the network runs only on the HIP device")
        L = lib()
        self.torch = torch
        self.max_batch, self.h, self.w = max_batch, h, w
        self.device = torch.device(device)
        nbytes = L.ibm_unet_workspace_bytes(max_batch, h, w)
        if nbytes == 0:
            raise ValueError("invalid network shape (height % 8, width % 64)")
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        hnd = C.c_void_p()
        rc = L.ibm_unet_create(max_batch, h, w, _ptr(self.ws), nbytes, C.c_void_p(self.stream.cuda_stream),
                               C.byref(hnd))
        if rc != ibm.OK:
            raise ibm.IbmError(f"ibm_unet_create failed: {ibm.status_string(rc)}")
        self._h = hnd
        self.n = param_count()

    def close(self):
        h = getattr(self, "_h", None)
        if h:
            lib().ibm_unet_destroy(h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def _err(self, what, rc):
        raise ibm.IbmError(f"{what} failed: {ibm.status_string(rc)} {lib().ibm_unet_last_error(self._h).decode()}")

    def set_params(self, params):
        vec = flatten_params(params) if isinstance(params, dict) else np.ascontiguousarray(params, np.float32)
        rc = lib().ibm_unet_set_params(self._h, vec.ctypes.data_as(C.POINTER(C.c_float)), vec.size)
        if rc:
            self._err("ibm_unet_set_params", rc)

    def _get(self, fn):
        out = np.empty(self.n, dtype=np.float32)
        rc = getattr(lib(), fn)(self._h, out.ctypes.data_as(C.POINTER(C.c_float)), self.n)
        if rc:
            self._err(fn, rc)
        return out

    def get_params(self) -> np.ndarray:
        return self._get("ibm_unet_get_params")

    def get_grads(self) -> np.ndarray:
        return self._get("ibm_unet_get_grads")

    def forward(self, x, y=None):
        b = x.shape[0]
        _check_f32_cuda(x, (b, IN_CHANNELS, self.h, self.w), "x")
        if y is None:
            y = self.torch.empty((b, 1, self.h, self.w), dtype=self.torch.float32, device=self.device)
        _check_f32_cuda(y, (b, 1, self.h, self.w), "y")
        rc = lib().ibm_unet_forward(self._h, _ptr(x), _ptr(y), b)
        if rc:
            self._err("ibm_unet_forward", rc)
        return y

    def loss_grad(self, x, target, weight=None) -> float:
        b = x.shape[0]
        _check_f32_cuda(x, (b, IN_CHANNELS, self.h, self.w), "x")
        _check_f32_cuda(target, (b, 1, self.h, self.w), "target")
        if weight is not None:
            _check_f32_cuda(weight, (b,), "weight")
        loss = C.c_float()
        rc = lib().ibm_unet_loss_grad(self._h, _ptr(x), _ptr(target), _ptr(weight), b, C.byref(loss))
        if rc:
            self._err("ibm_unet_loss_grad", rc)
        return float(loss.value)

    def adam_step(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        rc = lib().ibm_unet_adam_step(self._h, lr, beta1, beta2, eps)
        if rc:
            self._err("ibm_unet_adam_step", rc)

    def train_step(self, x, target, lr, want_loss=True, weight=None):
        b = x.shape[0]
        _check_f32_cuda(x, (b, IN_CHANNELS, self.h, self.w), "x")
        _check_f32_cuda(target, (b, 1, self.h, self.w), "target")
        if weight is not None:
            _check_f32_cuda(weight, (b,), "weight")
        loss = C.c_float()
        rc = lib().ibm_unet_train_step(self._h, _ptr(x), _ptr(target), _ptr(weight), b, lr,
                                       C.byref(loss) if want_loss else None)
        if rc:
            self._err("ibm_unet_train_step", rc)
        return float(loss.value) if want_loss else None


def conv3x3(op, x=None, w=None, b=None, gy=None, n=None, h=None, wd=None, cin=None, cout=None, stream=None):
    """One network convolution layer through ibm_unet_conv3x3 (float32 device
    tensors; see the header for the operations)."""
    import torch
    L = lib()
    ref = x if x is not None else gy
    if n is None:
        n, h, wd = ref.shape[0], ref.shape[2], ref.shape[3]
        cout, cin = w.shape[0], w.shape[1]
    nbytes = L.ibm_unet_conv_workspace_bytes(n, h, wd, cin, cout)
    if nbytes == 0:
        raise ValueError("invalid convolution shape")
    ws = torch.empty(nbytes, dtype=torch.uint8, device=ref.device)
    if op == CONV_FORWARD:
        out = torch.empty((n, cout, h, wd), dtype=torch.float32, device=ref.device)
    elif op == CONV_DGRAD:
        out = torch.empty((n, cin, h, wd), dtype=torch.float32, device=ref.device)
    else:
        out = torch.empty(cout * cin * 9 + cout, dtype=torch.float32, device=ref.device)
    st = stream if stream is not None else torch.cuda.current_stream(ref.device)
    rc = L.ibm_unet_conv3x3(op, n, h, wd, cin, cout, _ptr(x), _ptr(w), _ptr(b), _ptr(gy), _ptr(out), _ptr(ws),
                            nbytes, C.c_void_p(st.cuda_stream))
    if rc:
        raise ibm.IbmError(f"ibm_unet_conv3x3 failed: {ibm.status_string(rc)}")
    torch.cuda.current_stream(ref.device).synchronize()
    return out
