"""ctypes binding of the warm-start network ABI (include/sqngd_net.h).

Argument marshalling only: every computation runs in the library's gfx950
kernels; torch provides device memory and the current stream.
"""
from __future__ import annotations

import ctypes

import torch

from . import inputs as I
from . import native as nat

SYMBOLS = ["sqngd_net_param_count", "sqngd_net_workspace_size", "sqngd_net_forward",
           "sqngd_net_backward", "sqngd_net_adam"]


class NetShape(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int32), ("N", ctypes.c_int32), ("L", ctypes.c_int32),
                ("batch", ctypes.c_int32), ("cond0", ctypes.c_float), ("cond1", ctypes.c_float),
                ("reserved", ctypes.c_int32 * 2)]


class NetOpt(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float),
                ("eps", ctypes.c_float)]


_ready = False


def lib():
    global _ready
    L = nat.load()
    if not _ready:
        P, i32 = ctypes.c_void_p, ctypes.c_int32
        L.sqngd_net_param_count.argtypes = [P, P]
        L.sqngd_net_workspace_size.argtypes = [P, P]
        L.sqngd_net_forward.argtypes = [P, P, P, P, P, ctypes.c_size_t, P]
        L.sqngd_net_backward.argtypes = [P, P, P, P, P, P, P, ctypes.c_size_t, P]
        L.sqngd_net_adam.argtypes = [P, P, i32, P, P, P, P]
        _ready = True
    return L


def shape(M: int, N: int, L: int, batch: int, cond=(1.0, 1.0)) -> NetShape:
    return NetShape(M, N, L, batch, float(cond[0]), float(cond[1]), (ctypes.c_int32 * 2)(0, 0))


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Net:
    """Workspace, parameters and Adam moments of one network shape on the GPU."""

    def __init__(self, M: int, N: int, L: int, batch: int, cond=(1.0, 1.0), params=None, seed: int = 0,
                 device="cuda"):
        self.M, self.N, self.L, self.batch = M, N, L, batch
        self.shape = shape(M, N, L, batch, cond)
        n = ctypes.c_int64()
        nat.check(lib().sqngd_net_param_count(ctypes.byref(self.shape), ctypes.byref(n)), "net_param_count")
        self.count = n.value
        b = ctypes.c_size_t()
        nat.check(lib().sqngd_net_workspace_size(ctypes.byref(self.shape), ctypes.byref(b)), "net_workspace_size")
        self.ws = torch.empty(b.value + 256, dtype=torch.uint8, device=device)
        off = (-self.ws.data_ptr()) % 256
        self.ws_view = self.ws[off: off + b.value]
        p = I.net_init(M, L, seed) if params is None else params
        self.params = torch.as_tensor(p, dtype=torch.float32).to(device).contiguous()
        assert self.params.numel() == self.count
        self.moments = torch.zeros(2 * self.count, dtype=torch.float32, device=device)
        self.grad = torch.zeros(self.count, dtype=torch.float32, device=device)
        self.loss = torch.zeros(1, dtype=torch.float32, device=device)
        self.logits = torch.empty((batch, M, N, L), dtype=torch.float32, device=device)
        self.steps = 0

    def forward(self, noise: torch.Tensor) -> torch.Tensor:
        noise = noise.contiguous()
        assert noise.shape == (self.batch, self.M, self.N) and noise.dtype == torch.float32
        nat.check(lib().sqngd_net_forward(ctypes.byref(self.shape), _ptr(self.params), _ptr(noise),
                                          _ptr(self.logits), _ptr(self.ws_view), self.ws_view.numel(),
                                          _stream()), "net_forward")
        return self.logits

    def backward(self, target: torch.Tensor | None = None, grad_logits: torch.Tensor | None = None):
        """Gradient into self.grad (and the loss into self.loss with a target)."""
        nat.check(lib().sqngd_net_backward(ctypes.byref(self.shape), _ptr(self.logits),
                                           _ptr(None if target is None else target.contiguous()),
                                           _ptr(None if grad_logits is None else grad_logits.contiguous()),
                                           _ptr(self.grad), _ptr(self.loss), _ptr(self.ws_view),
                                           self.ws_view.numel(), _stream()), "net_backward")
        return self.grad

    def adam(self, lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
        self.steps += 1
        o = NetOpt(lr, beta1, beta2, eps)
        nat.check(lib().sqngd_net_adam(ctypes.byref(self.shape), ctypes.byref(o), self.steps, _ptr(self.params),
                                       _ptr(self.moments), _ptr(self.grad), _stream()), "net_adam")

    def train_step(self, noise, target, lr: float = 1e-3):
        self.forward(noise)
        self.backward(target=target)
        self.adam(lr)
        return self.loss
