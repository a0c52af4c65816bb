"""ctypes binding of the paper's transmit parameterisation (include/sqngd_sqn.h)
and the driver of Algorithm 1 with it.

Argument marshalling only: the network, the staircase, the hard quantiser,
Adam, the threshold sort and the filter projection run in the library's
gfx950 kernels, the AF, the loss and the waveform / filter gradients in the
fused pass (sqngd_af_backward with the waveform given); torch provides device
memory and the current stream.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import inputs as I
from . import native as nat

SYMBOLS = ["sqngd_sqn_param_count", "sqngd_sqn_workspace_size", "sqngd_sqn_forward", "sqngd_sqn_soft",
           "sqngd_sqn_hard", "sqngd_sqn_backward", "sqngd_sqn_backward_adam", "sqngd_sqn_adam", "sqngd_sqn_adam_project", "sqngd_sqn_adam_sort",
           "sqngd_sqn_count", "sqngd_sqn_sort", "sqngd_sqn_project"]


class SqnShape(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int32), ("N", ctypes.c_int32), ("B", ctypes.c_int32), ("copies", ctypes.c_int32),
                ("c", ctypes.c_float), ("designs", ctypes.c_int32), ("reserved", ctypes.c_int32 * 2)]


_ready = False


def lib():
    global _ready
    L = nat.load()
    if not _ready:
        P, i32, i64, f, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_float, ctypes.c_size_t
        L.sqngd_sqn_param_count.argtypes = [i32, P]
        L.sqngd_sqn_workspace_size.argtypes = [P, P]
        L.sqngd_sqn_forward.argtypes = [P, P, P, P, P, sz, P]
        L.sqngd_sqn_soft.argtypes = [P, P, P, P, P]
        L.sqngd_sqn_hard.argtypes = [P, P, P, P, P, P]
        L.sqngd_sqn_backward.argtypes = [P, P, P, P, P, P, P, P, P, P, P, sz, P]
        L.sqngd_sqn_adam.argtypes = [P, P, P, P, i64, P, i32, i32, f, f, f, f, P]
        L.sqngd_sqn_backward_adam.argtypes = [P, P, P, P, P, P, P, P, P, P, P, P, i32, i32, f, f, f, f, P, sz, P]
        L.sqngd_sqn_adam_project.argtypes = [i32, i32, P, P, P, P, P, i32, i32, f, f, f, f, P]
        L.sqngd_sqn_adam_sort.argtypes = [P, P, P, P, i32, i32, P, i32, i32, f, f, f, f, P]
        L.sqngd_sqn_count.argtypes = [P, P]
        L.sqngd_sqn_sort.argtypes = [P, i32, i32, P]
        L.sqngd_sqn_project.argtypes = [i32, i32, P, P]
        for n in SYMBOLS:
            getattr(L, n).restype = ctypes.c_int
        _ready = True
    return L


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def adam(p, g, m, v, t: int, lr: float, beta1: float, beta2: float, eps: float, step=None, step_mul: int = 0):
    """Adam with step count t, or step_mul * step[0] + t with a device counter."""
    nat.check(lib().sqngd_sqn_adam(_ptr(p), _ptr(g), _ptr(m), _ptr(v), p.numel(), _ptr(step), int(step_mul), int(t),
                                   float(lr), float(beta1), float(beta2), float(eps), _stream()), "sqn_adam")


def adam_project(h, g, m, v, rows: int, N: int, t: int, lr: float, beta1: float, beta2: float, eps: float,
                 step=None, step_mul: int = 0):
    """Adam on filter rows then their energy projection (one launch)."""
    nat.check(lib().sqngd_sqn_adam_project(int(rows), int(N), _ptr(h), _ptr(g), _ptr(m), _ptr(v), _ptr(step),
                                           int(step_mul), int(t), float(lr), float(beta1), float(beta2), float(eps),
                                           _stream()), "sqn_adam_project")


def adam_sort(rho, g, m, v, K: int, designs: int, t: int, lr: float, beta1: float, beta2: float, eps: float,
              step=None, step_mul: int = 0):
    """Adam on each design's thresholds then their sort (one launch)."""
    nat.check(lib().sqngd_sqn_adam_sort(_ptr(rho), _ptr(g), _ptr(m), _ptr(v), int(K), int(designs), _ptr(step),
                                        int(step_mul), int(t), float(lr), float(beta1), float(beta2), float(eps),
                                        _stream()), "sqn_adam_sort")


class SQN:
    """The transmit network and staircase of R stacked designs of one shape on
    the GPU (shape, workspace); every per-design array is [R][...]."""

    def __init__(self, M: int, N: int, B: int, copies: int, c: float, device="cuda", designs: int = 1):
        self.M, self.N, self.B, self.copies, self.c = M, N, B, copies, float(c)
        self.R = int(designs)
        self.D, self.K = M * N, B * copies
        self.shape = SqnShape(M, N, B, copies, float(c), self.R, (ctypes.c_int32 * 2)(0, 0))
        n = ctypes.c_int64()
        nat.check(lib().sqngd_sqn_param_count(self.D, ctypes.byref(n)), "sqn_param_count")
        self.count = n.value
        b = ctypes.c_size_t()
        nat.check(lib().sqngd_sqn_workspace_size(ctypes.byref(self.shape), ctypes.byref(b)), "sqn_workspace_size")
        self.ws = torch.empty(b.value + 256, dtype=torch.uint8, device=device)
        off = (-self.ws.data_ptr()) % 256
        self.ws_view = self.ws[off: off + b.value]
        self.device = torch.device(device)

    def forward(self, theta, y0, z=None):
        z = torch.empty(self.R * self.D, dtype=torch.float32, device=self.device) if z is None else z
        nat.check(lib().sqngd_sqn_forward(ctypes.byref(self.shape), _ptr(theta), _ptr(y0), _ptr(z), _ptr(self.ws_view),
                                          self.ws_view.numel(), _stream()), "sqn_forward")
        return z

    def soft(self, z, rho, s=None):
        s = torch.empty(self.R * self.D, dtype=torch.complex64, device=self.device) if s is None else s
        nat.check(lib().sqngd_sqn_soft(ctypes.byref(self.shape), _ptr(z), _ptr(rho), _ptr(s), _stream()), "sqn_soft")
        return s

    def hard(self, z, rho, want_idx=True, want_x=True):
        idx = torch.empty(self.R * self.D, dtype=torch.int32, device=self.device) if want_idx else None
        x = torch.empty(self.R * self.D, dtype=torch.complex64, device=self.device) if want_x else None
        nat.check(lib().sqngd_sqn_hard(ctypes.byref(self.shape), _ptr(z), _ptr(rho), _ptr(idx), _ptr(x), _stream()),
                  "sqn_hard")
        return idx, x

    def backward(self, theta, y0, z, rho, s, grad_s, grad_h=None):
        """grad_h (optional): the filter gradient of the same evaluation when the
        filters are the soft waveform itself (matched filtering); it adds to grad_s."""
        gt = torch.empty(self.R * self.count, dtype=torch.float32, device=self.device)
        gr = torch.empty(self.R * self.K, dtype=torch.float32, device=self.device)
        nat.check(lib().sqngd_sqn_backward(ctypes.byref(self.shape), _ptr(theta), _ptr(y0), _ptr(z), _ptr(rho),
                                           _ptr(s), _ptr(grad_s), _ptr(grad_h), _ptr(gt), _ptr(gr),
                                           _ptr(self.ws_view),
                                           self.ws_view.numel(), _stream()), "sqn_backward")
        return gt, gr

    def backward_adam(self, theta, y0, z, rho, s, grad_s, m, v, t: int, lr: float, beta1: float, beta2: float,
                      eps: float, grad_h=None, step=None, step_mul: int = 0):
        """backward, then Adam on theta in place (the gradient is not stored);
        returns the threshold gradient."""
        gr = torch.empty(self.R * self.K, dtype=torch.float32, device=self.device)
        nat.check(lib().sqngd_sqn_backward_adam(ctypes.byref(self.shape), _ptr(theta), _ptr(y0), _ptr(z), _ptr(rho),
                                                _ptr(s), _ptr(grad_s), _ptr(grad_h), _ptr(m), _ptr(v), _ptr(gr),
                                                _ptr(step), int(step_mul), int(t), float(lr), float(beta1),
                                                float(beta2), float(eps), _ptr(self.ws_view), self.ws_view.numel(),
                                                _stream()), "sqn_backward_adam")
        return gr

    def sort(self, rho):
        nat.check(lib().sqngd_sqn_sort(_ptr(rho), self.K, self.R, _stream()), "sqn_sort")

    def project(self, h):
        nat.check(lib().sqngd_sqn_project(self.M * self.R, self.N, _ptr(h), _stream()), "sqn_project")


class SQNDesign:
    """Algorithm 1 with the paper's transmit side for one design: the ResNet
    parameters theta and thresholds rho (step B, Adam with lr_z, thresholds
    sorted after each update) and the filters h (step A, Adam with lr_h and
    the energy projection), from the fixed network input y0 = vec(Y0) of
    random discrete normalised phases. The filters start as the matched filter
    of X0 = exp(j 2 pi Y0) (h0 = x0), projected.

    matched=True is the AF extension of SQN the paper compares against
    (Sec. IV): no receive-filter optimisation, the filters are the waveform
    itself (the soft one in step B, whose loss then depends on it through
    both roles, the hard one when evaluated); step A is skipped.

    seed may be a list: R independent designs (random restarts) of the same
    problem run stacked -- one sqngd batch of R problems for the AF and one
    stacked transmit network -- each from its own seed (theta, y0); explicit
    theta, rho, y0, h are then the stacked [R][...] arrays."""

    def __init__(self, prob: dict, opt: dict, copies: int, c: float, seed=0, theta=None, rho=None,
                 y0=None, h=None, device="cuda", matched: bool = False):
        self.prob, self.opt = dict(prob), dict(opt)
        self.matched = bool(matched)
        seeds = [int(x) for x in seed] if isinstance(seed, (list, tuple)) else [int(seed)]
        self.R = R = len(seeds)
        M, N, B = prob["M"], prob["N"], prob["L"]
        self.sqn = SQN(M, N, B, copies, c, device, designs=R)
        self.batch = nat.Batch([dict(prob, schedule=prob.get("schedule", nat.SCHED_AUTO))] * R, device=device)
        dev = self.sqn.device
        f32 = lambda a: torch.as_tensor(np.asarray(a, np.float32)).to(dev).reshape(-1).contiguous()
        self.theta = f32(np.concatenate([I.sqn_init(M * N, sd) for sd in seeds]) if theta is None else theta)
        self.rho = f32(np.tile(I.sqn_thresholds(B, copies), R) if rho is None else rho)
        self.y0 = f32(np.concatenate([I.sqn_input(M, N, B, sd + 1) for sd in seeds]) if y0 is None else y0)
        self.z = self.sqn.forward(self.theta, self.y0)
        if h is None:
            # Algorithm 1's start: X0 = exp(j 2 pi Y0) from the same discrete
            # phases as the network input, the filters its matched filter
            # (h0 = x0, so that h^H x0 = N), then the energy projection
            y = self.y0.double()
            self.h = torch.polar(torch.ones_like(y), 2.0 * np.pi * y).to(torch.complex64).contiguous()
            self.sqn.project(self.h)
        else:
            self.h = torch.as_tensor(np.asarray(h, np.complex64)).to(dev).reshape(-1).contiguous()
        zeros = lambda n: torch.zeros(n, dtype=torch.float32, device=dev)
        self.mt, self.vt = zeros(R * self.sqn.count), zeros(R * self.sqn.count)
        self.mr, self.vr = zeros(R * self.sqn.K), zeros(R * self.sqn.K)
        self.mh, self.vh = zeros(2 * R * M * N), zeros(2 * R * M * N)
        self.counter = torch.zeros(1, dtype=torch.int32, device=dev)  # outer iterations done
        self.stats_a = self.batch.new_stats()
        self.stats_b = self.batch.new_stats()
        self.graph = None

    @property
    def t(self) -> int:
        return int(self.counter.item())

    def iteration(self):
        """Enqueue one outer iteration (Adam step counts from the device counter)."""
        o = self.opt
        b1, b2, eps = o["beta1"], o["beta2"], o["eps"]
        nh, nx = int(o["n_h"]), int(o["n_x"])
        self.z = self.sqn.forward(self.theta, self.y0, self.z)
        _, x = self.sqn.hard(self.z, self.rho, want_idx=False)
        for i in range(0 if self.matched else int(o["n_h"])):
            _, gh, _ = self.batch.af_backward(None, self.h, nat.WAVE_GIVEN, s_given=x, want_z=False, want_h=True,
                                              stats=self.stats_a)
            adam_project(self.h, gh, self.mh, self.vh, self.R * self.prob["M"], self.prob["N"], i + 1, o["lr_h"],
                         b1, b2, eps, step=self.counter, step_mul=nh)
        for j in range(int(o["n_x"])):
            self.z = self.sqn.forward(self.theta, self.y0, self.z)
            s = self.sqn.soft(self.z, self.rho)
            _, gh, gs = self.batch.af_backward(None, s if self.matched else self.h, nat.WAVE_GIVEN, s_given=s,
                                               want_z=False, want_h=self.matched, want_s=True, stats=self.stats_b)
            gr = self.sqn.backward_adam(self.theta, self.y0, self.z, self.rho, s, gs, self.mt, self.vt, j + 1,
                                        o["lr_z"], b1, b2, eps, grad_h=gh, step=self.counter, step_mul=nx)
            adam_sort(self.rho, gr, self.mr, self.vr, self.sqn.K, self.R, j + 1, o["lr_z"], b1, b2, eps,
                      step=self.counter, step_mul=nx)
        nat.check(lib().sqngd_sqn_count(_ptr(self.counter), _stream()), "sqn_count")

    def capture(self):
        """Record one outer iteration in a HIP graph; run() replays it."""
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.iteration()
        self.graph = g
        return g

    def run(self, iters: int, use_graph: bool = True):
        if not use_graph:
            for _ in range(iters):
                self.iteration()
            return
        if self.graph is None:
            self.capture()
        for _ in range(iters):
            self.graph.replay()

    def hard_stats(self):
        z = self.sqn.forward(self.theta, self.y0)
        _, x = self.sqn.hard(z, self.rho, want_idx=False)
        h = x if self.matched else self.h
        st = nat.decode_stats(self.batch.af_forward(None, h, nat.WAVE_GIVEN, s_given=x).cpu().numpy())
        return st[0] if self.R == 1 else st

    def hard_indices(self):
        z = self.sqn.forward(self.theta, self.y0)
        idx, _ = self.sqn.hard(z, self.rho, want_x=False)
        shape = (self.prob["M"], self.prob["N"]) if self.R == 1 else (self.R, self.prob["M"], self.prob["N"])
        return idx.cpu().numpy().reshape(shape)
