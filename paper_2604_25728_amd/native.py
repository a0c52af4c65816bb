"""ctypes binding of libsqngd.so (C ABI in include/sqngd.h).

Argument marshalling only: every step of the hot path runs in the library's
HIP kernels. PyTorch provides device memory and the current stream. Loading
fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsqngd.so")

OK = 0
WAVE_SOFT, WAVE_HARD, WAVE_GIVEN = 0, 1, 2
SQ_PHASE_MEAN, SQ_PHASOR_MEAN = 0, 1
OPT_SGD = 1
SCHED_AUTO, SCHED_THROUGHPUT, SCHED_SPLIT2, SCHED_SPLIT4, SCHED_SPLIT8, SCHED_SPLIT12, SCHED_SPLIT16 = 0, 1, 2, 4, 8, 12, 16
SCHED_GROUPED, SCHED_FUSED, SCHED_PAIR = 32, 33, 40

SYMBOLS = [
    "sqngd_buffer_sizes", "sqngd_workspace_size", "sqngd_workspace_init", "sqngd_af_forward",
    "sqngd_af_backward", "sqngd_step", "sqngd_run", "sqngd_hard_quantize", "sqngd_status_string",
    "sqngd_last_hip_error", "sqngd_profile_enable", "sqngd_profile_read", "sqngd_set_roi_weights",
    "sqngd_af_backward_noalloc", "sqngd_workspace_release", "sqngd_set_stop_mask", "sqngd_stop_update",
    "sqngd_profile_groups",
]
E_SCRATCH = -6
MASK_TAU0 = 0      # eq. 8: an auto pair's whole tau = 0 Doppler cut is outside the ROI
MASK_MAINLOBE = 1  # only the cut's mainlobe cells |nu_f| < 1 are outside it
NOALLOC_SCRATCH_BYTES = 32 << 20


class Problem(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int32), ("N", ctypes.c_int32), ("L", ctypes.c_int32),
                ("F", ctypes.c_int32), ("nu_min", ctypes.c_float), ("nu_max", ctypes.c_float),
                ("tau_lo", ctypes.c_int32), ("tau_hi", ctypes.c_int32), ("p", ctypes.c_float),
                ("snrl_target_db", ctypes.c_float), ("w_psl", ctypes.c_float),
                ("w_snrl", ctypes.c_float), ("temperature", ctypes.c_float),
                ("sq_mode", ctypes.c_int32), ("schedule", ctypes.c_int32), ("auto_mask", ctypes.c_int32)]


class Opt(ctypes.Structure):
    _fields_ = [("lr_z", ctypes.c_float), ("lr_h", ctypes.c_float), ("beta1", ctypes.c_float),
                ("beta2", ctypes.c_float), ("eps", ctypes.c_float), ("n_h", ctypes.c_int32),
                ("n_x", ctypes.c_int32), ("T0", ctypes.c_float), ("T1", ctypes.c_float),
                ("total_iters", ctypes.c_int32), ("flags", ctypes.c_int32)]


STATS_FIELDS = ["loss", "lp", "l_snrl", "psl_auto", "psl_cross", "pslr_db", "snrl_db_max", "p_min"]
STATS_WORDS = 16  # sqngd_stats is 64 bytes

assert ctypes.sizeof(Problem) == 64 and ctypes.sizeof(Opt) == 44


class SQNGDError(RuntimeError):
    pass


_lib = None


def load():
    """Load libsqngd.so (built in-tree by __graft_entry__.build())."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise SQNGDError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    lib = ctypes.CDLL(LIB_PATH)
    P, i32, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_size_t
    lib.sqngd_buffer_sizes.argtypes = [P, i32, P, P, P, P]
    lib.sqngd_workspace_size.argtypes = [P, i32, P]
    lib.sqngd_workspace_init.argtypes = [P, i32, P, sz, P]
    lib.sqngd_workspace_release.argtypes = [P]
    lib.sqngd_set_stop_mask.argtypes = [P, i32, P, P, sz]
    lib.sqngd_stop_update.argtypes = [i32, P, ctypes.c_float, i32, P, P, P, P, P, P]
    lib.sqngd_set_roi_weights.argtypes = [P, i32, P, P, sz]
    lib.sqngd_af_forward.argtypes = [P, i32, P, i32, P, P, P, P, P, sz, P]
    lib.sqngd_af_backward.argtypes = [P, i32, P, i32, P, P, P, P, P, P, P, P, sz, P]
    lib.sqngd_af_backward_noalloc.argtypes = [P, i32, P, i32, P, P, P, P, P, P, P, P]
    lib.sqngd_step.argtypes = [P, i32, P, P, P, P, P, P, P, sz, P]
    lib.sqngd_run.argtypes = [P, i32, P, i32, P, P, P, P, P, P, sz, P]
    lib.sqngd_hard_quantize.argtypes = [P, i32, P, P, P, P, sz, P]
    lib.sqngd_status_string.argtypes = [ctypes.c_int]
    lib.sqngd_status_string.restype = ctypes.c_char_p
    lib.sqngd_last_hip_error.argtypes = []
    lib.sqngd_profile_enable.argtypes = [i32, i32]
    lib.sqngd_profile_read.argtypes = [P, i32, P]
    lib.sqngd_profile_groups.argtypes = [P, i32, P]
    for name in SYMBOLS:
        if name not in ("sqngd_status_string",):
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def status_string(rc: int) -> str:
    return load().sqngd_status_string(int(rc)).decode()


def check(rc: int, what: str):
    if rc != OK:
        hip = load().sqngd_last_hip_error()
        raise SQNGDError(f"{what}: {status_string(rc)} (status {rc}, hip error {hip})")


def profile_enable(max_launches: int, repeat: int = 1):
    """Bracket the next max_launches fused-pass launches with HIP events (0: off),
    each issued `repeat` times back to back inside its bracket."""
    check(load().sqngd_profile_enable(int(max_launches), int(repeat)), "profile_enable")


def profile_read(capacity: int = 65536) -> np.ndarray:
    """Durations (ms) of the fused-pass launches recorded since profile_enable."""
    buf = (ctypes.c_float * capacity)()
    cnt = ctypes.c_int32()
    check(load().sqngd_profile_read(buf, capacity, ctypes.byref(cnt)), "profile_read")
    return np.array(buf[: min(cnt.value, capacity)], dtype=np.float64)


def profile_groups(capacity: int = 65536) -> np.ndarray:
    """FFT-length groups (bit g: length 128 << g) of each recorded launch."""
    buf = (ctypes.c_int32 * capacity)()
    cnt = ctypes.c_int32()
    check(load().sqngd_profile_groups(buf, capacity, ctypes.byref(cnt)), "profile_groups")
    return np.array(buf[: min(cnt.value, capacity)], dtype=np.int64)


def make_problems(probs) -> ctypes.Array:
    """ctypes array of sqngd_problem from problem dicts (see inputs.make_problem)."""
    arr = (Problem * len(probs))()
    for i, d in enumerate(probs):
        p = arr[i]
        for k in ("M", "N", "L", "F", "tau_lo", "tau_hi", "sq_mode"):
            setattr(p, k, int(d[k]))
        p.schedule = int(d.get("schedule", SCHED_AUTO))
        p.auto_mask = int(d.get("auto_mask", MASK_TAU0))
        for k in ("nu_min", "nu_max", "p", "snrl_target_db", "w_psl", "w_snrl", "temperature"):
            setattr(p, k, float(d[k]))
    return arr


def make_opt(d: dict) -> Opt:
    o = Opt()
    for k in ("lr_z", "lr_h", "beta1", "beta2", "eps", "T0", "T1"):
        setattr(o, k, float(d[k]))
    for k in ("n_h", "n_x", "total_iters", "flags"):
        setattr(o, k, int(d[k]))
    return o


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def decode_stats(words: np.ndarray) -> list[dict]:
    """sqngd_stats records (int32 [n][16]) as dicts."""
    words = np.ascontiguousarray(words, dtype=np.int32).reshape(-1, STATS_WORDS)
    f = words.view(np.float32)
    out = []
    for r in range(words.shape[0]):
        d = {k: float(f[r, i]) for i, k in enumerate(STATS_FIELDS)}
        d["arg"] = tuple(int(v) for v in words[r, 8:12])
        d["nonfinite"] = int(words[r, 12])
        out.append(d)
    return out


def af_backward_noalloc(probs, z, h, wave_mode=WAVE_SOFT, s_given=None, grad_loss=None, want_z=True,
                        want_h=True, want_s=False, stats=None, device="cuda"):
    """sqngd_af_backward_noalloc: the gradients of sqngd_af_backward for the
    packed batch `probs` without a workspace (the library's static scratch on
    the current GPU). Returns (grad_z, grad_h, grad_s), None where not wanted."""
    import torch
    lib = load()
    arr = make_problems(probs)
    zf, wc = ctypes.c_int64(), ctypes.c_int64()
    check(lib.sqngd_buffer_sizes(arr, len(probs), ctypes.byref(zf), ctypes.byref(wc), None, None), "buffer_sizes")
    gz = torch.empty(zf.value, dtype=torch.float32, device=device) if want_z else None
    gh = torch.empty(wc.value, dtype=torch.complex64, device=device) if want_h else None
    gs = torch.empty(wc.value, dtype=torch.complex64, device=device) if want_s else None
    check(lib.sqngd_af_backward_noalloc(arr, len(probs), _ptr(z), int(wave_mode), _ptr(s_given), _ptr(h),
                                        _ptr(grad_loss), _ptr(gz), _ptr(gh), _ptr(gs), _ptr(stats), _stream()),
          "af_backward_noalloc")
    return gz, gh, gs


class Batch:
    """A batch of design problems bound to one workspace on the current GPU.

    Buffers follow the packing of include/sqngd.h: every per-problem array is
    laid out back to back in problem order (flat tensors)."""

    def __init__(self, probs, device="cuda"):
        import torch
        self.lib = load()
        self.probs = [dict(p) for p in probs]
        self.n = len(self.probs)
        self._arr = make_problems(self.probs)
        zf, wc, af, cc = (ctypes.c_int64() for _ in range(4))
        check(self.lib.sqngd_buffer_sizes(self._arr, self.n, ctypes.byref(zf), ctypes.byref(wc),
                                          ctypes.byref(af), ctypes.byref(cc)), "buffer_sizes")
        self.z_floats, self.wave_c64, self.adam_floats, self.cube_c64 = (
            zf.value, wc.value, af.value, cc.value)
        nb = ctypes.c_size_t()
        check(self.lib.sqngd_workspace_size(self._arr, self.n, ctypes.byref(nb)), "workspace_size")
        self.ws_bytes = nb.value
        self.device = torch.device(device)
        self.ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
        off = (-self.ws.data_ptr()) % 256
        self._ws_ptr = ctypes.c_void_p(self.ws.data_ptr() + off)
        check(self.lib.sqngd_workspace_init(self._arr, self.n, self._ws_ptr, self.ws_bytes,
                                            _stream()), "workspace_init")
        self.roi_w = None
        # element offsets of each problem in the packed buffers
        self.off_z, self.off_w, self.off_cube, self.off_adam = [], [], [], []
        oz = ow = oc = oa = 0
        for p in self.probs:
            self.off_z.append(oz)
            self.off_w.append(ow)
            self.off_cube.append(oc)
            self.off_adam.append(oa)
            oz += p["M"] * p["N"] * p["L"]
            ow += p["M"] * p["N"]
            oc += p["M"] * p["M"] * p["F"] * (2 * p["N"] - 1)
            oa += 2 * p["M"] * p["N"] * p["L"] + 4 * p["M"] * p["N"]

    def __del__(self):
        # drop the library's plan for this workspace before its memory goes back to the allocator
        try:
            self.lib.sqngd_workspace_release(self._ws_ptr)
        except Exception:
            pass

    def set_roi_weights(self, ws=None):
        """Attach the ROI weights w(tau, f) of eq. 8-9: a list of [F][2N-1]
        arrays (one per problem, None entries meaning w = 1) or None for w = 1
        everywhere. The packed device copy is kept by the batch."""
        import torch
        if ws is None or all(w is None for w in ws):
            self.roi_w = None
        else:
            parts = []
            for p, w in zip(self.probs, ws):
                shape = (p["F"], 2 * p["N"] - 1)
                w = np.ones(shape, np.float32) if w is None else np.asarray(w, np.float32)
                if w.shape != shape:
                    raise ValueError(f"ROI weights of shape {w.shape}, expected {shape}")
                parts.append(torch.as_tensor(w).reshape(-1))
            self.roi_w = torch.cat(parts).to(self.device)
        check(self.lib.sqngd_set_roi_weights(self._arr, self.n, _ptr(self.roi_w), self._ws_ptr, self.ws_bytes),
              "set_roi_weights")

    def set_stop_mask(self, stopped=None):
        """Attach a device int32 [n] stop mask (None detaches): later optimiser
        steps keep the parameters of problems whose entry is nonzero."""
        self.stop_mask = stopped
        check(self.lib.sqngd_set_stop_mask(self._arr, self.n, _ptr(stopped), self._ws_ptr, self.ws_bytes),
              "set_stop_mask")

    # -------------------------------------------------------------- packing
    def pack_z(self, zs):
        import torch
        return torch.cat([torch.as_tensor(np.asarray(z, np.float32)).reshape(-1) for z in zs]).to(
            self.device)

    def pack_w(self, ws):
        import torch
        return torch.cat([torch.as_tensor(np.asarray(w, np.complex64)).reshape(-1) for w in ws]).to(
            self.device)

    def unpack_w(self, t, i):
        p = self.probs[i]
        return t[self.off_w[i]: self.off_w[i] + p["M"] * p["N"]].reshape(p["M"], p["N"])

    def unpack_z(self, t, i):
        p = self.probs[i]
        return t[self.off_z[i]: self.off_z[i] + p["M"] * p["N"] * p["L"]].reshape(
            p["M"], p["N"], p["L"])

    def unpack_adam(self, t, i):
        """Problem i's Adam state (flat: m_z, v_z, m_h, v_h as in SQNGD_ADAM_FLOATS)."""
        p = self.probs[i]
        return t[self.off_adam[i]: self.off_adam[i] + 2 * p["M"] * p["N"] * p["L"] + 4 * p["M"] * p["N"]]

    def unpack_roi(self, i):
        """Problem i's attached ROI weights [F][2N-1] (a view of the packed copy)."""
        off = sum(q["F"] * (2 * q["N"] - 1) for q in self.probs[:i])
        p = self.probs[i]
        return self.roi_w[off: off + p["F"] * (2 * p["N"] - 1)].reshape(p["F"], 2 * p["N"] - 1)

    def unpack_cube(self, t, i):
        p = self.probs[i]
        n = p["M"] * p["M"] * p["F"] * (2 * p["N"] - 1)
        return t[self.off_cube[i]: self.off_cube[i] + n].reshape(p["M"], p["M"], p["F"], 2 * p["N"] - 1)

    def new_stats(self, count=None):
        import torch
        return torch.zeros((count or self.n, STATS_WORDS), dtype=torch.int32, device=self.device)

    # --------------------------------------------------------------- entry points
    def af_forward(self, z, h, wave_mode=WAVE_SOFT, s_given=None, cube=False, stats=None):
        import torch
        stats = self.new_stats() if stats is None else stats
        cube_t = torch.empty(self.cube_c64, dtype=torch.complex64, device=self.device) if cube else None
        check(self.lib.sqngd_af_forward(self._arr, self.n, _ptr(z), int(wave_mode), _ptr(s_given),
                                        _ptr(h), _ptr(stats), _ptr(cube_t), self._ws_ptr,
                                        self.ws_bytes, _stream()), "af_forward")
        return (stats, cube_t) if cube else stats

    def af_backward(self, z, h, wave_mode=WAVE_SOFT, s_given=None, grad_loss=None, want_z=True,
                    want_h=True, want_s=False, stats=None):
        import torch
        gz = torch.empty(self.z_floats, dtype=torch.float32, device=self.device) if want_z else None
        gh = torch.empty(self.wave_c64, dtype=torch.complex64, device=self.device) if want_h else None
        gs = torch.empty(self.wave_c64, dtype=torch.complex64, device=self.device) if want_s else None
        check(self.lib.sqngd_af_backward(self._arr, self.n, _ptr(z), int(wave_mode), _ptr(s_given),
                                         _ptr(h), _ptr(grad_loss), _ptr(gz), _ptr(gh), _ptr(gs),
                                         _ptr(stats), self._ws_ptr, self.ws_bytes, _stream()),
              "af_backward")
        return gz, gh, gs

    def step(self, opt: Opt, z, h, adam, counter, stats=None):
        check(self.lib.sqngd_step(self._arr, self.n, ctypes.byref(opt), _ptr(z), _ptr(h), _ptr(adam),
                                  _ptr(counter), _ptr(stats), self._ws_ptr, self.ws_bytes,
                                  _stream()), "step")

    def run(self, opt: Opt, n_iters: int, z, h, adam, counter, stats=None):
        check(self.lib.sqngd_run(self._arr, self.n, ctypes.byref(opt), int(n_iters), _ptr(z), _ptr(h),
                                 _ptr(adam), _ptr(counter), _ptr(stats), self._ws_ptr, self.ws_bytes,
                                 _stream()), "run")

    def hard_quantize(self, z, want_idx=True, want_x=True):
        import torch
        idx = torch.empty(self.wave_c64, dtype=torch.int32, device=self.device) if want_idx else None
        x = torch.empty(self.wave_c64, dtype=torch.complex64, device=self.device) if want_x else None
        check(self.lib.sqngd_hard_quantize(self._arr, self.n, _ptr(z), _ptr(idx), _ptr(x),
                                           self._ws_ptr, self.ws_bytes, _stream()), "hard_quantize")
        return idx, x


def stop_update(stats, min_gain_db: float, patience: int, step_counter, best_db, stall, stopped, stop_iter):
    """sqngd_stop_update on the current stream: one checkpoint of the stopping
    rule for every problem whose hard statistics are in `stats`."""
    n = int(best_db.numel())
    check(load().sqngd_stop_update(n, _ptr(stats), float(min_gain_db), int(patience), _ptr(step_counter),
                                   _ptr(best_db), _ptr(stall), _ptr(stopped), _ptr(stop_iter), _stream()),
          "stop_update")
