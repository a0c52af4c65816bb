"""Host-side checks of the C ABI: exported symbols, struct layouts, and the
argument validation that runs before any HIP call (no GPU needed)."""
import ctypes
import os
import re

import pytest

from paper_2604_25728_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sqngd.h")
NET_HEADER = os.path.join(ROOT, "include", "sqngd_net.h")


@pytest.fixture(scope="module")
def nat():
    from paper_2604_25728_amd import native
    if not os.path.exists(native.LIB_PATH):
        from paper_2604_25728_amd import build
        build.build()
    native.load()
    return native


def _declared(path=HEADER):
    text = open(path).read()
    return sorted(set(re.findall(r"^(?:const\s+)?\w+\*?\s+\**(sqngd_\w+)\(", text, flags=re.M)))


def test_header_symbols_exported(nat):
    names = _declared()
    assert len(names) >= 9
    lib = nat.load()
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(nat.SYMBOLS) == names


def test_every_header_in_include_is_exported(nat):
    from paper_2604_25728_amd import netnative
    lib = nat.load()
    inc = os.path.join(ROOT, "include")
    for h in sorted(os.listdir(inc)):
        for n in _declared(os.path.join(inc, h)):
            assert hasattr(lib, n), (h, n)
    assert sorted(netnative.SYMBOLS) == _declared(NET_HEADER)
    from paper_2604_25728_amd import sqnnative
    assert sorted(sqnnative.SYMBOLS) == _declared(os.path.join(inc, "sqngd_sqn.h"))


def test_struct_layouts(nat):
    assert ctypes.sizeof(nat.Problem) == 64
    assert ctypes.sizeof(nat.Opt) == 44
    text = open(HEADER).read()
    assert "} sqngd_problem;" in text and "} sqngd_stats;" in text


def test_status_strings(nat):
    assert nat.status_string(0) == "ok"
    for rc in (-1, -2, -3, -4, -5, -6):
        assert nat.status_string(rc) != "unknown status"


def _arr(nat, **over):
    p = I.make_problem(2, 64, 4, 33, p=8.0)
    p.update(over)
    return nat.make_problems([p])


def _ws_size(nat, arr, n=1):
    b = ctypes.c_size_t()
    rc = nat.load().sqngd_workspace_size(arr, n, ctypes.byref(b))
    return rc, b.value


def test_workspace_size_and_buffer_sizes(nat):
    lib = nat.load()
    rc, nb = _ws_size(nat, _arr(nat))
    assert rc == 0 and nb > 0 and nb % 256 == 0
    zf, wc, af, cc = (ctypes.c_int64() for _ in range(4))
    probs = nat.make_problems([I.make_problem(2, 64, 4, 33), I.make_problem(3, 100, 8, 5)])
    assert lib.sqngd_buffer_sizes(probs, 2, ctypes.byref(zf), ctypes.byref(wc), ctypes.byref(af),
                                  ctypes.byref(cc)) == 0
    assert zf.value == 2 * 64 * 4 + 3 * 100 * 8
    assert wc.value == 2 * 64 + 3 * 100
    assert af.value == (2 * 2 * 64 * 4 + 4 * 2 * 64) + (2 * 3 * 100 * 8 + 4 * 3 * 100)
    assert cc.value == 4 * 33 * 127 + 9 * 5 * 199
    # the workspace grows with the batch
    rc2, nb2 = _ws_size(nat, probs, 2)
    assert rc2 == 0 and nb2 > nb


@pytest.mark.parametrize("field,value,code", [
    ("M", 0, -1), ("M", 17, -2), ("N", 1, -1), ("N", 2049, -2), ("L", 1, -1), ("L", 65, -2),
    ("F", 0, -1), ("F", 4097, -2), ("p", 1.5, -1), ("p", 65.0, -1), ("p", float("nan"), -1),
    ("temperature", 0.0, -1), ("w_psl", -1.0, -1), ("snrl_target_db", -0.1, -1),
    ("tau_lo", -64, -1), ("tau_hi", 64, -1), ("sq_mode", 2, -1), ("nu_min", 1.0, -1),
])
def test_problem_validation(nat, field, value, code):
    rc, _ = _ws_size(nat, _arr(nat, **{field: value}))
    assert rc == code, (field, value, rc)


def test_mask_schedule_and_pair_count_limits(nat):
    for mask, code in ((0, 0), (1, 0), (2, -1), (-1, -1)):
        arr = _arr(nat)
        arr[0].auto_mask = mask
        assert _ws_size(nat, arr)[0] == code, mask
    for sched, code in ((3, -1), (-1, -1), (34, -1), (41, -1), (0, 0), (1, 0), (2, 0), (4, 0), (8, 0), (12, 0),
                        (16, 0), (32, 0), (33, 0), (40, 0)):
        arr = _arr(nat)
        arr[0].schedule = sched
        assert _ws_size(nat, arr)[0] == code, sched
    # the largest problem the limits allow still has cell indices below 2^32
    assert _ws_size(nat, _arr(nat, M=16, N=1024, F=4096))[0] == 0


def test_entry_points_reject_before_touching_the_device(nat):
    lib = nat.load()
    arr = _arr(nat)
    fake = ctypes.c_void_p(0x100000)      # never dereferenced: validation fails first
    odd = ctypes.c_void_p(0x100002)
    ws = ctypes.c_void_p(0x200000)
    _, nb = _ws_size(nat, arr)
    stats = ctypes.c_void_p(0x300000)
    # bad wave mode / missing pointers
    assert lib.sqngd_af_forward(arr, 1, fake, 7, None, fake, stats, None, ws, nb, None) == -1
    assert lib.sqngd_af_forward(arr, 1, None, 0, None, fake, stats, None, ws, nb, None) == -1
    assert lib.sqngd_af_forward(arr, 1, fake, 2, None, fake, stats, None, ws, nb, None) == -1
    assert lib.sqngd_af_forward(arr, 1, fake, 0, None, None, stats, None, ws, nb, None) == -1
    # misalignment
    assert lib.sqngd_af_forward(arr, 1, fake, 0, None, odd, stats, None, ws, nb, None) == -4
    assert lib.sqngd_af_forward(arr, 1, fake, 0, None, fake, stats, None,
                                ctypes.c_void_p(0x200010), nb, None) == -4
    # workspace too small, then not initialised for this batch
    assert lib.sqngd_af_forward(arr, 1, fake, 0, None, fake, stats, None, ws, nb - 256, None) == -3
    assert lib.sqngd_af_forward(arr, 1, fake, 0, None, fake, stats, None, ws, nb, None) == -3
    # backward: logits gradient is undefined for a given waveform
    assert lib.sqngd_af_backward(arr, 1, None, 2, fake, fake, None, fake, None, None, None, ws, nb,
                                 None) == -1
    assert lib.sqngd_af_backward(arr, 1, fake, 0, None, fake, None, None, None, None, None, ws, nb,
                                 None) == -1
    # step options
    opt = nat.make_opt(I.make_opt())
    st = ctypes.c_void_p(0x400000)
    assert lib.sqngd_step(arr, 1, ctypes.byref(opt), fake, fake, fake, st, None, ws, nb, None) == -3
    for field, value in (("beta1", 1.0), ("eps", 0.0), ("lr_z", -1.0), ("n_h", -1), ("T0", 0.0),
                         ("total_iters", 0), ("flags", 8)):
        bad = nat.make_opt(I.make_opt())
        setattr(bad, field, value)
        assert lib.sqngd_step(arr, 1, ctypes.byref(bad), fake, fake, fake, st, None, ws, nb,
                              None) == -1, field
    zero = nat.make_opt(I.make_opt(n_h=0, n_x=0))
    assert lib.sqngd_step(arr, 1, ctypes.byref(zero), fake, fake, fake, st, None, ws, nb, None) == -1
    assert lib.sqngd_step(arr, 1, None, fake, fake, fake, st, None, ws, nb, None) == -1
    # hard quantise
    assert lib.sqngd_hard_quantize(arr, 1, fake, None, None, ws, nb, None) == -1
    assert lib.sqngd_hard_quantize(arr, 1, fake, fake, None, ws, nb, None) == -3
    # batch count
    assert lib.sqngd_workspace_init(arr, 0, ws, nb, None) == -1
    assert lib.sqngd_workspace_init(None, 1, ws, nb, None) == -1
    assert lib.sqngd_workspace_init(arr, 1, ws, nb - 256, None) == -3
    assert lib.sqngd_last_hip_error() == 0


def test_profile_hook_validation(nat):
    """The profiling switch validates its arguments on the host; switching it
    off needs no device."""
    lib = nat.load()
    assert lib.sqngd_profile_enable(-1, 1) == -1
    assert lib.sqngd_profile_enable(1, 0) == -1
    assert lib.sqngd_profile_enable(1, 1001) == -1
    assert lib.sqngd_profile_enable(1 << 17, 1) == -1
    assert lib.sqngd_profile_enable(0, 1) == 0
    cnt = ctypes.c_int32(-1)
    assert lib.sqngd_profile_read(None, 0, ctypes.byref(cnt)) == 0 and cnt.value == 0
    assert lib.sqngd_profile_read(None, 0, None) == -1


def test_net_validation(nat):
    """Network shape checks run on the host; counts follow the layer table."""
    from paper_2604_25728_amd import netnative as NN
    lib = NN.lib()
    n = ctypes.c_int64()
    b = ctypes.c_size_t()
    ok = NN.shape(4, 512, 8, 16)
    assert lib.sqngd_net_param_count(ctypes.byref(ok), ctypes.byref(n)) == 0
    assert n.value == I.net_param_count(4, 8)
    assert lib.sqngd_net_workspace_size(ctypes.byref(ok), ctypes.byref(b)) == 0 and b.value > 0
    for args, code in (((7, 512, 8, 16), -2), ((4, 500, 8, 16), -2), ((4, 512, 6, 16), -2),
                       ((3, 512, 4, 16), -2), ((4, 512, 8, 0), -1), ((0, 512, 8, 4), -1)):
        s = NN.shape(*args)
        assert lib.sqngd_net_param_count(ctypes.byref(s), ctypes.byref(n)) == code, args
    bad = NN.shape(4, 512, 8, 16, cond=(float("nan"), 1.0))
    assert lib.sqngd_net_workspace_size(ctypes.byref(bad), ctypes.byref(b)) == -1
    # entry points reject before touching the device
    assert lib.sqngd_net_forward(ctypes.byref(ok), None, None, None, None, 0, None) == -1
    dummy = ctypes.c_void_p(256)
    assert lib.sqngd_net_forward(ctypes.byref(ok), dummy, dummy, dummy, dummy, 16, None) == -3
    assert lib.sqngd_net_backward(ctypes.byref(ok), None, None, None, dummy, None, dummy, 1 << 40, None) == -1
    o = NN.NetOpt(1e-3, 0.9, 0.999, 1e-8)
    assert lib.sqngd_net_adam(ctypes.byref(ok), ctypes.byref(o), 0, dummy, dummy, dummy, None) == -1


def test_set_roi_weights_validation(nat):
    """Argument checks of sqngd_set_roi_weights run before any HIP call."""
    import ctypes
    lib = nat.load()
    probs = nat.make_problems([I.config("m2n64")["problem"]])
    ws = ctypes.create_string_buffer(1 << 16)
    base = (ctypes.addressof(ws) + 255) // 256 * 256
    # a misaligned weight pointer
    assert lib.sqngd_set_roi_weights(probs, 1, ctypes.c_void_p(base + 2), ctypes.c_void_p(base), 1 << 15) == -4
    # no problems
    assert lib.sqngd_set_roi_weights(None, 1, None, ctypes.c_void_p(base), 1 << 15) == -1
    # a workspace that was never initialised for this batch
    assert lib.sqngd_set_roi_weights(probs, 1, None, ctypes.c_void_p(base), 1 << 15) in (-3,)


def test_sqn_validation(nat):
    """Argument checks of the transmit-network entry points (no HIP call)."""
    import ctypes
    from paper_2604_25728_amd import sqnnative as SN
    lib = SN.lib()
    n = ctypes.c_int64()
    assert lib.sqngd_sqn_param_count(0, ctypes.byref(n)) == -1
    assert lib.sqngd_sqn_param_count(4097, ctypes.byref(n)) == -2
    assert lib.sqngd_sqn_param_count(32, ctypes.byref(n)) == 0
    assert n.value == I.sqn_param_count(32)
    b = ctypes.c_size_t()
    good = SN.SqnShape(2, 16, 4, 3, 30.0, 0, (ctypes.c_int32 * 2)(0, 0))
    assert lib.sqngd_sqn_workspace_size(ctypes.byref(good), ctypes.byref(b)) == 0 and b.value > 0
    for bad, rc in (((2, 16, 1, 3, 30.0), -1), ((2, 16, 4, 3, -1.0), -1), ((2, 16, 65, 3, 30.0), -2),
                    ((2, 16, 4, 2000, 30.0), -2), ((64, 128, 4, 3, 30.0), -2), ((2, 16, 4, 3, 30.0, -1), -1),
                    ((2, 16, 4, 3, 30.0, 65536), -2)):
        bad = bad if len(bad) == 6 else bad + (0,)
        sh = SN.SqnShape(*bad, (ctypes.c_int32 * 2)(0, 0))
        assert lib.sqngd_sqn_workspace_size(ctypes.byref(sh), ctypes.byref(b)) == rc, bad
    assert lib.sqngd_sqn_sort(None, 4, 1, None) == -1
    assert lib.sqngd_sqn_sort(ctypes.c_void_p(16), 4, 0, None) == -1
    assert lib.sqngd_sqn_sort(ctypes.c_void_p(16), 5000, 1, None) == -2
    # R stacked designs: the workspace is R slices of one design's
    one, three = ctypes.c_size_t(), ctypes.c_size_t()
    assert lib.sqngd_sqn_workspace_size(ctypes.byref(SN.SqnShape(2, 16, 4, 3, 30.0, 1, (ctypes.c_int32 * 2)(0, 0))),
                                        ctypes.byref(one)) == 0
    assert lib.sqngd_sqn_workspace_size(ctypes.byref(SN.SqnShape(2, 16, 4, 3, 30.0, 3, (ctypes.c_int32 * 2)(0, 0))),
                                        ctypes.byref(three)) == 0
    assert one.value == b.value and three.value >= 3 * one.value - 256
    assert lib.sqngd_sqn_adam(None, None, None, None, 4, None, 0, 1, 1e-3, 0.9, 0.999, 1e-8, None) == -1
    v = ctypes.c_void_p(256)
    assert lib.sqngd_sqn_adam(v, v, v, v, 4, None, 0, 0, 1e-3, 0.9, 0.999, 1e-8, None) == -1  # t = 0
    assert lib.sqngd_sqn_count(None, None) == -1
    assert lib.sqngd_sqn_project(0, 4, ctypes.c_void_p(16), None) == -1
    # forward reads theta in 16-byte pieces; a 4-byte-aligned theta is refused
    ws = ctypes.c_void_p(4096)
    assert lib.sqngd_sqn_forward(ctypes.byref(good), ctypes.c_void_p(260), v, v, ws, b.value, None) == -4
    assert lib.sqngd_sqn_forward(ctypes.byref(good), v, v, v, ws, b.value - 4, None) == -3
    # fused Adam entry points: the same argument checks as sqngd_sqn_adam
    assert lib.sqngd_sqn_adam_project(0, 4, v, v, v, v, None, 0, 1, 1e-3, 0.9, 0.999, 1e-8, None) == -1
    assert lib.sqngd_sqn_adam_project(2, 4, v, v, v, v, None, 0, 0, 1e-3, 0.9, 0.999, 1e-8, None) == -1
    assert lib.sqngd_sqn_adam_sort(v, v, v, v, 5000, 1, None, 0, 1, 1e-3, 0.9, 0.999, 1e-8, None) == -2
    assert lib.sqngd_sqn_adam_sort(v, v, v, v, 4, 1, None, 0, 1, 1e-3, 1.0, 0.999, 1e-8, None) == -1
    # backward with Adam on theta: argument checks before any HIP call
    assert lib.sqngd_sqn_backward_adam(ctypes.byref(good), v, v, v, v, v, v, None, None, v, v, None, 0, 1, 1e-3,
                                       0.9, 0.999, 1e-8, ws, b.value, None) == -1
    assert lib.sqngd_sqn_backward_adam(ctypes.byref(good), v, v, v, v, v, v, None, v, v, v, None, 0, 0, 1e-3,
                                       0.9, 0.999, 1e-8, ws, b.value, None) == -1


def test_noalloc_validation_before_any_hip_call(nat):
    """sqngd_af_backward_noalloc checks its arguments and the batch's scratch
    need on the host: bad arguments and a batch larger than the static scratch
    return their status without touching the device (no GPU here)."""
    lib = nat.load()
    fake = ctypes.c_void_p(1 << 20)   # aligned, never dereferenced on these paths
    big = nat.make_problems([I.make_problem(16, 2048, 64, 129)])
    rc, need = _ws_size(nat, big)
    assert rc == 0 and need > nat.NOALLOC_SCRATCH_BYTES
    rc = lib.sqngd_af_backward_noalloc(big, 1, fake, 0, None, fake, None, fake, fake, None, None, None)
    assert rc == nat.E_SCRATCH
    arr = _arr(nat)
    # NULL filters, bad mode, GIVEN without waveforms, misaligned output
    assert lib.sqngd_af_backward_noalloc(arr, 1, fake, 0, None, None, None, fake, None, None, None, None) == -1
    assert lib.sqngd_af_backward_noalloc(arr, 1, fake, 7, None, fake, None, fake, None, None, None, None) == -1
    assert lib.sqngd_af_backward_noalloc(arr, 1, None, 2, None, fake, None, None, fake, None, None, None) == -1
    assert lib.sqngd_af_backward_noalloc(arr, 1, fake, 0, None, fake, None, ctypes.c_void_p((1 << 20) + 2),
                                         None, None, None, None) == -4
    # an invalid problem
    bad = _arr(nat, p=1.0)
    assert lib.sqngd_af_backward_noalloc(bad, 1, fake, 0, None, fake, None, fake, None, None, None, None) == -1


def test_workspace_release_of_unknown_workspace(nat):
    lib = nat.load()
    assert lib.sqngd_workspace_release(ctypes.c_void_p(1 << 24)) == -1
    assert lib.sqngd_workspace_release(None) == -1


def test_stop_update_validation(nat):
    lib = nat.load()
    fake = ctypes.c_void_p(1 << 20)
    f = ctypes.c_float
    assert lib.sqngd_stop_update(0, fake, f(0.0), 2, None, fake, fake, fake, fake, None) == -1
    assert lib.sqngd_stop_update(4, fake, f(0.0), 0, None, fake, fake, fake, fake, None) == -1
    assert lib.sqngd_stop_update(4, None, f(0.0), 2, None, fake, fake, fake, fake, None) == -1
    assert lib.sqngd_stop_update(4, fake, f(float("nan")), 2, None, fake, fake, fake, fake, None) == -1
    assert lib.sqngd_stop_update(4, fake, f(0.0), 2, None, ctypes.c_void_p((1 << 20) + 2), fake, fake, fake,
                                 None) == -4
    assert lib.sqngd_set_stop_mask(_arr(nat), 1, ctypes.c_void_p(3), fake, 1 << 20) == -4
