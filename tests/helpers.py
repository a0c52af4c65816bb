"""Small numpy helpers shared by the GPU parity tests (no arithmetic of the
method: they read an oracle cube)."""
import numpy as np


def peak_and_gap(cube, prob, weights=None):
    """The region-of-interest peak of w|A| over a cube [M][M][F][2N-1] in (m, l,
    f, tau) scan order -- as (m, l, tau, f) -- and the relative gap between
    the largest and the second largest cell value."""
    cube = np.asarray(cube)
    M, _, F, T = cube.shape
    N = (T + 1) // 2
    tau = np.arange(-(N - 1), N)
    v = np.abs(cube) * (1.0 if weights is None else np.asarray(weights)[None, None])
    inside = np.broadcast_to(((tau >= prob["tau_lo"]) & (tau <= prob["tau_hi"]))[None, None, None, :],
                             v.shape).copy()
    # auto pairs' tau = 0 cells outside the region: every bin (eq. 8), or with
    # auto_mask = 1 the bins of the Doppler mainlobe |nu| < 1
    cut = np.ones(F, dtype=bool)
    if prob.get("auto_mask", 0) == 1:
        cut = np.abs(np.linspace(prob["nu_min"], prob["nu_max"], F) if F > 1
                     else np.array([prob["nu_min"]])) < 1.0
    for m in range(M):
        inside[m, m, cut, N - 1] = False
    v = np.where(inside, v, -1.0).reshape(-1)
    top2 = np.partition(v, -2)[-2:]
    hi, lo = float(top2.max()), float(top2.min())
    m, l, f, k = np.unravel_index(int(np.argmax(v)), cube.shape)
    return (int(m), int(l), int(tau[k]), int(f)), (hi - lo) / hi


def check_peak(st, cube, prob, weights=None, margin=1e-4):
    """The GPU's reported peak cell equals the first largest oracle cell
    wherever that cell leads the next by more than `margin` (relative): FP32
    rounding cannot reorder cells that far apart. Returns whether it checked."""
    arg, gap = peak_and_gap(cube, prob, weights)
    if gap <= margin:
        return False
    assert tuple(st["arg"]) == arg, (st["arg"], arg, gap)
    return True
