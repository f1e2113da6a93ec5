"""Growth-rate fit of the transverse field energy (oracle side).  Test infrastructure.

Sec. 3 compares maximum instability growth rates.  Reading used here: the
transverse energy W(n) = 1/2 sum (Ex^2 + Ey^2 + Bx^2 + By^2) dV is recorded
every step; the fit window opens at the first step where W exceeds ten times
its running minimum and closes at the first later step where W exceeds 1e-2
of the initial beam kinetic energy (or at the last step).  The growth rate of
the field amplitude is half the least-squares slope of ln W against t = n dt.
"""
import math


def fit_window(W, wkin0):
    n = len(W)
    run_min = math.inf
    start = None
    for i, w in enumerate(W):
        if w > 0.0:
            run_min = min(run_min, w)
            if start is None and w > 10.0 * run_min:
                start = i
    if start is None:
        start = next((i for i, w in enumerate(W) if w > 0.0), 0)
    stop = n
    for i in range(start, n):
        if W[i] > 1e-2 * wkin0:
            stop = i + 1
            break
    return start, stop


def growth_rate(W, dt, wkin0):
    """Return (Gamma, (start, stop)); Gamma in inverse time units."""
    start, stop = fit_window(W, wkin0)
    pts = [(i * dt, math.log(W[i])) for i in range(start, stop) if W[i] > 0.0]
    if len(pts) < 2:
        return 0.0, (start, stop)
    # normal equations of the straight-line fit, written out
    m = len(pts)
    st = sum(t for t, _ in pts)
    sy = sum(y for _, y in pts)
    stt = sum(t * t for t, _ in pts)
    sty = sum(t * y for t, y in pts)
    slope = (m * sty - st * sy) / (m * stt - st * st)
    return 0.5 * slope, (start, stop)
