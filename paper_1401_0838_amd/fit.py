"""Growth rate of the numerical instability from a field-energy trace.

Sec. 3 reports maximum growth rates of the instability.  The transverse field
energy W(n) = 1/2 sum (Ex^2 + Ey^2 + Bx^2 + By^2) dV grows as exp(2 Gamma t)
while the instability is linear.  The fit window opens at the first step
where W has risen ten-fold above its running minimum and closes once W
reaches 1e-2 of the beam's initial kinetic energy (or at the end of the
trace); Gamma is half the slope of the least-squares line of ln W against t.
"""
import numpy as np


def growth_rate(W, dt, wkin0):
    W = np.asarray(W, dtype=np.float64)
    pos = W > 0
    if not pos.any():
        return 0.0, (0, len(W))
    runmin = np.minimum.accumulate(np.where(pos, W, np.inf))
    up = np.nonzero(pos & (W > 10.0 * runmin))[0]
    start = int(up[0]) if up.size else int(np.nonzero(pos)[0][0])
    hit = np.nonzero(W[start:] > 1e-2 * wkin0)[0]
    stop = start + int(hit[0]) + 1 if hit.size else len(W)
    sel = np.arange(start, stop)
    sel = sel[W[sel] > 0]
    if sel.size < 2:
        return 0.0, (start, stop)
    slope = np.polyfit(sel * dt, np.log(W[sel]), 1)[0]
    return 0.5 * float(slope), (start, stop)
