"""Growth rate of the numerical instability from a field-energy trace.

Sec. 3 reports maximum growth rates of the instability.  The transverse field
energy W(n) = 1/2 sum (Ex^2 + Ey^2 + Bx^2 + By^2) dV grows as exp(2 Gamma t)
while the instability is linear.  A run starts from E = B = 0, so W first
rises from zero to the shot-noise level; that start-up rise is left out by
searching only after one plasma period 2 pi / omega_p.  The search stops once
W reaches 1e-2 of the beam's initial kinetic energy (or at the end of the
trace).  Gamma is half the steepest least-squares slope of ln W against
t = n dt over the windows of that span whose length is an eighth of it (at
least 16 steps): the maximum growth rate of the run.
"""
import math

import numpy as np

OMEGA_P = 0.1        # plasma frequency of the synthetic beams (c / dz units)
MIN_LEN = 16


def search_span(W, dt, wkin0, omega_p=OMEGA_P):
    """(first, stop) of the steps the window search covers."""
    n = len(W)
    first = min(n, int(math.ceil(2.0 * math.pi / (omega_p * dt))))
    hit = np.nonzero(np.asarray(W[first:], dtype=np.float64) > 1e-2 * wkin0)[0]
    stop = first + int(hit[0]) + 1 if hit.size else n
    return first, stop


def growth_rate(W, dt, wkin0, omega_p=OMEGA_P):
    """Return (Gamma, (start, stop)) with [start, stop) the steepest window."""
    W = np.asarray(W, dtype=np.float64)
    first, stop = search_span(W, dt, wkin0, omega_p)
    span = stop - first
    if span < 2:
        return 0.0, (first, stop)
    L = min(span, max(MIN_LEN, span // 8))
    seg = W[first:stop]
    if np.any(seg <= 0) or not np.all(np.isfinite(seg)):
        return float("nan"), (first, stop)
    y = np.log(seg)
    t = np.arange(span, dtype=np.float64) * dt     # shifted to the span's start: same slopes
    # least-squares slope of every window [s, s + L) from running sums
    cs = lambda v: np.concatenate(([0.0], np.cumsum(v)))
    St, Sy, Stt, Sty = cs(t), cs(y), cs(t * t), cs(t * y)
    k = np.arange(span - L + 1)
    st, sy = St[k + L] - St[k], Sy[k + L] - Sy[k]
    stt, sty = Stt[k + L] - Stt[k], Sty[k + L] - Sty[k]
    slope = (L * sty - st * sy) / (L * stt - st * st)
    best = int(np.argmax(slope))
    return 0.5 * float(slope[best]), (first + best, first + best + L)
