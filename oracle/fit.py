"""Growth-rate fit of the transverse field energy (oracle side).  Test infrastructure.

Sec. 3 compares maximum instability growth rates.  Reading used here: the
transverse energy W(n) = 1/2 sum (Ex^2 + Ey^2 + Bx^2 + By^2) dV is recorded
every step.  A run starts from E = B = 0, so W first climbs from zero to the
shot-noise level; the search for the growth phase starts after one plasma
period 2 pi / omega_p, which leaves that start-up rise out, and ends at the
first later step where W exceeds 1e-2 of the initial beam kinetic energy (or
at the last step).  Every window of consecutive steps inside that span whose
length is an eighth of the span (at least 16 steps) gets a least-squares
straight line of ln W against t = n dt; the growth rate of the field
amplitude is half the steepest of those slopes.
"""
import math

OMEGA_P = 0.1
MIN_LEN = 16


def search_span(W, dt, wkin0, omega_p=OMEGA_P):
    n = len(W)
    first = min(n, int(math.ceil(2.0 * math.pi / (omega_p * dt))))
    stop = n
    for i in range(first, n):
        if W[i] > 1e-2 * wkin0:
            stop = i + 1
            break
    return first, stop


def line_slope(ts, ys):
    """Least-squares slope, normal equations written out."""
    m = len(ts)
    st = sum(ts)
    sy = sum(ys)
    stt = sum(t * t for t in ts)
    sty = sum(t * y for t, y in zip(ts, ys))
    return (m * sty - st * sy) / (m * stt - st * st)


def growth_rate(W, dt, wkin0, omega_p=OMEGA_P):
    """Return (Gamma, (start, stop)); Gamma in inverse time units and [start,
    stop) the steepest window."""
    first, stop = search_span(W, dt, wkin0, omega_p)
    span = stop - first
    if span < 2:
        return 0.0, (first, stop)
    L = min(span, max(MIN_LEN, span // 8))
    if any(not (W[i] > 0.0) or math.isinf(W[i]) for i in range(first, stop)):
        return float("nan"), (first, stop)
    best, best_s = -math.inf, first
    for s in range(first, stop - L + 1):
        ts = [(i - first) * dt for i in range(s, s + L)]
        ys = [math.log(W[i]) for i in range(s, s + L)]
        k = line_slope(ts, ys)
        if k > best:
            best, best_s = k, s
    return 0.5 * best, (best_s, best_s + L)
