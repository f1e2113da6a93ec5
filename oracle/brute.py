"""Brute-force PIC step for tiny grids (pins the C oracle).  Test infrastructure.

Written independently of pic_oracle.c, in a different formulation, so that a
dropped term, a sign, an index or a transposed operand in either one shows up
as a mismatch:
  * curls are dense matrices built from periodic shift matrices (Kronecker
    products), not stencil loops (the Cole-Karkkainen curl as the product of
    an averaging matrix and the difference matrix);
  * the correction polynomials and filter passes are applied in Fourier space
    by an explicit DFT multiply: symbol s = sin^2(k_z dz / 2) for Psi (Sec. 2)
    and 1 - 4 w sin^2(k dx / 2) per (w, 1-2w, w) pass (Sec. 3, Eq. 6);
  * the gather weights are dense over every node, from the explicit spline
    formulas with periodic minimum-image distances;
  * the Boris rotation is written as a Rodrigues rotation by the angle
    2 atan(|t|) about -t (algebraically the same map as the Boris scheme);
  * the Esirkepov current is built from dense per-axis shape vectors with a
    periodic running sum started at a node outside the particle's support.
Grids must be large enough (>= 8 nodes on every active axis) for the minimum
image and for that start node to exist.
"""
import numpy as np


def spline(o, t):
    """Centred B-spline of order o at t (vectorised, piecewise definition)."""
    t = np.asarray(t, dtype=np.float64)
    a = np.abs(t)
    if o == 0:
        return np.where((t >= -0.5) & (t < 0.5), 1.0, 0.0)
    if o == 1:
        return np.where(a < 1.0, 1.0 - a, 0.0)
    if o == 2:
        return np.where(a < 0.5, 0.75 - a * a, np.where(a < 1.5, 0.5 * (1.5 - a) ** 2, 0.0))
    if o == 3:
        return np.where(a < 1.0, 2.0 / 3.0 - a * a + 0.5 * a ** 3,
                        np.where(a < 2.0, (2.0 - a) ** 3 / 6.0, 0.0))
    raise ValueError(o)


def _minimg(t, n):
    """Periodic minimum-image offset in [-n/2, n/2)."""
    return np.mod(t + 0.5 * n, n) - 0.5 * n


class BruteSim:
    """State: E, B, J as (3, nz, ny, nx); particles x (3, N) absolute, u (3, N)."""

    STAG_E = ((1, 0, 0), (0, 1, 0), (0, 0, 1))
    STAG_B = ((0, 1, 1), (1, 0, 1), (1, 1, 0))

    def __init__(self, dims, shape, d, dt, order, q, m, w, psi_e=None, psi_b=None,
                 filt=(), jbg=(0.0, 0.0, 0.0), interp="galerkin", solver="yee", ratio=False):
        self.dims = dims
        self.shape = tuple(shape)                 # (nz, ny, nx)
        self.d = tuple(d)                         # (dx, dy, dz)
        self.dt, self.order, self.q, self.m, self.w = dt, order, q, m, w
        self.psi_e, self.psi_b = psi_e, psi_b
        self.filt = list(filt)
        self.jbg = np.asarray(jbg, dtype=np.float64)
        self.interp = interp
        self.ratio = ratio
        nz, ny, nx = self.shape
        self.N = nx * ny * nz
        self.E = np.zeros((3,) + self.shape)
        self.B = np.zeros((3,) + self.shape)
        self.J = np.zeros((3,) + self.shape)
        # dense shift matrices: (Sh[a] f)[p] = f[p + e_a] (periodic)
        idx = np.arange(self.N).reshape(self.shape)
        self.Sh = []
        for axis in (2, 1, 0):                    # array axis of x, y, z
            tgt = np.roll(idx, -1, axis=axis).ravel()
            M = np.zeros((self.N, self.N))
            M[np.arange(self.N), tgt] = 1.0
            self.Sh.append(M)
        I = np.eye(self.N)
        self.Df = [(self.Sh[a] - I) / self.d[a] for a in range(3)]     # forward
        self.Db = [(I - self.Sh[a].T) / self.d[a] for a in range(3)]   # backward
        if dims == 2:
            self.Df[1] = np.zeros_like(I)
            self.Db[1] = np.zeros_like(I)
        # Faraday's law differences: Yee, or Cole-Karkkainen (2D): the x difference
        # smoothed along z and the z difference along x by the symmetric
        # (1/8, 3/4, 1/8) average, as matrix products
        self.DfF = list(self.Df)
        if solver == "ck":
            beta = 0.125
            avg = [(1 - 2 * beta) * I + beta * (self.Sh[a] + self.Sh[a].T) for a in range(3)]
            self.DfF[0] = avg[2] @ self.Df[0]
            self.DfF[2] = avg[0] @ self.Df[2]

    # ---------------------------------------------------------- fields
    def _curl(self, F, D):
        Fx, Fy, Fz = (F[c].ravel() for c in range(3))
        cx = D[1] @ Fz - D[2] @ Fy
        cy = D[2] @ Fx - D[0] @ Fz
        cz = D[0] @ Fy - D[1] @ Fx
        return np.stack([cx, cy, cz]).reshape((3,) + self.shape)

    def yee(self):
        self.B -= 0.5 * self.dt * self._curl(self.E, self.DfF)
        jt = self.J + self.jbg[:, None, None, None]
        self.E += self.dt * (self._curl(self.B, self.Db) - jt)
        self.B -= 0.5 * self.dt * self._curl(self.E, self.DfF)

    def _symbols(self):
        nz, ny, nx = self.shape
        kz = 2 * np.pi * np.fft.fftfreq(nz)[:, None, None]
        ky = 2 * np.pi * np.fft.fftfreq(ny)[None, :, None]
        kx = 2 * np.pi * np.fft.fftfreq(nx)[None, None, :]
        sz = np.sin(kz / 2) ** 2
        filt = np.ones(self.shape)
        axes = [kx, kz] if self.dims == 2 else [kx, ky, kz]
        for k in axes:
            for wgt in self.filt:
                filt = filt * (1.0 - 4.0 * wgt * np.sin(k / 2) ** 2)
        return sz, filt

    def seen_plane(self, F, coef):
        sz, filt = self._symbols()
        P = np.zeros_like(sz) + (1.0 if coef is None else 0.0)
        if coef is not None:
            for j, a in enumerate(coef):
                P = P + a * sz ** j
        return np.real(np.fft.ifftn(np.fft.fftn(F) * P * filt))

    def seen(self):
        pe, pb = self.psi_e, self.psi_b
        if self.ratio:
            # Psi_E / Psi_B as one Fourier multiplier on the transverse E only
            sz, filt = self._symbols()
            mult = sum(a * sz ** j for j, a in enumerate(pe)) / sum(b * sz ** j for j, b in enumerate(pb))
            Et = np.stack([np.real(np.fft.ifftn(np.fft.fftn(self.E[c]) * mult * filt)) for c in range(2)]
                          + [self.seen_plane(self.E[2], None)])
            Bt = np.stack([self.seen_plane(self.B[c], None) for c in range(3)])
            return Et, Bt
        Et = np.stack([self.seen_plane(self.E[0], pe), self.seen_plane(self.E[1], pe),
                       self.seen_plane(self.E[2], pb)])
        Bt = np.stack([self.seen_plane(self.B[c], pb) for c in range(3)])
        return Et, Bt

    # ---------------------------------------------------------- particles
    def _weights(self, pos, stag, ords):
        """Dense (nz, ny, nx) interpolation weights for one point."""
        nz, ny, nx = self.shape
        n = (nx, ny, nz)
        vecs = []
        for a in range(3):
            if a == 1 and self.dims == 2:
                vecs.append(np.ones(1))
                continue
            c = pos[a] / self.d[a]
            if self.interp == "momentum":
                # weights w_n on the integer nodes, each node holding the mean of
                # the Yee samples at n - 1/2 and n + 1/2 (array slots n - 1 and n):
                # sample m then carries (w_m + w_{m+1}) / 2
                w = spline(ords[a], _minimg(c - np.arange(n[a]), n[a]))
                if stag[a]:
                    w = 0.5 * (w + np.roll(w, -1))
                vecs.append(w)
                continue
            nodes = np.arange(n[a]) + 0.5 * stag[a]
            vecs.append(spline(ords[a], _minimg(c - nodes, n[a])))
        return vecs[2][:, None, None] * vecs[1][None, :, None] * vecs[0][None, None, :]

    def _ords(self, stag):
        if self.interp == "galerkin":
            return [self.order - s for s in stag]
        return [self.order] * 3

    def gather(self, pos, Et, Bt):
        Eo = np.array([np.sum(self._weights(pos, self.STAG_E[c], self._ords(self.STAG_E[c])) * Et[c])
                       for c in range(3)])
        Bo = np.array([np.sum(self._weights(pos, self.STAG_B[c], self._ords(self.STAG_B[c])) * Bt[c])
                       for c in range(3)])
        return Eo, Bo

    def boris(self, u, E, B):
        eps = self.q * self.dt / (2.0 * self.m)
        um = u + eps * E
        g = np.sqrt(1.0 + um @ um)
        t = eps * B / g
        tn = np.sqrt(t @ t)
        if tn == 0.0:
            up = um
        else:
            nvec = -t / tn
            th = 2.0 * np.arctan(tn)
            up = (um * np.cos(th) + np.cross(nvec, um) * np.sin(th)
                  + nvec * (nvec @ um) * (1.0 - np.cos(th)))
        return up + eps * E

    def _shape_vec(self, c, n):
        return spline(self.order, _minimg(c - np.arange(n), n))

    def deposit(self, p0, p1, vy):
        nz, ny, nx = self.shape
        n = (nx, ny, nz)
        S0, S1, DS = [], [], []
        for a in range(3):
            if a == 1 and self.dims == 2:
                S0.append(np.ones(1)); S1.append(np.ones(1)); DS.append(np.zeros(1))
                continue
            s0 = self._shape_vec(p0[a] / self.d[a], n[a])
            s1 = self._shape_vec(p1[a] / self.d[a], n[a])
            S0.append(s0); S1.append(s1); DS.append(s1 - s0)
        qw = self.q * self.w
        if self.dims == 2:
            dV = self.d[0] * self.d[2]
        else:
            dV = self.d[0] * self.d[1] * self.d[2]

        def run_sum(W, axis, a):
            # periodic running sum along `axis`, started just after a node that
            # lies outside both the old and the new support on that axis
            start = int(np.nonzero((S0[a] == 0.0) & (S1[a] == 0.0))[0][0])
            Wr = np.roll(W, -(start + 1), axis=axis)
            cs = np.cumsum(Wr, axis=axis)
            return np.roll(cs, start + 1, axis=axis)

        def tri(Sb0, DSb, Sc0, DSc):
            return (np.outer(Sb0, Sc0) + 0.5 * np.outer(DSb, Sc0) + 0.5 * np.outer(Sb0, DSc)
                    + np.outer(DSb, DSc) / 3.0)

        if self.dims == 2:
            # arrays indexed [z, x] then expanded to (nz, 1, nx)
            Wx = np.outer(S0[2] + 0.5 * DS[2], DS[0])
            Wz = np.outer(DS[2], S0[0] + 0.5 * DS[0])
            Jx = -qw * self.d[0] / (self.dt * dV) * run_sum(Wx, 1, 0)
            Jz = -qw * self.d[2] / (self.dt * dV) * run_sum(Wz, 0, 2)
            Wy = tri(S0[2], DS[2], S0[0], DS[0])
            Jy = qw * vy / dV * Wy
            self.J[0] += Jx[:, None, :]
            self.J[1] += Jy[:, None, :]
            self.J[2] += Jz[:, None, :]
            return
        # 3D: build each W on the (z, y, x) grid
        Wx = DS[0][None, None, :] * tri(S0[2], DS[2], S0[1], DS[1])[:, :, None]
        Wy = DS[1][None, :, None] * tri(S0[2], DS[2], S0[0], DS[0])[:, None, :]
        Wz = DS[2][:, None, None] * tri(S0[1], DS[1], S0[0], DS[0])[None, :, :]
        self.J[0] += -qw * self.d[0] / (self.dt * dV) * run_sum(Wx, 2, 0)
        self.J[1] += -qw * self.d[1] / (self.dt * dV) * run_sum(Wy, 1, 1)
        self.J[2] += -qw * self.d[2] / (self.dt * dV) * run_sum(Wz, 0, 2)

    def step(self, x, u):
        """Advance fields and particles (x, u arrays of shape (3, N), modified in place)."""
        self.yee()
        Et, Bt = self.seen()
        self.J[:] = 0.0
        nz, ny, nx = self.shape
        L = (nx * self.d[0], ny * self.d[1], nz * self.d[2])
        for p in range(x.shape[1]):
            p0 = x[:, p].copy()
            Eo, Bo = self.gather(p0, Et, Bt)
            un = self.boris(u[:, p], Eo, Bo)
            g = np.sqrt(1.0 + un @ un)
            v = un / g
            p1 = p0 + self.dt * v
            if self.dims == 2:
                p1[1] = p0[1]
            self.deposit(p0, p1, v[1])
            u[:, p] = un
            x[:, p] = np.mod(p1, L)
            if self.dims == 2:
                x[1, p] = 0.0
