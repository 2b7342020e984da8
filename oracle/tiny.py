"""Second, independent FP64 oracle in numpy, for tiny grids.

TEST INFRASTRUCTURE ONLY.  Written separately from the C oracle (whole-array
numpy operations on a ghost-padded copy instead of per-point loops) so that
agreement between the two checks each of them.  Same method and readings:
8th-order 25-point Laplacian (section "Finite Differences"), leapfrog
Eq. (minimod-semidisc), zero ghost cells or periodic wrap, Cerjan sponge,
kappa = 1 recursive-convolution CPML, exact discrete adjoint and gradient
with respect to m = 1/v^2.  Arrays are [z][y][x].
"""
import math

import numpy as np

BC_NONE, BC_SPONGE, BC_CPML, BC_PERIODIC = 0, 1, 2, 3
R4 = 4
# second-derivative weights (fractions written out) and first-derivative weights
_A = np.array([1.6, -0.2, 8.0 / 315.0, -1.0 / 560.0])
_B = np.array([0.8, -0.2, 4.0 / 105.0, -1.0 / 280.0])


def _pad(f, periodic):
    return np.pad(f, R4, mode="wrap" if periodic else "constant")


def _shift(fp, axis, m):
    """View of the padded field displaced by m cells along axis (0=x,1=y,2=z)."""
    nz, ny, nx = (s - 2 * R4 for s in fp.shape)
    sl = [slice(R4, R4 + nz), slice(R4, R4 + ny), slice(R4, R4 + nx)]
    ai = 2 - axis
    sl[ai] = slice(R4 + m, R4 + m + (nz, ny, nx)[ai])
    return fp[tuple(sl)]


def d2(f, axis, h, periodic=False):
    fp = _pad(f, periodic)
    out = np.zeros_like(f)
    for m in range(1, 5):
        out += _A[m - 1] * (_shift(fp, axis, m) + _shift(fp, axis, -m) - 2.0 * f)
    return out / (h * h)


def d1(f, axis, h, periodic=False):
    fp = _pad(f, periodic)
    out = np.zeros_like(f)
    for m in range(1, 5):
        out += _B[m - 1] * (_shift(fp, axis, m) - _shift(fp, axis, -m))
    return out / h


def lap(f, h, periodic=False):
    return sum(d2(f, ax, h[ax], periodic) for ax in range(3))


def _depth(n, nb):
    k = np.arange(n)
    return np.maximum(np.maximum(nb - k, nb - (n - 1 - k)), 0)


def sponge(shape, nb, sigma):
    nz, ny, nx = shape
    g1 = [np.where(_depth(n, nb) > 0, np.exp(-(sigma * _depth(n, nb)) ** 2), 1.0) for n in (nx, ny, nz)]
    return g1[2][:, None, None] * g1[1][None, :, None] * g1[0][None, None, :]


def cpml_ab(n, nb, h, dt, vmax, R, f0):
    dep = _depth(n, nb)
    q = dep / nb
    d0 = -3.0 * vmax * math.log(R) / (2.0 * nb * h)
    d = d0 * q * q
    alpha = math.pi * f0 * (1.0 - q)
    b = np.exp(-(d + alpha) * dt)
    with np.errstate(invalid="ignore", divide="ignore"):
        a = np.where(d + alpha > 0, d * (b - 1.0) / (d + alpha), 0.0)
    inside = dep == 0
    return np.where(inside, 0.0, a), np.where(inside, 1.0, b), ~inside


def _bcast(v, axis):
    return v[None, None, :] if axis == 0 else (v[None, :, None] if axis == 1 else v[:, None, None])


class Problem:
    def __init__(self, shape, h, dt, vel, bc=BC_NONE, nb=0, sigma=0.015, R=1e-3, f0=15.0, vmax=None):
        self.shape = tuple(shape)
        self.h = tuple(float(x) for x in h)  # (hx, hy, hz)
        self.dt = float(dt)
        self.vel = np.asarray(vel, dtype=np.float64)
        self.D = (self.dt * self.vel) ** 2
        self.bc = bc
        self.periodic = bc == BC_PERIODIC
        self.G = sponge(self.shape, nb, sigma) if bc == BC_SPONGE else np.ones(self.shape)
        if bc == BC_CPML:
            vmax = float(self.vel.max()) if vmax is None else vmax
            n_ax = (self.shape[2], self.shape[1], self.shape[0])
            self.cp = [cpml_ab(n_ax[ax], nb, self.h[ax], self.dt, vmax, R, f0) for ax in range(3)]

    def _source(self, pts, vals, scale):
        s = np.zeros(self.shape)
        for (i, j, k), v in zip(pts, vals):
            s[k, j, i] += v * scale
        return s

    def step(self, pm, pc, s, mem):
        L = lap(pc, self.h, self.periodic)
        if self.bc == BC_CPML:
            for ax in range(3):
                a, b, inl = (_bcast(x, ax) for x in self.cp[ax])
                psi = np.where(inl, b * mem[ax] + a * d1(pc, ax, self.h[ax]), 0.0)
                dpsi = d1(psi, ax, self.h[ax])
                zeta = np.where(inl, b * mem[3 + ax] + a * (d2(pc, ax, self.h[ax]) + dpsi), 0.0)
                L = L + np.where(inl, dpsi + zeta, 0.0)
                mem[ax] = psi
                mem[3 + ax] = zeta
        G = self.G
        return G * (2.0 * pc - G * pm + self.D * (L + s))

    def forward(self, src, wav, rec, T, pm=None, pc=None, keep=False):
        pm = np.zeros(self.shape) if pm is None else pm.copy()
        pc = np.zeros(self.shape) if pc is None else pc.copy()
        mem = np.zeros((6,) + self.shape)
        inv_vol = 1.0 / (self.h[0] * self.h[1] * self.h[2])
        traces = np.zeros((T, len(rec)))
        hist = [pm, pc]
        for n in range(T):
            s = self._source(src, wav[n], inv_vol)
            pn = self.step(pm, pc, s, mem)
            traces[n] = [pn[k, j, i] for (i, j, k) in rec]
            pm, pc = pc, pn
            if keep:
                hist.append(pn)
        return traces, pm, pc, (hist if keep else None)

    def adjoint(self, rec, resid, T, src):
        assert self.bc != BC_CPML
        e2 = np.zeros(self.shape)
        e1 = np.zeros(self.shape)
        adj = np.zeros((T, len(src)))
        etas = [None] * (T + 1)
        for m in range(T, 0, -1):
            rt = self._source(rec, resid[m - 1], 1.0)
            en = self.step(e2, e1, rt, None)
            adj[m - 1] = [en[k, j, i] for (i, j, k) in src]
            etas[m] = en
            e2, e1 = e1, en
        return adj, etas

    def gradient(self, src, wav, rec, d_obs, T):
        traces, _, _, hist = self.forward(src, wav, rec, T, keep=True)
        resid = traces - d_obs
        loss = 0.5 * float(np.sum(resid ** 2))
        _, etas = self.adjoint(rec, resid, T, src)
        G = self.G
        grad = np.zeros(self.shape)
        # hist[t + 1] = p^t for t = -1 .. T
        for n in range(T):
            d2p = hist[n + 2] - 2.0 * G * hist[n + 1] + G * G * hist[n]
            grad -= etas[n + 1] * d2p / (self.dt ** 2 * G)
        return grad, traces, loss
