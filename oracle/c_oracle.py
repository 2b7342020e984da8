"""ctypes wrapper of the plain-C FP64 oracle (minimod_oracle.c).

TEST INFRASTRUCTURE ONLY.  Every array crossing this boundary is a C-ordered
numpy array indexed [z][y][x] (x fastest); point lists are int32 [n][3] in
(i, j, k) = (x, y, z) order.

Boundary kinds: 0 none (zero ghost cells), 1 sponge, 2 CPML, 3 periodic;
fs = 1 puts a free surface on the top face (p = 0 at k = 0, odd mirror above).
"""
import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = os.path.join(_HERE, "liboracle.so")

BC_NONE, BC_SPONGE, BC_CPML, BC_PERIODIC = 0, 1, 2, 3


class _Grid(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("hx", ctypes.c_double), ("hy", ctypes.c_double), ("hz", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("bc", ctypes.c_int), ("nb", ctypes.c_int),
        ("sigma", ctypes.c_double),
        ("R", ctypes.c_double), ("f0", ctypes.c_double), ("vmax", ctypes.c_double),
        ("wx0", ctypes.c_int), ("wy0", ctypes.c_int), ("wz0", ctypes.c_int),
        ("wnx", ctypes.c_int), ("wny", ctypes.c_int), ("wnz", ctypes.c_int),
        ("fs", ctypes.c_int),
    ]


@dataclass
class Grid:
    """Problem description for the oracle (sizes in cells, metres, seconds)."""
    nx: int
    ny: int
    nz: int
    hx: float
    hy: float
    hz: float
    dt: float
    bc: int = BC_NONE
    nb: int = 0
    sigma: float = 0.015
    R: float = 1e-3
    f0: float = 15.0
    vmax: float = 0.0
    fs: int = 0  # free surface at k = 0

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def n(self):
        return self.nx * self.ny * self.nz

    def _c(self, window=None):
        w = (0, 0, 0, 0, 0, 0) if window is None else tuple(window[0]) + tuple(window[1])
        return _Grid(self.nx, self.ny, self.nz, self.hx, self.hy, self.hz, self.dt,
                     self.bc, self.nb, self.sigma, self.R, self.f0, self.vmax, *w, int(self.fs))


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            raise RuntimeError(f"oracle library not built: {_LIB} (run `make -C oracle`)")
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        fp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        gp = ctypes.POINTER(_Grid)
        L.orc_dt_stab.restype = ctypes.c_double
        L.orc_dt_stab.argtypes = [ctypes.c_double] * 4
        L.orc_ricker.restype = None
        L.orc_ricker.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int, dp]
        L.orc_laplacian.restype = None
        L.orc_laplacian.argtypes = [gp, dp, dp]
        L.orc_sponge_G.restype = ctypes.c_double
        L.orc_sponge_G.argtypes = [gp, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.orc_cpml_coeffs.restype = None
        L.orc_cpml_coeffs.argtypes = [gp, ctypes.c_int, ctypes.c_int, dp, dp]
        L.orc_forward.restype = ctypes.c_int
        L.orc_forward.argtypes = [gp, fp, ctypes.c_int, ip, dp, ctypes.c_int, ip, ctypes.c_int, dp, dp, dp, dp]
        L.orc_step_points.restype = ctypes.c_int
        L.orc_step_points.argtypes = [gp, fp, dp, dp, dp, ctypes.c_int, ip, dp, dp]
        L.orc_energy.restype = ctypes.c_double
        L.orc_energy.argtypes = [gp, fp, dp, dp]
        L.orc_adjoint.restype = ctypes.c_int
        L.orc_adjoint.argtypes = [gp, fp, ctypes.c_int, ip, dp, ctypes.c_int, ctypes.c_int, ip, dp]
        L.orc_gradient.restype = ctypes.c_int
        L.orc_gradient.argtypes = [gp, fp, ctypes.c_int, ip, dp, ctypes.c_int, ip, dp, ctypes.c_int,
                                   ctypes.c_int, dp, dp, dp]
        L.orc_num_threads.restype = ctypes.c_int
        L.orc_num_threads.argtypes = []
        L.orc_set_num_threads.restype = None
        L.orc_set_num_threads.argtypes = [ctypes.c_int]
        L.orc_iso_dt_stab.restype = ctypes.c_double
        L.orc_iso_dt_stab.argtypes = [ctypes.c_double] * 4
        L.orc_iso_dplus.restype = None
        L.orc_iso_dplus.argtypes = [gp, dp, ctypes.c_int, dp]
        L.orc_iso_forward.restype = ctypes.c_int
        L.orc_iso_forward.argtypes = [gp, fp, dp, ctypes.c_int, ip, dp, ctypes.c_int, ip, ctypes.c_int, dp, dp]
        L.orc_iso_cpml_coeffs.restype = None
        L.orc_iso_cpml_coeffs.argtypes = [gp, ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, dp]
        L.orc_iso_energy.restype = ctypes.c_double
        L.orc_iso_energy.argtypes = [gp, fp, dp, dp, dp, dp]
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if a is not None else None


def _f(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _i(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def _pts(p):
    p = np.ascontiguousarray(np.asarray(p, dtype=np.int32).reshape(-1, 3))
    return p


def _vel(g, vel):
    v = np.ascontiguousarray(vel, dtype=np.float64)
    assert v.shape == g.shape, (v.shape, g.shape)
    return v


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"{what} failed with oracle status {rc}")


def dt_stab(vmax, hx, hy, hz):
    return lib().orc_dt_stab(vmax, hx, hy, hz)


def ricker(f0, t0, dt, n):
    out = np.zeros(n, dtype=np.float64)
    lib().orc_ricker(f0, t0, dt, n, _d(out))
    return out


def laplacian(g: Grid, p):
    p = np.ascontiguousarray(p, dtype=np.float64)
    out = np.zeros(g.shape)
    gc = g._c()
    lib().orc_laplacian(ctypes.byref(gc), _d(p), _d(out))
    return out


def sponge_G(g: Grid, i, j, k):
    gc = g._c()
    return lib().orc_sponge_G(ctypes.byref(gc), i, j, k)


def cpml_coeffs(g: Grid, axis, k):
    gc = g._c()
    a = ctypes.c_double()
    b = ctypes.c_double()
    lib().orc_cpml_coeffs(ctypes.byref(gc), axis, k, ctypes.byref(a), ctypes.byref(b))
    return a.value, b.value


def forward(g: Grid, vel, src, wav, rec, T, p_prev=None, p_cur=None, cpml_mem=None, want_traces=True):
    """Run T steps.  Returns (traces [T][nrec], p_prev, p_cur, cpml_mem)."""
    vel = _vel(g, vel)
    src = _pts(src)
    rec = _pts(rec)
    nsrc, nrec = len(src), len(rec)
    wav = np.ascontiguousarray(np.asarray(wav, dtype=np.float64).reshape(T, nsrc)) if nsrc else np.zeros((T, 0))
    p_prev = np.zeros(g.shape) if p_prev is None else np.array(p_prev, dtype=np.float64, order="C")
    p_cur = np.zeros(g.shape) if p_cur is None else np.array(p_cur, dtype=np.float64, order="C")
    if g.bc == BC_CPML:
        cpml_mem = np.zeros((6,) + g.shape) if cpml_mem is None else np.array(cpml_mem, dtype=np.float64, order="C")
    else:
        cpml_mem = None
    traces = np.zeros((T, nrec)) if want_traces else None
    gc = g._c()
    rc = lib().orc_forward(ctypes.byref(gc), _f(vel), nsrc, _i(src), _d(wav), nrec, _i(rec), T,
                           _d(traces), _d(p_prev), _d(p_cur), _d(cpml_mem))
    _check(rc, "orc_forward")
    return traces, p_prev, p_cur, cpml_mem


def step_points(g: Grid, vel, p_prev, p_cur, cpml_mem, pts, src_term=None, window=None):
    """p^{n+1} at the points `pts` (global (i, j, k)).  With window =
    ((i0, j0, k0), (wnx, wny, wnz)) the arrays hold only that box ([wnz][wny][wnx],
    cpml_mem [6][wnz][wny][wnx])."""
    if window is None:
        vel = _vel(g, vel)
    else:
        vel = np.ascontiguousarray(vel, dtype=np.float64)
        assert vel.shape == tuple(window[1][::-1]), (vel.shape, window)
    pts = _pts(pts)
    p_prev = np.ascontiguousarray(p_prev, dtype=np.float64)
    p_cur = np.ascontiguousarray(p_cur, dtype=np.float64)
    mem = None if cpml_mem is None else np.ascontiguousarray(cpml_mem, dtype=np.float64)
    st = None if src_term is None else np.ascontiguousarray(src_term, dtype=np.float64)
    out = np.zeros(len(pts))
    gc = g._c(window)
    rc = lib().orc_step_points(ctypes.byref(gc), _f(vel), _d(p_prev), _d(p_cur), _d(mem), len(pts), _i(pts),
                               _d(st), _d(out))
    _check(rc, "orc_step_points")
    return out


def energy(g: Grid, vel, pn, pn1):
    vel = _vel(g, vel)
    gc = g._c()
    return lib().orc_energy(ctypes.byref(gc), _f(vel), _d(np.ascontiguousarray(pn, dtype=np.float64)),
                            _d(np.ascontiguousarray(pn1, dtype=np.float64)))


def adjoint(g: Grid, vel, rec, resid, T, src):
    vel = _vel(g, vel)
    rec = _pts(rec)
    src = _pts(src)
    resid = np.ascontiguousarray(np.asarray(resid, dtype=np.float64).reshape(T, len(rec)))
    adj = np.zeros((T, len(src)))
    gc = g._c()
    rc = lib().orc_adjoint(ctypes.byref(gc), _f(vel), len(rec), _i(rec), _d(resid), T, len(src), _i(src), _d(adj))
    _check(rc, "orc_adjoint")
    return adj


def gradient(g: Grid, vel, src, wav, rec, d_obs, T, ckpt=None):
    """Returns (grad [nz][ny][nx] w.r.t. m = 1/v^2, traces [T][nrec], loss)."""
    vel = _vel(g, vel)
    src = _pts(src)
    rec = _pts(rec)
    wav = np.ascontiguousarray(np.asarray(wav, dtype=np.float64).reshape(T, len(src)))
    d_obs = np.ascontiguousarray(np.asarray(d_obs, dtype=np.float64).reshape(T, len(rec)))
    grad = np.zeros(g.shape)
    traces = np.zeros((T, len(rec)))
    loss = ctypes.c_double()
    gc = g._c()
    rc = lib().orc_gradient(ctypes.byref(gc), _f(vel), len(src), _i(src), _d(wav), len(rec), _i(rec), _d(d_obs),
                            T, ckpt or T, _d(grad), _d(traces), ctypes.byref(loss))
    _check(rc, "orc_gradient")
    return grad, traces, loss.value


def num_threads():
    return lib().orc_num_threads()


def set_num_threads(n):
    lib().orc_set_num_threads(int(n))


# ------------------------------------------------------------ acoustic_iso
def iso_dt_stab(vmax, hx, hy, hz):
    """Largest stable dt of the staggered order-8 leapfrog (acoustic_iso)."""
    return lib().orc_iso_dt_stab(vmax, hx, hy, hz)


def iso_dplus(g: Grid, f, ax):
    """Staggered first difference D+ of a cell field along axis ax (0 x, 1 y,
    2 z); element (k, j, i) is the value at the face (i, j, k) + 1/2 e_ax."""
    f = _vel(g, f)
    out = np.zeros(g.shape)
    lib().orc_iso_dplus(ctypes.byref(g._c()), _d(f), ax, _d(out))
    return out


def iso_cpml_coeffs(g: Grid, axis, k, face):
    """acoustic_iso CPML (a, b) of axis `axis` at cell k (face=0) or at the
    face k + 1/2 (face=1)."""
    a = ctypes.c_double()
    b = ctypes.c_double()
    lib().orc_iso_cpml_coeffs(ctypes.byref(g._c()), axis, k, int(face), ctypes.byref(a), ctypes.byref(b))
    return a.value, b.value


def iso_forward(g: Grid, vel, rho, src, wav, rec, T, state=None):
    """acoustic_iso run of T steps.  state = [4][nz][ny][nx] (p^n, u_x, u_y,
    u_z at n-1/2; u_x[k][j][i] is the face i+1/2), and with CPML six more
    (psi_px, psi_py, psi_pz at the faces, psi_ux, psi_uy, psi_uz at the
    cells), zero if None.  Returns (traces [T][nrec], end state)."""
    vel = _vel(g, vel)
    rho = _vel(g, rho)
    src = _pts(src)
    rec = _pts(rec)
    nsrc, nrec = len(src), len(rec)
    wav = np.ascontiguousarray(np.asarray(wav, dtype=np.float64).reshape(T, nsrc)) if nsrc else np.zeros((T, 0))
    nst = 10 if g.bc == BC_CPML else 4
    st = np.zeros((nst,) + g.shape) if state is None else np.array(state, dtype=np.float64, order="C")
    assert st.shape == (nst,) + g.shape, st.shape
    traces = np.zeros((T, nrec))
    rc = lib().orc_iso_forward(ctypes.byref(g._c()), _f(vel), _d(rho), nsrc, _i(src), _d(wav), nrec, _i(rec), T,
                               _d(traces), _d(st))
    _check(rc, "orc_iso_forward")
    return traces, st


def iso_energy(g: Grid, vel, rho, p_n, p_n1, u_half):
    vel = _vel(g, vel)
    rho = _vel(g, rho)
    p_n = _vel(g, p_n)
    p_n1 = _vel(g, p_n1)
    u_half = np.ascontiguousarray(u_half, dtype=np.float64)
    return lib().orc_iso_energy(ctypes.byref(g._c()), _f(vel), _d(rho), _d(p_n), _d(p_n1), _d(u_half))
