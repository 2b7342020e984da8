"""Pins of the oracle's acoustic_iso propagator (first-order variable-density
system on a staggered grid) against what mathematics fixes: the staggered
derivative's exactness and textbook truncation constant, the stability limit,
exact discrete energy conservation, the exact evolution of a Fourier mode, and
the equivalence with a second-order scheme for constant density (an
independent numpy restatement)."""
import json
import math
import os

import numpy as np
import pytest

from oracle import c_oracle as C

GOLD = os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")
CS = np.array([1225.0 / 1024.0, -245.0 / 3072.0, 49.0 / 5120.0, -5.0 / 7168.0])


def _gold():
    with open(GOLD) as f:
        return json.load(f)


@pytest.mark.parametrize("ax", [0, 1, 2])
def test_iso_staggered_derivative_exactness_and_error_constant(ax):
    """D+ is exact on polynomials up to degree 8 at the faces and, for x^9
    centred on a face, returns the textbook constant -35/294912 * 9! h^8."""
    n = (21, 19, 23)
    h = (10.0, 7.5, 12.5)
    g = C.Grid(n[0], n[1], n[2], h[0], h[1], h[2], 1e-4)
    k, j, i = np.meshgrid(np.arange(n[2]), np.arange(n[1]), np.arange(n[0]), indexing="ij")
    pos = (i, j, k)[ax] * h[ax]
    c0 = (n[ax] // 2 + 0.5) * h[ax]  # a face in the middle
    interior = (((i, j, k)[ax] >= 4) & ((i, j, k)[ax] <= n[ax] - 5))
    for d in range(0, 9):
        f = ((pos - c0) / h[ax]) ** d
        got = C.iso_dplus(g, f, ax)
        xf = (pos + 0.5 * h[ax] - c0) / h[ax]
        want = d * xf ** max(d - 1, 0) / h[ax] if d > 0 else 0.0 * xf
        err = np.abs(got - want)[interior].max()
        assert err <= 1e-9 * max(1.0, np.abs(want[interior]).max()), (d, err)
    num, den = _gold()["staggered_order8_d1_error"]
    f = (pos - c0) ** 9
    got = C.iso_dplus(g, f, ax)
    face = ((i, j, k)[ax] == n[ax] // 2)  # the face at c0 (cell n//2 holds face n//2 + 1/2)
    want = num / den * 362880.0 * h[ax] ** 8
    assert np.allclose(got[face], want, rtol=1e-9, atol=0)


def test_iso_stability_limit():
    g = _gold()
    C8 = CS[0] - CS[1] + CS[2] - CS[3]
    assert C8 == pytest.approx(1.2863095, rel=1e-7)
    assert 1500.0 * C.iso_dt_stab(1500.0, 10.0, 10.0, 10.0) / 10.0 == pytest.approx(
        g["staggered_order8_courant_limit_equal_spacing"], rel=1e-5)


def _model(rng, shape):
    from scipy.ndimage import gaussian_filter
    v = 1800.0 + 1200.0 * rng.random(shape)
    rho = 1000.0 + 1500.0 * gaussian_filter(rng.random(shape), 1.0)
    return v, rho


def test_iso_energy_is_conserved():
    """Without sponge and source, E = sum |u^{n+1/2}|^2 / b + sum p^n p^{n+1} / K
    is constant (D- = -(D+)^T with zero ghosts), for variable v and rho."""
    rng = np.random.default_rng(70)
    shape = (14, 16, 18)
    v, rho = _model(rng, shape)
    h = (10.0, 9.0, 11.0)
    dt = 0.9 * C.iso_dt_stab(v.max(), *h)
    g = C.Grid(shape[2], shape[1], shape[0], *h, dt)
    w = rng.standard_normal((6, 2))
    src = [[9, 8, 7], [3, 12, 4]]
    _, st = C.iso_forward(g, v, rho, src, w, [[1, 1, 1]], 6)

    def energy_after(state, steps):
        _, a = C.iso_forward(g, v, rho, src, np.zeros((steps, 2)), [[1, 1, 1]], steps, state=state)
        _, b = C.iso_forward(g, v, rho, src, np.zeros((1, 2)), [[1, 1, 1]], 1, state=a)
        return C.iso_energy(g, v, rho, a[0], b[0], b[1:]), a

    e0, _ = energy_after(st, 0)
    e1, _ = energy_after(st, 300)
    assert e0 > 0 and abs(e1 - e0) <= 1e-10 * e0


@pytest.mark.parametrize("ax,kmode", [(0, 3), (2, 5)])
def test_iso_fourier_mode_evolves_exactly(ax, kmode):
    """Periodic box, constant v and rho: with p^0 = cos(k x) and u^{-1/2} =
    (dt b S / 2) sin(k (x + h/2)), S = (2/h) sum c_m sin((m - 1/2) k h), the
    scheme gives p^n = cos(n theta) cos(k x) with cos theta = 1 - dt^2 v^2 S^2 / 2."""
    n = (24, 20, 30)
    h = (10.0, 8.0, 12.0)
    v0, rho0 = 2500.0, 1800.0
    dt = 0.7 * C.iso_dt_stab(v0, *h)
    g = C.Grid(n[0], n[1], n[2], *h, dt, bc=C.BC_PERIODIC)
    shape = (n[2], n[1], n[0])
    k3, j3, i3 = np.meshgrid(np.arange(n[2]), np.arange(n[1]), np.arange(n[0]), indexing="ij")
    idx = (i3, j3, k3)[ax]
    kk = 2 * np.pi * kmode / (n[ax] * h[ax])
    x = idx * h[ax]
    S = 2.0 / h[ax] * np.sum(CS * np.sin((np.arange(1, 5) - 0.5) * kk * h[ax]))
    b = 1.0 / rho0
    st = np.zeros((4,) + shape)
    st[0] = np.cos(kk * x)
    st[1 + ax] = dt * b * S / 2 * np.sin(kk * (x + h[ax] / 2))
    T = 60
    _, out = C.iso_forward(g, np.full(shape, v0), np.full(shape, rho0), np.zeros((0, 3)), np.zeros((T, 0)),
                           [[0, 0, 0]], T, state=st)
    theta = np.arccos(1 - dt * dt * v0 * v0 * S * S / 2)
    assert np.abs(out[0] - np.cos(T * theta) * np.cos(kk * x)).max() <= 1e-11


def _dplus_np(p, ax, h):
    """Numpy restatement of the staggered forward difference with zero ghosts."""
    a = 2 - ax
    n = p.shape[a]
    pad = [(0, 0)] * 3
    pad[a] = (4, 4)
    q = np.pad(p, pad)
    out = np.zeros_like(p)
    for m in range(1, 5):
        out += CS[m - 1] / h * (np.take(q, np.arange(n) + 4 + m, axis=a) - np.take(q, np.arange(n) + 4 - (m - 1), axis=a))
    return out


def _dminus_np(u, ax, h):
    a = 2 - ax
    n = u.shape[a]
    pad = [(0, 0)] * 3
    pad[a] = (4, 4)
    q = np.pad(u, pad)
    out = np.zeros_like(u)
    for m in range(1, 5):
        out += CS[m - 1] / h * (np.take(q, np.arange(n) + 4 + m - 1, axis=a) - np.take(q, np.arange(n) + 4 - m, axis=a))
    return out


def test_iso_constant_density_equals_second_order_form():
    """For constant rho the first-order scheme is, exactly, the second-order
    leapfrog p^{n+1} - 2 p^n + p^{n-1} = dt^2 v^2 D-.(D+ p^n) + dt K (s^n - s^{n-1})
    (restated here in numpy with zero ghosts)."""
    rng = np.random.default_rng(71)
    shape = (12, 13, 15)
    h = (10.0, 11.0, 9.0)
    v = 1800.0 + 1000.0 * rng.random(shape)
    rho = np.full(shape, 1700.0)
    dt = 0.8 * C.iso_dt_stab(v.max(), *h)
    g = C.Grid(shape[2], shape[1], shape[0], *h, dt)
    T = 40
    src = np.array([[7, 6, 5]])
    w = rng.standard_normal((T, 1))
    tr, _ = C.iso_forward(g, v, rho, src, w, [[7, 6, 5]], T)
    K = rho * v * v
    b = 1.0 / rho
    pm = np.zeros(shape)
    pc = np.zeros(shape)
    s_prev = np.zeros(shape)
    out = []
    for n in range(T):
        s = np.zeros(shape)
        s[5, 6, 7] = w[n, 0] / (h[0] * h[1] * h[2])
        lap = sum(_dminus_np(_dplus_np(pc, ax, h[ax]), ax, h[ax]) for ax in range(3))
        pn = 2 * pc - pm + dt * dt * K * b * lap + dt * K * (s - s_prev)
        pm, pc, s_prev = pc, pn, s
        out.append(pc[5, 6, 7])
    assert np.abs(np.array(out) - tr[:, 0]).max() <= 1e-12 * np.abs(tr).max()


def test_iso_sponge_with_zero_strength_is_bc_none_and_sponge_absorbs():
    rng = np.random.default_rng(72)
    shape = (16, 17, 18)
    v, rho = _model(rng, shape)
    h = (10.0, 10.0, 10.0)
    dt = 0.6 * C.iso_dt_stab(v.max(), *h)
    T = 120
    w = C.ricker(40.0, 0.03, dt, T)[:, None]
    src, rec = [[9, 8, 8]], [[2, 2, 2], [15, 14, 13]]
    g0 = C.Grid(shape[2], shape[1], shape[0], *h, dt)
    gs0 = C.Grid(shape[2], shape[1], shape[0], *h, dt, bc=C.BC_SPONGE, nb=4, sigma=0.0)
    a, sa = C.iso_forward(g0, v, rho, src, w, rec, T)
    b, sb = C.iso_forward(gs0, v, rho, src, w, rec, T)
    assert np.array_equal(a, b) and np.array_equal(sa, sb)
    gs = C.Grid(shape[2], shape[1], shape[0], *h, dt, bc=C.BC_SPONGE, nb=4, sigma=0.1)
    wl = np.concatenate([w, np.zeros((300, 1))])
    _, sc = C.iso_forward(gs, v, rho, src, wl, rec, T + 300)
    _, sd = C.iso_forward(g0, v, rho, src, wl, rec, T + 300)
    assert np.abs(sc[0]).max() < 0.2 * np.abs(sd[0]).max()


def test_iso_cpml_with_no_damping_is_bc_none():
    """CPML with R = 1 (d0 = 0) and f0 = 0 (alpha = 0) has a = 0, b = 1: the
    memory variables stay zero and the run equals bc none bitwise (pressure,
    velocities, traces), with and without a free surface."""
    rng = np.random.default_rng(81)
    shape = (15, 16, 17)
    v, rho = _model(rng, shape)
    h = (10.0, 11.0, 9.0)
    dt = 0.5 * C.iso_dt_stab(v.max(), *h)
    T = 50
    w = rng.standard_normal((T, 2))
    src, rec = [[8, 7, 6], [2, 3, 1]], [[1, 1, 1], [15, 14, 13], [8, 8, 0]]
    for fs in (0, 1):
        g0 = C.Grid(shape[2], shape[1], shape[0], *h, dt, fs=fs)
        gc = C.Grid(shape[2], shape[1], shape[0], *h, dt, bc=C.BC_CPML, nb=4, R=1.0, f0=0.0, vmax=v.max(), fs=fs)
        a, sa = C.iso_forward(g0, v, rho, src, w, rec, T)
        b, sb = C.iso_forward(gc, v, rho, src, w, rec, T)
        assert np.array_equal(a, b) and np.array_equal(sa, sb[:4])
        assert not np.any(sb[4:])


def _iso_reflection(bc, nb):
    """Largest difference, at receivers inside the undamped core, between a
    40^3 run with the given boundary and a run on a 100^3 grid whose own
    boundary is too far to be seen in the window, relative to the peak of
    the direct wave there (constant v and rho)."""
    n_small, margin = 40, 30
    hh = 10.0
    c = 2000.0
    f0 = 25.0
    dt = 0.5 * C.iso_dt_stab(c, hh, hh, hh)
    T = int(0.3 / dt)  # 0.3 s: the reflection from the 40^3 boundary arrives, not the one from the 100^3 boundary
    w = C.ricker(f0, 1.5 / f0, dt, T)[:, None]
    ctr = n_small // 2
    off = [(6, 0, 0), (0, -6, 0), (0, 0, 6), (4, 4, 4), (-5, 3, 0)]
    rec = [[ctr + a, ctr + b, ctr + c_] for a, b, c_ in off]
    g = C.Grid(n_small, n_small, n_small, hh, hh, hh, dt, bc=bc, nb=nb, R=1e-3, f0=f0, vmax=c)
    shp = g.shape
    small, _ = C.iso_forward(g, np.full(shp, c), np.full(shp, 1500.0), [[ctr] * 3], w, rec, T)
    nbig = n_small + 2 * margin
    gb = C.Grid(nbig, nbig, nbig, hh, hh, hh, dt)
    rec_b = [[x + margin for x in r] for r in rec]
    big, _ = C.iso_forward(gb, np.full(gb.shape, c), np.full(gb.shape, 1500.0), [[ctr + margin] * 3], w, rec_b, T)
    return np.abs(small - big).max() / np.abs(big).max()


@pytest.mark.slow
def test_iso_cpml_absorbs():
    """CPML leaves a reflection far below that of the zero-ghost boundary, and
    a wider layer absorbs better (as for the constant-density propagator)."""
    r_none = _iso_reflection(C.BC_NONE, 10)
    r10 = _iso_reflection(C.BC_CPML, 10)
    r5 = _iso_reflection(C.BC_CPML, 5)
    assert r_none > 0.05, r_none
    assert r10 < 2e-2 and r10 < 0.1 * r_none, (r10, r_none)
    assert r10 < r5, (r10, r5)


@pytest.mark.parametrize("nb,h,vmax,R", [(20, 10.0, 4500.0, 1e-3), (32, 12.5, 5000.0, 1e-4)])
def test_iso_cpml_profiles_match_pml_reflection_theory(nb, h, vmax, R):
    """The damping d recovered from (a, b) at the cells and at the faces (b =
    exp(-(d + alpha) dt), a / (b - 1) = d / (d + alpha)) against PML theory:
    R = exp(-(2 / c) * integral of d over the layer), so the layer sums of
    d h over the cells (depths 1 .. nb) and over the faces (depths 1/2 ..
    nb - 1/2) must give ln R within the quadrature errors of a quadratic
    profile sampled at those points: the cell sum overshoots the integral by
    (1 + 3/(2 nb) + 1/(2 nb^2)), the face (midpoint) sum undershoots it by
    (1 - 1/(4 nb^2)).  alpha is pi f0 at the interface falling linearly to 0
    at the outer edge, both ends agree at the same depth, the face beyond the
    last cell takes the outermost value, and outside the layers a = 0, b = 1."""
    f0 = 17.0
    n = 2 * nb + 11
    dt = 1e-4
    hs = (h, 0.8 * h, 1.3 * h)
    g = C.Grid(n, n + 1, n + 2, hs[0], hs[1], hs[2], dt, bc=C.BC_CPML, nb=nb, R=R, f0=f0, vmax=vmax)

    def d_alpha(ab):
        a, b = ab
        sgm = -math.log(b) / dt
        d = a / (b - 1.0) * sgm
        return d, sgm - d

    for ax in range(3):
        na = (n, n + 1, n + 2)[ax]
        sums = []
        for face in (0, 1):
            tot = 0.0
            for j in range(1, nb + 1):
                # depth j (cells) or j - 1/2 (faces): index nb - j from the low end
                lo = C.iso_cpml_coeffs(g, ax, nb - j, face)
                hi = C.iso_cpml_coeffs(g, ax, na - 1 - (nb - j) - face, face)
                assert lo == pytest.approx(hi, rel=1e-12, abs=1e-15)
                d, alpha = d_alpha(lo)
                q = (j - 0.5 * face) / nb
                assert alpha == pytest.approx(math.pi * f0 * (1.0 - q), rel=1e-9, abs=1e-9)
                tot += d * hs[ax]
            sums.append((-2.0 / vmax * tot) / math.log(R))
            assert C.iso_cpml_coeffs(g, ax, nb + face * 0, 0) == (0.0, 1.0)
        assert sums[0] == pytest.approx((nb + 1) * (2 * nb + 1) / (2.0 * nb * nb), rel=1e-9), (ax, sums)
        assert sums[1] == pytest.approx(1.0 - 1.0 / (4.0 * nb * nb), rel=1e-9), (ax, sums)
        # the face beyond the last cell and the last cell carry the outermost coefficients
        assert C.iso_cpml_coeffs(g, ax, na - 1, 1) == pytest.approx(C.iso_cpml_coeffs(g, ax, na - 1, 0), rel=1e-12)
        # the faces just inside the layers: depth 1/2
        assert C.iso_cpml_coeffs(g, ax, nb, 1) == (0.0, 1.0)
        assert C.iso_cpml_coeffs(g, ax, nb - 1, 1) != (0.0, 1.0)
        assert C.iso_cpml_coeffs(g, ax, na - 1 - nb, 1) != (0.0, 1.0)
        assert C.iso_cpml_coeffs(g, ax, na - 2 - nb, 1) == (0.0, 1.0)


def _mirror_z(a, nz):
    """[nz] planes k = 0.. -> [2 nz - 1] planes, k mirrored about the first."""
    return np.concatenate([a[:0:-1], a], axis=0)


def test_iso_free_surface_equals_the_mirrored_problem():
    """A free surface at k = 0 is the symmetry plane of a grid twice as deep
    with the model mirrored and an image source of opposite sign (ordinary
    zero ghosts there): the run with the surface must equal the lower half of
    that run, pressure, all three velocities and the traces, and p = 0 on
    the surface plane.  Sources sit below and on the surface (the latter
    injects nothing), receivers too.  The staggered grid is not symmetric at
    its far z ends (the last face is stored, the one before the first is
    not), so the grid is deep enough that no wave reaches them in T steps."""
    rng = np.random.default_rng(72)
    shape = (40, 12, 13)
    nz, ny, nx = shape
    v, rho = _model(rng, shape)
    h = (10.0, 9.0, 11.0)
    dt = 0.8 * C.iso_dt_stab(v.max(), *h)
    T = 45
    src = [[6, 5, 3], [2, 9, 0], [9, 3, 6]]
    rec = [[4, 4, 0], [6, 5, 1], [1, 10, 5], [12, 0, 10]]
    w = rng.standard_normal((T, len(src)))
    g = C.Grid(nx, ny, nz, *h, dt, fs=1)
    tr, st = C.iso_forward(g, v, rho, src, w, rec, T)
    K0 = nz - 1
    gm = C.Grid(nx, ny, 2 * nz - 1, *h, dt)
    src_m = [[i, j, K0 + k] for i, j, k in src] + [[i, j, K0 - k] for i, j, k in src]
    w_m = np.concatenate([w, -w], axis=1)
    rec_m = [[i, j, K0 + k] for i, j, k in rec]
    trm, stm = C.iso_forward(gm, _mirror_z(v, nz), _mirror_z(rho, nz), src_m, w_m, rec_m, T)
    scale = np.abs(stm).max()
    assert scale > 0
    assert np.abs(st[0][0]).max() == 0.0
    for a in range(4):
        assert np.abs(st[a] - stm[a][K0:]).max() <= 1e-12 * scale, a
    assert np.abs(tr - trm).max() <= 1e-12 * np.abs(trm).max()
    # the velocities of the mirrored run are symmetric in the way the surface assumes:
    # u_z even about the plane (face -1/2 - m mirrors face m + 1/2), p odd
    assert np.abs(stm[0][K0 - 3:K0] + stm[0][K0 + 3:K0:-1]).max() <= 1e-12 * scale
    assert np.abs(stm[3][K0 - 3:K0] - stm[3][K0 + 2:K0 - 1:-1]).max() <= 1e-12 * scale


def test_iso_free_surface_conserves_energy_and_works_with_the_sponge():
    rng = np.random.default_rng(73)
    shape = (13, 14, 12)
    v, rho = _model(rng, shape)
    h = (10.0, 11.0, 9.0)
    dt = 0.9 * C.iso_dt_stab(v.max(), *h)
    g = C.Grid(shape[2], shape[1], shape[0], *h, dt, fs=1)
    src = [[6, 7, 4]]
    _, st = C.iso_forward(g, v, rho, src, rng.standard_normal((5, 1)), [[1, 1, 1]], 5)

    def energy(state):
        _, b = C.iso_forward(g, v, rho, src, np.zeros((1, 1)), [[1, 1, 1]], 1, state=state)
        return C.iso_energy(g, v, rho, state[0], b[0], b[1:])

    _, later = C.iso_forward(g, v, rho, src, np.zeros((250, 1)), [[1, 1, 1]], 250, state=st)
    e0, e1 = energy(st), energy(later)
    assert e0 > 0 and abs(e1 - e0) <= 1e-10 * e0
    # with a sponge on the other five faces the field decays and the surface stays at zero
    gs = C.Grid(shape[2], shape[1], shape[0], *h, dt, bc=C.BC_SPONGE, nb=3, sigma=0.2, fs=1)
    _, s1 = C.iso_forward(gs, v, rho, src, rng.standard_normal((5, 1)), [[1, 1, 1]], 5)
    _, s2 = C.iso_forward(gs, v, rho, src, np.zeros((400, 1)), [[1, 1, 1]], 400, state=s1)
    assert np.abs(s2[0][0]).max() == 0.0
    assert np.abs(s2[0]).max() < 0.2 * np.abs(s1[0]).max()


def test_iso_density_contrast_reflects_with_the_impedance_ratio():
    """A plane wave at normal incidence on a density step (same velocity)
    reflects with R = (Z2 - Z1) / (Z2 + Z1), Z = rho v: here rho triples, R = 1/2.
    Periodic 4 x 4 x 700 column, plane source at k = 150, step at k = 300,
    receiver at k = 200; the direct and reflected peaks are compared before
    any wrapped arrival."""
    nx, ny, nz = 4, 4, 700
    h = 10.0
    v0 = 2000.0
    shape = (nz, ny, nx)
    v = np.full(shape, v0)
    rho = np.full(shape, 1000.0)
    rho[300:] = 3000.0
    dt = 0.5 * C.iso_dt_stab(v0, h, h, h)
    g = C.Grid(nx, ny, nz, h, h, h, dt, bc=C.BC_PERIODIC)
    t_end = 2.0
    T = int(t_end / dt)
    f0 = 8.0
    w = C.ricker(f0, 1.5 / f0, dt, T)
    src = np.array([[i, j, 150] for i in range(nx) for j in range(ny)])
    tr, _ = C.iso_forward(g, v, rho, src, np.repeat(w[:, None], len(src), axis=1), [[1, 1, 200]], T)
    t = (np.arange(T) + 1) * dt
    t_direct = 1.5 / f0 + 50 * h / v0
    t_refl = 1.5 / f0 + 250 * h / v0
    win = 0.08
    a_dir = np.abs(tr[np.abs(t - t_direct) < win, 0]).max()
    a_ref = np.abs(tr[np.abs(t - t_refl) < win, 0]).max()
    assert a_ref / a_dir == pytest.approx(0.5, rel=0.03), a_ref / a_dir


def _peak_time(tr, dt):
    """Time of the largest sample of a trace, refined by the parabola through
    it and its two neighbours (traces[n] holds time (n + 1) dt)."""
    n = int(np.argmax(tr))
    y0, y1, y2 = tr[n - 1], tr[n], tr[n + 1]
    off = 0.5 * (y0 - y2) / (y0 - 2.0 * y1 + y2)
    return (n + 1 + off) * dt


@pytest.mark.parametrize("ax", [0, 1, 2])
@pytest.mark.parametrize("rho_pair", [(1000.0, 3000.0), (1500.0, 2500.0)])
def test_iso_long_wave_speed_across_thin_layers_is_the_homogenised_speed(ax, rho_pair):
    """Layers one cell thick normal to the propagation axis: constant bulk
    modulus K, density alternating cell by cell.  A wave much longer than the
    layering travels at the speed of the homogenised medium,
    c = 1 / sqrt(<rho> <1/K>) (effective density = arithmetic mean of rho
    along the path, effective compliance = mean of 1/K), here
    sqrt(K / <rho>) = 2000 m/s for both density pairs; a face buoyancy that
    averages 1/rho instead gives sqrt(K <1/rho>) = 2309 m/s for 1000/3000.
    Periodic 4 x 4 x 400 column, plane source, 4 Hz Ricker (wavelength 50
    cells), speed from the peak times at 20 and 100 cells from the source."""
    n_long, h, K, f0 = 400, 10.0, 8.0e9, 4.0
    shape_xyz = [4, 4, 4]
    shape_xyz[ax] = n_long
    nx, ny, nz = shape_xyz
    pos = np.arange(n_long)
    rho_line = np.where(pos % 2 == 0, rho_pair[0], rho_pair[1])
    sh = [1, 1, 1]
    sh[2 - ax] = n_long
    rho = np.broadcast_to(rho_line.reshape(sh), (nz, ny, nx)).copy()
    v = np.sqrt(K / rho)
    dt = 0.5 * C.iso_dt_stab(v.max(), h, h, h)
    g = C.Grid(nx, ny, nz, h, h, h, dt, bc=C.BC_PERIODIC)
    T = int(1.1 / dt)  # the far peak arrives at 1.5 / f0 + 1000 m / c = 0.875 s
    w = C.ricker(f0, 1.5 / f0, dt, T)

    def pt(a, b, c_long):
        q = [a, b]
        q.insert(ax, c_long)
        return q

    src = np.array([pt(a, b, 100) for a in range(4) for b in range(4)])
    rec = np.array([pt(1, 2, 120), pt(1, 2, 200)])
    tr, _ = C.iso_forward(g, v.astype(np.float32).astype(np.float64), rho, src,
                          np.repeat(w[:, None], len(src), axis=1), rec, T)
    c = 80 * h / (_peak_time(tr[:, 1], dt) - _peak_time(tr[:, 0], dt))
    c_hom = 1.0 / np.sqrt(rho_line.mean() * np.mean(1.0 / np.full(n_long, K)))
    assert c == pytest.approx(c_hom, rel=5e-3), (c, c_hom)
