"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these compares the oracle with itself: each checks a closed form, an
invariant, a special case, a textbook error constant, or agreement with the
independent numpy implementation (oracle/tiny.py).  A plausible slip in the
oracle (a wrong weight, a dropped term, a swapped axis, a sign, an
off-by-one in the time index) fails at least one of them.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import c_oracle as C
from oracle import tiny as TN

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


# --------------------------------------------------------------------- P1
def _coords(n, h):
    return (np.arange(n) - (n - 1) / 2.0) * h


@pytest.mark.parametrize("ex", [(0, 0, 0), (2, 0, 0), (0, 2, 0), (0, 0, 2), (4, 0, 0), (0, 6, 0), (0, 0, 8),
                                (9, 0, 0), (0, 9, 0), (0, 0, 9), (3, 5, 7), (9, 9, 9), (8, 2, 5)])
def test_p1_polynomial_exactness(ex):
    """Order-8 central weights differentiate every polynomial of degree <= 9
    per axis exactly (section "Finite Differences": Taylor coefficients of
    order 8).  Unequal spacings catch a swapped axis."""
    nx, ny, nz = 13, 12, 11
    hx, hy, hz = 0.21, 0.17, 0.23
    x = _coords(nx, hx)[None, None, :]
    y = _coords(ny, hy)[None, :, None]
    z = _coords(nz, hz)[:, None, None]
    a, b, c = ex
    p = x ** a * y ** b * z ** c
    exact = np.zeros_like(p)
    if a >= 2:
        exact = exact + a * (a - 1) * x ** (a - 2) * y ** b * z ** c
    if b >= 2:
        exact = exact + b * (b - 1) * x ** a * y ** (b - 2) * z ** c
    if c >= 2:
        exact = exact + c * (c - 1) * x ** a * y ** b * z ** (c - 2)
    g = C.Grid(nx, ny, nz, hx, hy, hz, 1.0)
    L = C.laplacian(g, p)
    sl = (slice(4, nz - 4), slice(4, ny - 4), slice(4, nx - 4))
    scale = np.abs(p).max() / min(hx, hy, hz) ** 2 + 1.0
    assert np.abs(L[sl] - exact[sl]).max() <= 1e-12 * scale


def test_p1_degree10_truncation_constant():
    """For degree 10 the order-8 second difference errs by the textbook
    truncation term -h^8 f^(10)/3150 = -1152 h^8 at x = 0 for f = x^10 (the
    leading error of the 8th-order central formula), on each axis with its
    own spacing."""
    gold = _gold("closed_forms.json")
    n = 9
    for axis, h in ((0, 0.5), (1, 0.7), (2, 0.9)):
        hs = [1.0, 1.0, 1.0]
        hs[axis] = h
        g = C.Grid(n, n, n, hs[0], hs[1], hs[2], 1.0)
        coord = _coords(n, h)
        shape = [1, 1, 1]
        shape[2 - axis] = n
        p = np.broadcast_to((coord ** 10).reshape(shape), (n, n, n)).copy()
        L = C.laplacian(g, p)
        want = -math.factorial(10) / gold["order8_d2_error_denominator"] * h ** 8
        assert abs(L[4, 4, 4] - want) <= 1e-9 * abs(want)


# --------------------------------------------------------------------- P2
def test_p2_periodic_fourier_mode():
    """On a periodic box with constant v, a Fourier mode started with
    p^{-1} = cos(theta) p^0 evolves as cos(n theta) exactly, with
    cos(theta) = 1 - dt^2 v^2/2 * sum_axes S(k h)/h^2 and
    S(phi) = 2 sum_m a_m (1 - cos m phi) (von Neumann symbol of the
    25-point stencil)."""
    nx, ny, nz = 16, 12, 10
    h = (10.0, 12.0, 9.0)
    v = 2000.0
    dt = 0.7 * C.dt_stab(v, *h)
    kx, ky, kz = 2 * np.pi * 3 / (nx * h[0]), 2 * np.pi * 2 / (ny * h[1]), 2 * np.pi * 1 / (nz * h[2])
    a = [8 / 5, -1 / 5, 8 / 315, -1 / 560]

    def S(phi):
        return sum(2 * a[m - 1] * (1 - math.cos(m * phi)) for m in range(1, 5))

    lam = sum(S(k * hh) / hh ** 2 for k, hh in ((kx, h[0]), (ky, h[1]), (kz, h[2])))
    cos_t = 1 - 0.5 * dt * dt * v * v * lam
    theta = math.acos(cos_t)
    X = np.arange(nx)[None, None, :] * h[0]
    Y = np.arange(ny)[None, :, None] * h[1]
    Z = np.arange(nz)[:, None, None] * h[2]
    mode = np.cos(kx * X + ky * Y + kz * Z) * np.ones((nz, ny, nx))
    g = C.Grid(nx, ny, nz, *h, dt, bc=C.BC_PERIODIC)
    T = 60
    _, pm, pc, _ = C.forward(g, np.full(g.shape, v), [], np.zeros((T, 0)), [], T, p_prev=cos_t * mode, p_cur=mode)
    assert np.abs(pc - math.cos(T * theta) * mode).max() < 1e-11
    assert np.abs(pm - math.cos((T - 1) * theta) * mode).max() < 1e-11


# --------------------------------------------------------------------- P3
@pytest.mark.parametrize("cfl", [0.5, 0.99, 1.0, 1.01])
def test_p3_checkerboard_cfl(cfl):
    """The checkerboard (-1)^(i+j+k) on an even periodic box is the fastest
    mode; with dt = cfl * dt_stab its symbol is mu = 4 cfl^2 and the leapfrog
    gives the Chebyshev recurrence p^{n+1} = (2 - mu) p^n - p^{n-1}: bounded
    for cfl < 1, linear growth at 1, exponential growth (x1.33/step) at 1.01."""
    n = 8
    h = (10.0, 7.0, 13.0)
    v = 3000.0
    dt = cfl * C.dt_stab(v, *h)
    i = np.arange(n)
    cb = ((-1.0) ** (i[:, None, None] + i[None, :, None] + i[None, None, :]))
    g = C.Grid(n, n, n, *h, dt, bc=C.BC_PERIODIC)
    T = 50
    _, _, pc, _ = C.forward(g, np.full(g.shape, v), [], np.zeros((T, 0)), [], T, p_prev=cb, p_cur=cb)
    mu = 4 * cfl * cfl
    a0, a1 = 1.0, 1.0
    for _ in range(T):
        a0, a1 = a1, (2 - mu) * a1 - a0
    assert np.abs(pc - a1 * cb).max() <= 1e-9 * max(1.0, abs(a1))
    if cfl < 1:
        assert abs(a1) <= 1.0 / math.sqrt(1 - cfl * cfl) + 1e-9
    if cfl > 1:
        assert abs(a1) > 1e5


def test_dt_stab_equal_spacing_courant_limit():
    """For equal spacing the stability limit is v dt / h = 2/sqrt(3 S),
    S = 4 (a1 + a3) = 6.5015873 -> 0.45286 (closed form of P3)."""
    gold = _gold("closed_forms.json")
    assert abs(C.dt_stab(1.0, 1.0, 1.0, 1.0) - gold["courant_limit_equal_spacing"]) < 5e-6


# --------------------------------------------------------------------- P4
@pytest.mark.parametrize("bc", [C.BC_NONE, C.BC_PERIODIC])
def test_p4_discrete_energy_conserved(bc):
    """E^{n+1/2} = sum (p^{n+1}-p^n)^2/(v^2 dt^2) - sum p^{n+1} L p^n is
    exactly conserved by the leapfrog for symmetric L (zero ghosts or
    periodic) and any v(x); it is positive for cfl <= 1."""
    rng = np.random.default_rng(11)
    nx, ny, nz = 18, 16, 14
    h = (10.0, 11.0, 9.0)
    vel = rng.uniform(1500, 4000, (nz, ny, nx))
    dt = 0.9 * C.dt_stab(vel.max(), *h)
    g = C.Grid(nx, ny, nz, *h, dt, bc=bc)
    pm = rng.standard_normal(g.shape)
    pc = rng.standard_normal(g.shape)
    E0 = C.energy(g, vel, pm, pc)
    assert E0 > 0
    Es = []
    for _ in range(10):
        _, pm, pc, _ = C.forward(g, vel, [], np.zeros((30, 0)), [], 30, p_prev=pm, p_cur=pc)
        Es.append(C.energy(g, vel, pm, pc))
    assert max(abs(E - E0) for E in Es) <= 1e-11 * E0


def test_p4_energy_nonincreasing_with_sponge_after_source():
    """With the sponge on, energy radiated by a source only decays once the
    source has stopped (absorbing layer), while bc none conserves it."""
    nx = ny = nz = 40
    h = (10.0,) * 3
    vel = np.full((nz, ny, nx), 2000.0)
    dt = 0.5 * C.dt_stab(2000.0, *h)
    T0 = 120
    f0 = 15.0
    wav = C.ricker(f0, 1.5 / f0, dt, T0)[:, None]
    wav[int(3.0 / f0 / dt):] = 0.0
    res = {}
    for bc in (C.BC_NONE, C.BC_SPONGE):
        g = C.Grid(nx, ny, nz, *h, dt, bc=bc, nb=10, sigma=0.05)
        _, pm, pc, _ = C.forward(g, vel, [[20, 20, 20]], wav, [], T0)
        E = [C.energy(g, vel, pm, pc)]
        for _ in range(6):
            _, pm, pc, _ = C.forward(g, vel, [], np.zeros((40, 0)), [], 40, p_prev=pm, p_cur=pc)
            E.append(C.energy(g, vel, pm, pc))
        res[bc] = E
    En = res[C.BC_NONE]
    assert max(abs(e - En[0]) for e in En) <= 1e-10 * En[0]
    Es = res[C.BC_SPONGE]
    assert Es[-1] < 0.2 * Es[0]


# --------------------------------------------------------------------- P5
@pytest.mark.slow
def test_p5_analytic_point_source():
    """Constant v: the discrete solution with the source scaled by
    dt^2 v^2/(hx hy hz) approaches the continuum Green's function solution
    w(t - r/c)/(4 pi r) of Eq. (acoustic_iso_cd); the error is small at
    >= 10 points per wavelength and falls at second order in dt."""
    n = 121
    hh = 10.0
    c = 2000.0
    f0 = 12.0
    t0 = 1.5 / f0
    vel = np.full((n, n, n), c)
    ctr = n // 2
    r_cells = (16, 24)
    rec = [[ctr + r, ctr, ctr] for r in r_cells]
    errs = []
    for cfl in (0.5, 0.25):
        dt = cfl * C.dt_stab(c, hh, hh, hh)
        # stop before the first boundary reflection reaches the far receiver
        t_end = t0 + 1.0 / f0 + (2 * (ctr - 1) - r_cells[-1]) * hh / c * 0.0 + (ctr - r_cells[-1]) * hh / c
        T = int(min(t_end, (2 * ctr - r_cells[-1] - 8) * hh / c) / dt)
        wav = C.ricker(f0, t0, dt, T)[:, None]
        g = C.Grid(n, n, n, hh, hh, hh, dt, bc=C.BC_NONE)
        tr, _, _, _ = C.forward(g, vel, [[ctr, ctr, ctr]], wav, rec, T)
        t = (np.arange(T) + 1) * dt  # traces[n] holds p^{n+1}
        e = []
        for q, r in enumerate(r_cells):
            R = r * hh
            ana = C.ricker(f0, t0 + R / c, dt, T + 1)[1:] / (4 * np.pi * R)
            assert np.allclose(t, (np.arange(1, T + 1)) * dt)
            e.append(np.linalg.norm(tr[:, q] - ana) / np.linalg.norm(ana))
        errs.append(e)
    assert max(errs[0]) < 2e-2, errs
    assert max(errs[1]) < max(errs[0]) / 2.5, errs


def test_p5_source_time_index_and_scaling_first_steps():
    """The first nonzero sample: with p^{-1} = p^0 = 0 and one source, p^1 at
    the source cell is D w_0 / (hx hy hz) exactly (Eq. (minimod-semidisc):
    f^n enters p^{n+1} through dt^2 v^2), and nothing reaches a neighbour
    before step 2."""
    nx, ny, nz = 12, 11, 10
    h = (10.0, 12.0, 8.0)
    vel = np.full((nz, ny, nx), 1800.0)
    dt = 1e-3
    g = C.Grid(nx, ny, nz, *h, dt)
    w = np.array([[0.7], [0.0], [0.0]])
    tr, _, _, _ = C.forward(g, vel, [[5, 5, 5]], w, [[5, 5, 5], [6, 5, 5]], 3)
    D = (dt * 1800.0) ** 2
    assert tr[0, 0] == pytest.approx(D * 0.7 / (h[0] * h[1] * h[2]), rel=1e-14)
    assert tr[0, 1] == 0.0
    assert tr[1, 1] != 0.0


# --------------------------------------------------------------------- P6
@pytest.mark.parametrize("bc", [C.BC_NONE, C.BC_SPONGE])
def test_p6_reciprocity(bc):
    """Source at A / receiver at B equals source at B / receiver at A for any
    v(x) when bc is none or the sponge: the propagator including the
    dt^2 v^2 source scaling is a symmetric operator."""
    rng = np.random.default_rng(5)
    nx, ny, nz = 22, 20, 18
    h = (10.0, 11.0, 12.0)
    vel = rng.uniform(1500, 3500, (nz, ny, nx))
    dt = 0.5 * C.dt_stab(vel.max(), *h)
    g = C.Grid(nx, ny, nz, *h, dt, bc=bc, nb=5, sigma=0.06)
    T = 80
    w = C.ricker(25.0, 0.06, dt, T)[:, None]
    A, B = [4, 6, 5], [15, 12, 11]
    tab, _, _, _ = C.forward(g, vel, [A], w, [B], T)
    tba, _, _, _ = C.forward(g, vel, [B], w, [A], T)
    assert np.abs(tab).max() > 0
    assert np.abs(tab - tba).max() <= 1e-12 * np.abs(tab).max()


# --------------------------------------------------------------------- P7
def test_p7_special_cases_reduce_to_none():
    """CPML with d = alpha = 0 (R = 1, f0 = 0) and the sponge with sigma = 0
    reproduce bc none exactly."""
    rng = np.random.default_rng(7)
    nx, ny, nz = 20, 19, 18
    h = (10.0, 10.0, 10.0)
    vel = rng.uniform(1500, 3000, (nz, ny, nx))
    dt = 0.5 * C.dt_stab(vel.max(), *h)
    T = 40
    w = rng.standard_normal((T, 1))
    src, rec = [[9, 9, 9]], [[2, 3, 4], [17, 16, 15], [0, 0, 0]]
    base = C.forward(C.Grid(nx, ny, nz, *h, dt), vel, src, w, rec, T)
    cp = C.forward(C.Grid(nx, ny, nz, *h, dt, bc=C.BC_CPML, nb=6, R=1.0, f0=0.0, vmax=vel.max()), vel, src, w, rec, T)
    sp = C.forward(C.Grid(nx, ny, nz, *h, dt, bc=C.BC_SPONGE, nb=6, sigma=0.0), vel, src, w, rec, T)
    for other in (cp, sp):
        assert np.array_equal(base[0], other[0])
        assert np.array_equal(base[2], other[2])


# --------------------------------------------------------------------- P8
def _reflection(bc, nb):
    """Largest difference, at receivers inside the undamped core, between a
    40^3 run with the given boundary and a run on a 100^3 grid whose own
    boundary is too far to be seen within the window, relative to the peak
    of the direct wave there."""
    n_small, margin = 40, 30
    hh = 10.0
    c = 2000.0
    f0 = 25.0
    dt = 0.5 * C.dt_stab(c, hh, hh, hh)
    T = 265
    w = C.ricker(f0, 1.5 / f0, dt, T)[:, None]
    ctr = n_small // 2
    off = [(6, 0, 0), (0, -6, 0), (0, 0, 6), (4, 4, 4), (-5, 3, 0)]
    rec = [[ctr + a, ctr + b, ctr + c_] for a, b, c_ in off]
    g = C.Grid(n_small, n_small, n_small, hh, hh, hh, dt, bc=bc, nb=nb, R=1e-3, f0=f0, vmax=c, sigma=0.04)
    small, _, _, _ = C.forward(g, np.full(g.shape, c), [[ctr] * 3], w, rec, T)
    nbig = n_small + 2 * margin
    gb = C.Grid(nbig, nbig, nbig, hh, hh, hh, dt, bc=C.BC_NONE)
    rec_b = [[x + margin for x in r] for r in rec]
    big, _, _, _ = C.forward(gb, np.full(gb.shape, c), [[ctr + margin] * 3], w, rec_b, T)
    return np.abs(small - big).max() / np.abs(big).max()


@pytest.mark.slow
def test_p8_cpml_absorbs():
    """CPML (the boundary the paper says every propagator uses) leaves a
    reflection far below that of the rigid zero-ghost boundary; a wider layer
    absorbs better.  The coefficient values themselves are pinned by
    test_cpml_profile_matches_pml_reflection_theory."""
    r_none = _reflection(C.BC_NONE, 10)
    r_cpml10 = _reflection(C.BC_CPML, 10)
    r_cpml5 = _reflection(C.BC_CPML, 5)
    assert r_none > 0.05, r_none
    assert r_cpml10 < 2e-2 and r_cpml10 < 0.1 * r_none, (r_cpml10, r_none)
    assert r_cpml10 < r_cpml5, (r_cpml10, r_cpml5)


@pytest.mark.parametrize("nb,h,vmax,R", [(20, 10.0, 4500.0, 1e-3), (32, 12.5, 5000.0, 1e-4), (300, 5.0, 2000.0, 1e-2)])
def test_cpml_profile_matches_pml_reflection_theory(nb, h, vmax, R):
    """Recover the damping d and the frequency shift alpha from the oracle's
    recursive-convolution coefficients (b = exp(-(d + alpha) dt) fixes
    d + alpha, a / (b - 1) = d / (d + alpha) fixes the split), then check them
    against PML theory rather than against their own formula: a layer with
    damping d(x) reflects a normally incident wave with
    R = exp(-(2 / c) * integral of d over the layer), so the layer sum of
    d h must give ln R up to its O(1/nb) quadrature error (a quadratic profile
    sampled at the cells: the exponent is (1 + 3/(2 nb) + 1/(2 nb^2)) times
    the continuous one).  alpha follows the standard CFS profile: pi f0 at
    the interface, falling linearly to 0 at the outer edge.  Both ends of each
    axis carry the same values at the same depth, each with its own spacing."""
    f0 = 17.0
    n = 2 * nb + 11
    dt = 1e-4
    hs = (h, 0.8 * h, 1.3 * h)
    g = C.Grid(n, n + 1, n + 2, hs[0], hs[1], hs[2], dt, bc=C.BC_CPML, nb=nb, R=R, f0=f0, vmax=vmax)
    for ax in range(3):
        na = (n, n + 1, n + 2)[ax]
        d_sum = 0.0
        for j in range(1, nb + 1):  # depth j: cell nb - j from the low end, its mirror at the high end
            lo = C.cpml_coeffs(g, ax, nb - j)
            hi = C.cpml_coeffs(g, ax, na - 1 - (nb - j))
            assert lo == hi
            a, b = lo
            s = -math.log(b) / dt
            d = a / (b - 1.0) * s
            alpha = s - d
            q = j / nb
            assert alpha == pytest.approx(math.pi * f0 * (1.0 - q), rel=1e-9, abs=1e-9)
            d_sum += d * hs[ax]
        ratio = (-2.0 / vmax * d_sum) / math.log(R)
        want = (nb + 1) * (2 * nb + 1) / (2.0 * nb * nb)
        assert ratio == pytest.approx(want, rel=1e-9), (ax, ratio, want)
        assert 1.0 < ratio < 1.0 + 2.0 / nb
        # outside the layers the memory is switched off
        assert C.cpml_coeffs(g, ax, nb) == (0.0, 1.0)


def test_cpml_mirror_and_axis_symmetry():
    """Constant v, centred source, cubic grid with equal spacing: the CPML
    wavefield is symmetric under each mirror and under every exchange of
    axes (a swapped or misplaced index in one axis breaks it)."""
    n = 25
    hh = 10.0
    dt = 0.5 * C.dt_stab(2500.0, hh, hh, hh)
    T = 60
    w = C.ricker(30.0, 0.05, dt, T)[:, None]
    for bc in (C.BC_CPML, C.BC_SPONGE):
        g = C.Grid(n, n, n, hh, hh, hh, dt, bc=bc, nb=7, R=1e-3, f0=30.0, vmax=2500.0, sigma=0.05)
        _, _, p, mem = C.forward(g, np.full(g.shape, 2500.0), [[12, 12, 12]], w, [], T)
        scale = np.abs(p).max()
        for ax in range(3):
            assert np.abs(p - np.flip(p, axis=ax)).max() <= 1e-12 * scale
        assert np.abs(p - p.transpose(1, 0, 2)).max() <= 1e-12 * scale
        assert np.abs(p - p.transpose(2, 1, 0)).max() <= 1e-12 * scale
        if bc == C.BC_CPML:
            # psi_x transforms into psi_y under the x <-> y exchange
            assert np.abs(mem[0] - mem[1].transpose(0, 2, 1)).max() <= 1e-12 * np.abs(mem[0]).max()


# --------------------------------------------------------------------- P9
@pytest.mark.parametrize("bc", [C.BC_NONE, C.BC_SPONGE, C.BC_PERIODIC, C.BC_CPML])
def test_p9_dot_product(bc):
    """<F s, r> = <s, F^T r>: the adjoint recursion is the exact transpose of
    the forward map from source wavelets to traces (for CPML including the
    transposed memory recursions; sources and receivers inside the layers
    too)."""
    rng = np.random.default_rng(9)
    nx, ny, nz = 21, 19, 17
    h = (10.0, 9.0, 11.0)
    vel = rng.uniform(1500, 3500, (nz, ny, nx))
    dt = 0.6 * C.dt_stab(vel.max(), *h)
    g = C.Grid(nx, ny, nz, *h, dt, bc=bc, nb=5, sigma=0.05, f0=40.0, vmax=float(vel.max()))
    T = 50
    src = rng.integers(0, [nx, ny, nz], size=(4, 3))
    rec = rng.integers(0, [nx, ny, nz], size=(7, 3))
    rec[3] = src[1]  # a receiver on a source cell
    w = rng.standard_normal((T, 4))
    r = rng.standard_normal((T, 7))
    tr, _, _, _ = C.forward(g, vel, src, w, rec, T)
    adj = C.adjoint(g, vel, rec, r, T, src)
    lhs = float(np.sum(tr * r))
    rhs = float(np.sum(w / (h[0] * h[1] * h[2]) * adj))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


# --------------------------------------------------------------------- P10
@pytest.mark.parametrize("bc", [C.BC_SPONGE, C.BC_CPML])
def test_p10_gradient_finite_differences(bc):
    """Central finite differences of J(m) along a smooth direction match
    <grad, dm> with O(eps^2) convergence; J and the gradient are w.r.t.
    squared slowness m = 1/v^2.  For CPML the damping profile is held fixed
    (vmax is given), so J depends on m only through the wave equation."""
    rng = np.random.default_rng(10)
    nx, ny, nz = 20, 18, 16
    h = (10.0, 10.0, 10.0)
    k = np.arange(nz)[:, None, None]
    vel_true = (2000.0 + 40.0 * k) * np.ones((nz, ny, nx))
    vel_true[6:11, 6:12, 7:13] += 250.0
    vel0 = (2000.0 + 40.0 * k) * np.ones((nz, ny, nx))
    dt = 0.5 * C.dt_stab(vel_true.max() * 1.05, *h)
    if bc == C.BC_SPONGE:
        g = C.Grid(nx, ny, nz, *h, dt, bc=C.BC_SPONGE, nb=4, sigma=0.08)
    else:
        g = C.Grid(nx, ny, nz, *h, dt, bc=C.BC_CPML, nb=4, R=1e-3, f0=30.0, vmax=float(vel_true.max()))
    T = 70
    w = C.ricker(30.0, 0.05, dt, T)[:, None]
    src = [[10, 9, 3]]
    rec = [[i, j, 2] for i in range(2, 18, 3) for j in range(2, 16, 3)]
    d_obs, _, _, _ = C.forward(g, vel_true, src, w, rec, T)
    grad, _, J0 = C.gradient(g, vel0, src, w, rec, d_obs, T)
    m0 = 1.0 / vel0 ** 2
    from scipy.ndimage import gaussian_filter
    dm = gaussian_filter(rng.standard_normal(m0.shape), 2.0)
    dm *= 1e-2 * np.abs(m0).max() / np.abs(dm).max()

    def J(m):
        tr, _, _, _ = C.forward(g, 1.0 / np.sqrt(m), src, w, rec, T)
        return 0.5 * np.sum((tr - d_obs) ** 2)

    want = float(np.sum(grad * dm))
    errs = []
    for eps in (2e-2, 1e-2, 5e-3):
        fd = (J(m0 + eps * dm) - J(m0 - eps * dm)) / (2 * eps)
        errs.append(abs(fd - want) / abs(want))
    assert errs[-1] < 1e-6, errs
    assert errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.0, errs


def test_p10_gradient_zero_residual_and_linearity():
    rng = np.random.default_rng(12)
    nx, ny, nz = 16, 15, 14
    h = (10.0, 10.0, 10.0)
    vel = rng.uniform(1800, 2600, (nz, ny, nx))
    dt = 0.5 * C.dt_stab(vel.max(), *h)
    g = C.Grid(nx, ny, nz, *h, dt, bc=C.BC_SPONGE, nb=4, sigma=0.06)
    T = 40
    w = C.ricker(30.0, 0.05, dt, T)[:, None]
    src = [[8, 7, 3]]
    rec = [[i, 5, 2] for i in range(1, 15, 2)]
    d, _, _, _ = C.forward(g, vel, src, w, rec, T)
    g0, _, J0 = C.gradient(g, vel, src, w, rec, d, T)
    assert J0 == 0.0 and np.all(g0 == 0.0)
    r = rng.standard_normal(d.shape)
    g1, _, _ = C.gradient(g, vel, src, w, rec, d - r, T)
    g2, _, _ = C.gradient(g, vel, src, w, rec, d - 2 * r, T)
    assert np.abs(g2 - 2 * g1).max() <= 1e-12 * np.abs(g1).max()


@pytest.mark.parametrize("bc", [C.BC_SPONGE, C.BC_CPML])
def test_gradient_checkpoint_interval_invariant(bc):
    """FP64 replay from checkpoints is exact: the gradient does not depend on
    the checkpoint interval (bitwise); CPML checkpoints carry the memory."""
    rng = np.random.default_rng(13)
    nx, ny, nz = 14, 13, 12
    h = (10.0, 10.0, 10.0)
    vel = rng.uniform(1800, 2600, (nz, ny, nx))
    dt = 0.5 * C.dt_stab(vel.max(), *h)
    g = C.Grid(nx, ny, nz, *h, dt, bc=bc, nb=3, sigma=0.06, f0=25.0, vmax=float(vel.max()))
    T = 45
    w = rng.standard_normal((T, 1))
    src, rec = [[7, 6, 5]], [[3, 3, 2], [9, 8, 2]]
    d = rng.standard_normal((T, 2)) * 1e-6
    a = C.gradient(g, vel, src, w, rec, d, T, ckpt=T)
    b = C.gradient(g, vel, src, w, rec, d, T, ckpt=7)
    assert np.array_equal(a[0], b[0]) and a[2] == b[2]


# --------------------------------------------------------------------- P12
@pytest.mark.parametrize("bc", [C.BC_NONE, C.BC_SPONGE, C.BC_CPML, C.BC_PERIODIC])
def test_p12_c_oracle_matches_numpy_oracle(bc):
    rng = np.random.default_rng(20 + bc)
    nx, ny, nz = 23, 19, 17
    h = (10.0, 11.0, 12.0)
    vel = rng.uniform(1500, 3000, (nz, ny, nx))
    dt = 0.5 * C.dt_stab(vel.max(), *h)
    T = 45
    src = np.array([[11, 9, 8], [5, 6, 7]])
    rec = np.array([[3, 4, 5], [12, 11, 10], [11, 9, 8], [0, 18, 16]])
    w = rng.standard_normal((T, 2))
    g = C.Grid(nx, ny, nz, *h, dt, bc=bc, nb=5, sigma=0.05, R=1e-3, f0=20.0, vmax=vel.max())
    tr, pm, pc, _ = C.forward(g, vel, src, w, rec, T)
    P = TN.Problem((nz, ny, nx), h, dt, vel, bc=bc, nb=5, sigma=0.05, R=1e-3, f0=20.0, vmax=vel.max())
    tr2, pm2, pc2, _ = P.forward(src, w, rec, T)
    assert np.abs(tr - tr2).max() <= 1e-13 * np.abs(tr).max()
    assert np.abs(pc - pc2).max() <= 1e-13 * np.abs(pc).max()
    assert np.abs(pm - pm2).max() <= 1e-13 * np.abs(pm).max()
    if bc != C.BC_CPML:
        r = rng.standard_normal((T, len(rec)))
        adj = C.adjoint(g, vel, rec, r, T, src)
        adj2, _ = P.adjoint(rec, r, T, src)
        assert np.abs(adj - adj2).max() <= 1e-13 * np.abs(adj).max()
        d_obs = tr + 1e-3 * rng.standard_normal(tr.shape) * np.abs(tr).max()
        gr, _, J = C.gradient(g, vel, src, w, rec, d_obs, T, ckpt=8)
        gr2, _, J2 = P.gradient(src, w, rec, d_obs, T)
        assert abs(J - J2) <= 1e-13 * J
        assert np.abs(gr - gr2).max() <= 1e-12 * np.abs(gr).max()


def test_step_points_matches_whole_step():
    """The point-wise step used for sampled checks on big grids agrees with a
    whole-grid step, CPML memory included."""
    rng = np.random.default_rng(30)
    nx, ny, nz = 24, 22, 20
    h = (10.0, 11.0, 12.0)
    vel = rng.uniform(1500, 3000, (nz, ny, nx))
    dt = 0.5 * C.dt_stab(vel.max(), *h)
    for bc in (C.BC_NONE, C.BC_SPONGE, C.BC_CPML):
        g = C.Grid(nx, ny, nz, *h, dt, bc=bc, nb=6, sigma=0.05, R=1e-3, f0=20.0, vmax=vel.max())
        T = 30
        w = rng.standard_normal((T + 1, 1))
        _, pm, pc, mem = C.forward(g, vel, [[12, 11, 10]], w[:T], [], T)
        pts = np.concatenate([rng.integers(0, [nx, ny, nz], size=(200, 3)), [[12, 11, 10], [0, 0, 0]]])
        st = np.zeros(len(pts))
        st[-2] = w[T, 0] / (h[0] * h[1] * h[2])
        got = C.step_points(g, vel, pm, pc, mem, pts, st)
        _, _, pn, _ = C.forward(g, vel, [[12, 11, 10]], w[T:], [], 1, p_prev=pm, p_cur=pc, cpml_mem=mem)
        want = pn[pts[:, 2], pts[:, 1], pts[:, 0]]
        assert np.abs(got - want).max() <= 1e-14 * np.abs(pn).max()


def test_step_points_on_a_storage_window_equals_full_arrays():
    """The windowed form used for sampled checks on the big grids gives the
    same numbers as the full arrays, and refuses a window that is too small."""
    rng = np.random.default_rng(31)
    nx, ny, nz = 30, 28, 26
    h = (10.0, 11.0, 12.0)
    vel = rng.uniform(1500, 3000, (nz, ny, nx))
    dt = 0.5 * C.dt_stab(vel.max(), *h)
    for bc in (C.BC_NONE, C.BC_SPONGE, C.BC_CPML):
        g = C.Grid(nx, ny, nz, *h, dt, bc=bc, nb=6, sigma=0.05, R=1e-3, f0=20.0, vmax=vel.max())
        _, pm, pc, mem = C.forward(g, vel, [[15, 14, 13]], rng.standard_normal((20, 1)), [], 20)
        pts = np.array([[0, 0, 0], [15, 14, 13], [29, 27, 25], [10, 3, 20], [5, 20, 2]])
        full = C.step_points(g, vel, pm, pc, mem, pts)
        for q, pt in enumerate(pts):
            lo = np.maximum(pt - 8, 0)
            hi = np.minimum(pt + 9, [nx, ny, nz])
            sl = (slice(lo[2], hi[2]), slice(lo[1], hi[1]), slice(lo[0], hi[0]))
            m = None if mem is None else np.ascontiguousarray(mem[(slice(None),) + sl])
            w = (tuple(int(v) for v in lo), tuple(int(v) for v in hi - lo))
            assert C.step_points(g, vel[sl], pm[sl], pc[sl], m, pt[None], window=w)[0] == full[q]
        sl = (slice(10, 14),) * 3
        m = None if mem is None else np.ascontiguousarray(mem[(slice(None),) + sl])
        with pytest.raises(RuntimeError):
            C.step_points(g, vel[sl], pm[sl], pc[sl], m, [[12, 12, 12]], window=((10, 10, 10), (4, 4, 4)))


# ----------------------------------------------------------------- wavelet
def test_ricker_is_normalised_second_derivative_of_gaussian():
    """w(t) = -(1/(2 pi^2 f0^2)) d^2/dt^2 exp(-pi^2 f0^2 (t-t0)^2): the Ricker
    wavelet (reading of the source term; the paper gives only fmax)."""
    f0, t0, dt = 15.0, 0.1, 1e-4
    n = 2000
    w = C.ricker(f0, t0, dt, n)
    t = np.arange(n) * dt
    hstep = 1e-5

    def gauss(tt):
        return np.exp(-(np.pi * f0 * (tt - t0)) ** 2)

    d2 = (gauss(t + hstep) - 2 * gauss(t) + gauss(t - hstep)) / hstep ** 2
    want = -d2 / (2 * np.pi ** 2 * f0 ** 2)
    assert np.abs(w - want).max() < 1e-5
    assert w[int(round(t0 / dt))] == pytest.approx(1.0, abs=1e-12)


# ------------------------------------------------------------ free surface
@pytest.mark.parametrize("bc", [C.BC_NONE, C.BC_SPONGE, C.BC_CPML])
def test_free_surface_equals_method_of_images(bc):
    """A free surface at k = 0 is the odd mirror of the problem: the run on
    nz planes with the free surface equals the upper half of a run on the
    2 nz - 1 planes of the mirrored model (velocity even in k) with the
    source and a negated image source, computed with ordinary zero ghosts;
    damping on the remaining faces is mirrored too."""
    rng = np.random.default_rng(60 + bc)
    nx, ny, nz = 19, 17, 15
    h = (10.0, 9.0, 11.0)
    vel = rng.uniform(1600, 3200, (nz, ny, nx))
    dt = 0.5 * C.dt_stab(vel.max(), *h)
    kw = dict(bc=bc, nb=4, sigma=0.06, f0=30.0, vmax=float(vel.max()))
    T = 60
    src = np.array([[9, 8, 3], [4, 11, 6]])
    w = rng.standard_normal((T, 2))
    rec = np.array([[2, 3, 1], [10, 9, 4], [17, 15, 13], [9, 8, 3], [5, 5, 0]])
    gfs = C.Grid(nx, ny, nz, *h, dt, fs=1, **kw)
    tr, pm, pc, _ = C.forward(gfs, vel, src, w, rec, T)
    # mirrored model: plane K = nz - 1 + k holds k, K = nz - 1 - k holds its image
    M = 2 * nz - 1
    velm = np.concatenate([vel[:0:-1], vel], axis=0)
    srcm = np.concatenate([src + [0, 0, nz - 1], src * [1, 1, -1] + [0, 0, nz - 1]])
    wm = np.concatenate([w, -w], axis=1)
    recm = rec + [0, 0, nz - 1]
    gm = C.Grid(nx, ny, M, *h, dt, **kw)
    trm, pmm, pcm, _ = C.forward(gm, velm, srcm, wm, recm, T)
    scale = np.abs(pc).max()
    assert np.abs(pcm[nz - 1:] - pc).max() <= 1e-12 * scale
    assert np.abs(pmm[nz - 1:] - pm).max() <= 1e-12 * scale
    assert np.abs(trm - tr).max() <= 1e-12 * np.abs(tr).max()
    assert np.all(pc[0] == 0.0) and np.all(tr[:, 4] == 0.0)  # surface plane and a receiver on it


def test_free_surface_conserves_energy():
    rng = np.random.default_rng(61)
    nx, ny, nz = 18, 16, 14
    h = (10.0, 10.0, 10.0)
    vel = rng.uniform(1500, 3000, (nz, ny, nx))
    dt = 0.8 * C.dt_stab(vel.max(), *h)
    g = C.Grid(nx, ny, nz, *h, dt, bc=C.BC_NONE, fs=1)
    T = 30
    w = np.zeros((T, 1))
    w[:5, 0] = [1.0, -2.0, 3.0, -1.0, 0.5]
    _, pm, pc, _ = C.forward(g, vel, [[9, 8, 5]], w, [[1, 1, 1]], T)
    e0 = C.energy(g, vel, pm, pc)
    _, pm2, pc2, _ = C.forward(g, vel, [[9, 8, 5]], np.zeros((200, 1)), [[1, 1, 1]], 200, p_prev=pm, p_cur=pc)
    e1 = C.energy(g, vel, pm2, pc2)
    assert e0 > 0 and abs(e1 - e0) <= 1e-10 * e0


@pytest.mark.parametrize("bc", [C.BC_NONE, C.BC_SPONGE, C.BC_CPML])
def test_free_surface_dot_product(bc):
    """The adjoint with a free surface (the same odd-mirror operator, and
    eta = 0 on the surface) is the exact transpose of the forward map,
    sources and receivers on the surface plane included."""
    rng = np.random.default_rng(62 + bc)
    nx, ny, nz = 20, 18, 16
    h = (10.0, 9.0, 11.0)
    vel = rng.uniform(1500, 3500, (nz, ny, nx))
    dt = 0.6 * C.dt_stab(vel.max(), *h)
    g = C.Grid(nx, ny, nz, *h, dt, bc=bc, nb=4, sigma=0.05, f0=40.0, vmax=float(vel.max()), fs=1)
    T = 50
    src = rng.integers(0, [nx, ny, nz], size=(4, 3))
    src[0, 2] = 0
    src[1, 2] = 2
    rec = rng.integers(0, [nx, ny, nz], size=(7, 3))
    rec[0, 2] = 1
    rec[3] = src[1]
    w = rng.standard_normal((T, 4))
    r = rng.standard_normal((T, 7))
    tr, _, _, _ = C.forward(g, vel, src, w, rec, T)
    adj = C.adjoint(g, vel, rec, r, T, src)
    lhs = float(np.sum(tr * r))
    rhs = float(np.sum(w / (h[0] * h[1] * h[2]) * adj))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    assert np.all(adj[:, 0] == 0.0)  # a source on the surface radiates nothing


def test_free_surface_gradient_finite_differences():
    rng = np.random.default_rng(63)
    nx, ny, nz = 18, 16, 14
    h = (10.0, 10.0, 10.0)
    k = np.arange(nz)[:, None, None]
    vel_true = (2000.0 + 40.0 * k) * np.ones((nz, ny, nx))
    vel_true[5:10, 5:11, 6:12] += 250.0
    vel0 = (2000.0 + 40.0 * k) * np.ones((nz, ny, nx))
    dt = 0.5 * C.dt_stab(vel_true.max() * 1.05, *h)
    g = C.Grid(nx, ny, nz, *h, dt, bc=C.BC_CPML, nb=4, f0=30.0, vmax=float(vel_true.max()), fs=1)
    T = 60
    w = C.ricker(30.0, 0.05, dt, T)[:, None]
    src, rec = [[9, 8, 2]], [[i, j, 1] for i in range(2, 16, 3) for j in range(2, 14, 3)]
    d_obs, _, _, _ = C.forward(g, vel_true, src, w, rec, T)
    grad, _, _ = C.gradient(g, vel0, src, w, rec, d_obs, T)
    m0 = 1.0 / vel0 ** 2
    from scipy.ndimage import gaussian_filter
    dm = gaussian_filter(rng.standard_normal(m0.shape), 2.0)
    dm *= 1e-2 * np.abs(m0).max() / np.abs(dm).max()

    def J(m):
        tr, _, _, _ = C.forward(g, 1.0 / np.sqrt(m), src, w, rec, T)
        return 0.5 * np.sum((tr - d_obs) ** 2)

    want = float(np.sum(grad * dm))
    errs = []
    for eps in (4e-3, 2e-3, 1e-3):
        fd = (J(m0 + eps * dm) - J(m0 - eps * dm)) / (2 * eps)
        errs.append(abs(fd - want) / abs(want))
    assert errs[-1] < 1e-6, errs
    assert errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.0, errs


@pytest.mark.parametrize("ax", [0, 1, 2])
def test_sponge_profile_read_from_one_step(ax):
    """The sponge factor seen by the update itself: from p^{-1} = 0 and
    p^0 = a unit impulse at cell c, one step gives G(c) (2 + D(c) c0) with
    the sponge and 2 + D(c) c0 without it, so their ratio is G(c).  Along a
    line through the centre (G of the other two axes is 1 there) this reads
    the 1D profile off the forward step and checks the Cerjan reading
    independently of the table code: exactly nb damped cells at each end
    (depth 1 at the innermost, nb at the outermost cell), 1 everywhere else,
    G(depth d) = G(depth 1)^(d^2) (a Gaussian in the depth), and
    -ln G(depth 1) = sigma^2.  A depth off by one cell, a layer one cell
    too wide or too narrow, or a non-Gaussian profile fails it."""
    nb, sigma, h = 6, 0.21, 10.0
    n = [15, 15, 15]
    n[ax] = 22
    nx, ny, nz = n
    vel = np.full((nz, ny, nx), 2000.0, dtype=np.float32)
    dt = 0.5 * C.dt_stab(2000.0, h, h, h)
    gs = C.Grid(nx, ny, nz, h, h, h, dt, bc=C.BC_SPONGE, nb=nb, sigma=sigma)
    g0 = C.Grid(nx, ny, nz, h, h, h, dt, bc=C.BC_NONE)
    prof = np.zeros(n[ax])
    for c in range(n[ax]):
        cell = [7, 7, 7]
        cell[ax] = c
        i, j, k = cell
        p0 = np.zeros((nz, ny, nx))
        p0[k, j, i] = 1.0
        _, _, s1, _ = C.forward(gs, vel, [], np.zeros((1, 0)), [], 1, p_prev=np.zeros_like(p0), p_cur=p0)
        _, _, n1, _ = C.forward(g0, vel, [], np.zeros((1, 0)), [], 1, p_prev=np.zeros_like(p0), p_cur=p0)
        prof[c] = s1[k, j, i] / n1[k, j, i]
    depth = np.maximum(np.maximum(nb - np.arange(n[ax]), nb - (n[ax] - 1 - np.arange(n[ax]))), 0)
    assert np.all(prof[depth == 0] == 1.0)
    assert np.all(prof[depth > 0] < 1.0)
    g1 = prof[nb - 1]
    assert -np.log(g1) == pytest.approx(sigma ** 2, rel=1e-12)
    want = g1 ** (depth.astype(np.float64) ** 2)
    assert np.allclose(prof, want, rtol=1e-12, atol=0)
