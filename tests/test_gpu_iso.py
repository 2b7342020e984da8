"""acoustic_iso (first-order variable-density system on the staggered grid)
on the GPU: parity with the FP64 oracle (traces, pressure and the three
face-velocity fields) for bc none, sponge and CPML, with and without the free
surface, every supported tile variant bitwise equal, graph and chunked runs
bitwise equal, state round trip, argument errors, and larger grids against
the oracle."""
import numpy as np
import pytest
import torch

from oracle import c_oracle as C
from paper_2007_06048_amd import minimod as mm
from paper_2007_06048_amd import workloads as W

from .gpu_util import DEV, rel

pytestmark = pytest.mark.gpu


def _case(bc, shape=(23, 29, 37), seed=80, T=120):
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    v = rng.uniform(1600.0, 3200.0, shape).astype(np.float32)
    rho = (310.0 * v.astype(np.float64) ** 0.25 * rng.uniform(0.9, 1.1, shape)).astype(np.float32)
    src = np.array([[nx // 2, ny // 2, nz // 2], [3, 4, 5], [nx // 2, ny // 2, nz // 2], [nx - 1, 0, 2]], np.int32)
    rec = np.concatenate([W.plane(nx, ny, 2, inc=3), [[nx // 2, ny // 2, nz // 2], [0, ny - 1, nz - 1]]]).astype(np.int32)
    p = mm.default_params(nx=nx, ny=ny, nz=nz, dx=10.0, dy=12.0, dz=9.0, bc=bc, nb=5, sponge_sigma=0.05,
                          cpml_f0=20.0, model=mm.MODEL_ISO, tile=0)
    w = rng.standard_normal((T, len(src))).astype(np.float32)
    return p, v, rho, src, rec, w, T


def _gpu(p, v, rho, src, rec, w, T, tile=None, graph=False, chunks=None):
    ctx = mm.Context.single(p, torch.from_numpy(v).to(DEV), src, rec, rho=torch.from_numpy(rho).to(DEV))
    if tile is not None:
        ctx.set_tile(tile)
    tr = torch.zeros((T, len(rec)), device=DEV)
    wt = torch.from_numpy(w).to(DEV)
    done = 0
    for c in (chunks or [T]):
        ctx.forward(c, wt[done:done + c], tr[done:done + c], graph=graph)
        done += c
    # p and the three velocities (with CPML the blob goes on with the layer memory)
    st = ctx.get_state().cpu().numpy()[:4 * v.size].reshape((4,) + v.shape)
    dt = ctx.dt
    ctx.close()
    return tr.cpu().numpy(), st, dt


def _oracle(p, dt, v, rho, src, rec, w, T):
    g = C.Grid(p.nx, p.ny, p.nz, p.dx, p.dy, p.dz, dt, bc=p.bc, nb=p.nb, sigma=p.sponge_sigma, R=p.cpml_R,
               f0=p.cpml_f0, vmax=float(v.max()), fs=p.free_surface)
    tr, st = C.iso_forward(g, v.astype(np.float64), rho.astype(np.float64), src, w.astype(np.float64), rec, T)
    return tr, st[:4]


@pytest.mark.parametrize("bc,fs", [(mm.BC_NONE, 0), (mm.BC_SPONGE, 0), (mm.BC_CPML, 0), (mm.BC_NONE, 1),
                                   (mm.BC_SPONGE, 1), (mm.BC_CPML, 1)])
def test_iso_matches_oracle(bc, fs):
    """Ragged grid, duplicate sources, receivers on sources and corners; with a
    free surface a source and a receiver sit on the surface plane (which
    injects and records nothing)."""
    p, v, rho, src, rec, w, T = _case(bc)
    p.free_surface = fs
    if fs:
        src = np.concatenate([src, [[4, 5, 0]]]).astype(np.int32)
        rec = np.concatenate([rec, [[4, 5, 0], [7, 3, 1]]]).astype(np.int32)
        w = np.concatenate([w, np.ones((T, 1), np.float32)], axis=1)
    tr, st, dt = _gpu(p, v, rho, src, rec, w, T)
    if fs:
        assert not st[0][0].any() and not tr[:, -2].any()
    assert dt == pytest.approx(0.5 * C.iso_dt_stab(float(v.max()), p.dx, p.dy, p.dz), rel=1e-15)
    rtr, rst = _oracle(p, dt, v, rho, src, rec, w, T)
    print("traces", rel(tr, rtr), "p", rel(st[0], rst[0]), "u", [rel(st[a], rst[a]) for a in (1, 2, 3)])
    assert rel(tr, rtr) <= 1e-5
    for a in range(4):
        assert rel(st[a], rst[a]) <= 1e-5, a


@pytest.mark.parametrize("shape", [(9, 11, 1), (9, 1, 13), (1, 11, 13), (1, 1, 40), (3, 70, 5)])
def test_iso_degenerate_grids_match_oracle(shape):
    """One-cell-thick grids, a single column, and a grid narrower than the
    stencil radius along x: every tile variant against the oracle (bc none,
    sources and receivers at the grid corners)."""
    rng = np.random.default_rng(84)
    nz, ny, nx = shape
    v = rng.uniform(1600.0, 3200.0, shape).astype(np.float32)
    rho = rng.uniform(1000.0, 2500.0, shape).astype(np.float32)
    src = np.array([[nx // 2, ny // 2, nz // 2], [0, 0, 0]], np.int32)
    rec = np.array([[nx - 1, ny - 1, nz - 1], [nx // 2, ny // 2, nz // 2], [0, ny - 1, 0]], np.int32)
    p = mm.default_params(nx=nx, ny=ny, nz=nz, dx=10.0, dy=12.0, dz=9.0, bc=mm.BC_NONE, model=mm.MODEL_ISO, tile=0)
    T = 30
    w = rng.standard_normal((T, len(src))).astype(np.float32)
    first = None
    for t in range(mm.num_tiles()):
        name = mm.tile_name(t)
        if "t512" in name or "t1024" in name:
            continue
        tr, st, dt = _gpu(p, v, rho, src, rec, w, T, tile=t)
        if first is None:
            first = (tr, st)
            rtr, rst = _oracle(p, dt, v, rho, src, rec, w, T)
            assert rel(tr, rtr) <= 1e-5 and all(rel(st[a], rst[a]) <= 1e-5 for a in range(4))
        else:
            assert np.array_equal(first[0], tr) and np.array_equal(first[1], st), name


def test_iso_zero_steps_no_sources_no_receivers():
    p, v, rho, src, rec, w, T = _case(mm.BC_SPONGE, seed=85, T=10)
    vt, rt = torch.from_numpy(v).to(DEV), torch.from_numpy(rho).to(DEV)
    ctx = mm.Context.single(p, vt, src, rec, rho=rt)
    ctx.forward(0, torch.zeros((0, len(src)), device=DEV), torch.zeros((0, len(rec)), device=DEV))
    assert ctx.info()["step"] == 0 and not ctx.get_state().any()
    none = np.zeros((0, 3), np.int32)
    tr, st, _ = _gpu(p, v, rho, none, rec, np.zeros((T, 0), np.float32), T)
    assert not st.any() and not tr.any()  # nothing excites the field
    tr, st, dt = _gpu(p, v, rho, src, none, w, T)
    rtr, rst = _oracle(p, dt, v, rho, src, none, w, T)
    assert tr.shape == (T, 0) and rel(st[0], rst[0]) <= 1e-5


def test_iso_cache_hints_do_not_change_results():
    p, v, rho, src, rec, w, T = _case(mm.BC_SPONGE, seed=86, T=40)
    out = []
    for h in (1, 2):
        p.cache_hints = h
        out.append(_gpu(p, v, rho, src, rec, w, T))
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])


@pytest.mark.parametrize("bc,fs", [(mm.BC_SPONGE, 0), (mm.BC_SPONGE, 1), (mm.BC_CPML, 0), (mm.BC_CPML, 1)])
def test_iso_every_tile_variant_bitwise(bc, fs):
    p, v, rho, src, rec, w, T = _case(bc, seed=81, T=60)
    p.free_surface = fs
    first = None
    n = 0
    for t in range(mm.num_tiles()):
        name = mm.tile_name(t)
        if "t512" in name or "t1024" in name:
            continue
        tr, st, _ = _gpu(p, v, rho, src, rec, w, T, tile=t)
        n += 1
        if first is None:
            first = (tr, st)
        else:
            assert np.array_equal(first[0], tr) and np.array_equal(first[1], st), name
    assert n >= 30


def test_iso_graph_and_chunked_runs_are_bitwise_equal():
    p, v, rho, src, rec, w, T = _case(mm.BC_SPONGE, seed=82, T=50)
    a = _gpu(p, v, rho, src, rec, w, T)
    b = _gpu(p, v, rho, src, rec, w, T, graph=True)
    c = _gpu(p, v, rho, src, rec, w, T, chunks=[1, 20, 0, 29])
    for other in (b, c):
        assert np.array_equal(a[0], other[0]) and np.array_equal(a[1], other[1])


@pytest.mark.parametrize("bc,fs", [(mm.BC_NONE, 0), (mm.BC_NONE, 1), (mm.BC_CPML, 0)])
def test_iso_state_round_trip_and_resume(bc, fs):
    """The state blob (with CPML, the layer memory too) restores a run
    bitwise."""
    p, v, rho, src, rec, w, T = _case(bc, seed=83, T=40)
    p.free_surface = fs
    whole = _gpu(p, v, rho, src, rec, w, T)
    ctx = mm.Context.single(p, torch.from_numpy(v).to(DEV), src, rec, rho=torch.from_numpy(rho).to(DEV))
    wt = torch.from_numpy(w).to(DEV)
    tr = torch.zeros((T, len(rec)), device=DEV)
    ctx.forward(25, wt[:25], tr[:25])
    st = ctx.get_state().clone()
    ctx.reset()
    ctx.set_state(st, 25)
    ctx.forward(T - 25, wt[25:], tr[25:])
    assert np.array_equal(tr.cpu().numpy(), whole[0])
    assert np.array_equal(ctx.get_state().cpu().numpy()[:4 * v.size].reshape((4,) + v.shape), whole[1])


def test_iso_argument_errors():
    p, v, rho, src, rec, w, T = _case(mm.BC_SPONGE, shape=(16, 16, 16), T=4)
    vt, rt = torch.from_numpy(v).to(DEV), torch.from_numpy(rho).to(DEV)
    for field, val, status in (("ckpt_every", 8, mm.MM_ERR_UNSUPPORTED), ("model", 7, mm.MM_ERR_ARG)):
        q = mm.default_params(**{k: getattr(p, k) for k, _ in mm.Params._fields_})
        setattr(q, field, val)
        q.nsteps_max = 10
        with pytest.raises(mm.MinimodError) as e:
            mm.Context.single(q, vt, src, rec, rho=rt)
        assert e.value.status == status, field
    with pytest.raises(mm.MinimodError) as e:
        mm.Context.single(p, vt, src, rec)  # no density
    assert e.value.status == mm.MM_ERR_ARG
    bad = rho.copy()
    bad[3, 4, 5] = 0.0
    with pytest.raises(mm.MinimodError) as e:
        mm.Context.single(p, vt, src, rec, rho=torch.from_numpy(bad).to(DEV))
    assert e.value.status == mm.MM_ERR_NONFINITE
    ctx = mm.Context.single(p, vt, src, rec, rho=rt)
    big = [t for t in range(mm.num_tiles()) if "t1024" in mm.tile_name(t)][0]
    with pytest.raises(mm.MinimodError) as e:
        ctx.set_tile(big)
    assert e.value.status == mm.MM_ERR_ARG


def test_iso_larger_grid_matches_oracle():
    """160^3, Gardner density, 20-cell sponge, 60 steps, autotuned tile."""
    n = 160
    wl = W.smooth_iso(n=n, nsteps=60)
    s = wl.shots[0]
    p = mm.default_params(nx=n, ny=n, nz=n, dx=wl.h, dy=wl.h, dz=wl.h, cfl=wl.cfl, bc=wl.bc, nb=wl.nb,
                          sponge_sigma=wl.sigma, model=mm.MODEL_ISO, tile=-1)
    ctx = mm.Context.single(p, torch.from_numpy(s.vel).to(DEV), s.src, s.rec, rho=torch.from_numpy(s.rho).to(DEV))
    T = wl.nsteps
    w = mm.ricker(wl.f0, wl.t0, ctx.dt, T).reshape(T, 1)
    tr = torch.zeros((T, len(s.rec)), device=DEV)
    ctx.forward(T, torch.from_numpy(w).to(DEV), tr)
    st = ctx.get_state().cpu().numpy().reshape((4,) + s.vel.shape)
    rtr, rst = _oracle(p, ctx.dt, s.vel, s.rho, s.src, s.rec, w, T)
    print("traces", rel(tr.cpu().numpy(), rtr), "p", rel(st[0], rst[0]))
    assert rel(tr.cpu().numpy(), rtr) <= 1e-5 and rel(st[0], rst[0]) <= 1e-5


def test_iso_cpml_larger_grid_matches_oracle():
    """120^3 smooth model with Gardner density, 16-cell CPML, 150 steps,
    autotuned tile: traces and pressure against the oracle."""
    n = 120
    wl = W.smooth_iso(n=n, nsteps=150)
    s = wl.shots[0]
    p = mm.default_params(nx=n, ny=n, nz=n, dx=wl.h, dy=wl.h, dz=wl.h, cfl=wl.cfl, bc=mm.BC_CPML, nb=16,
                          cpml_f0=wl.f0, model=mm.MODEL_ISO, tile=-1)
    ctx = mm.Context.single(p, torch.from_numpy(s.vel).to(DEV), s.src, s.rec, rho=torch.from_numpy(s.rho).to(DEV))
    T = wl.nsteps
    w = mm.ricker(wl.f0, wl.t0, ctx.dt, T).reshape(T, 1)
    tr = torch.zeros((T, len(s.rec)), device=DEV)
    ctx.forward(T, torch.from_numpy(w).to(DEV), tr)
    st = ctx.get_state().cpu().numpy()[:s.vel.size].reshape(s.vel.shape)
    rtr, rst = _oracle(p, ctx.dt, s.vel, s.rho, s.src, s.rec, w, T)
    print("traces", rel(tr.cpu().numpy(), rtr), "p", rel(st, rst[0]))
    assert rel(tr.cpu().numpy(), rtr) <= 1e-5 and rel(st, rst[0]) <= 1e-5
