"""GPU forward parity: the HIP library against the FP64 oracle (element by
element, relative L2), plus exact properties of the GPU path itself.

Tolerance: relative L2 <= 1e-5 over the run for FP32 fields against the FP64
oracle (the bar stated for the 200-step plain forward); measured values are
printed."""
import numpy as np
import pytest
import torch

from paper_2007_06048_amd import minimod as mm
from paper_2007_06048_amd import workloads as W

from .gpu_util import DEV, gpu_forward, oracle_forward, params, rel

pytestmark = pytest.mark.gpu


def _ricker_rows(f0, t0, dt, T, nsrc=1):
    w = mm.ricker(f0, t0, dt, T).astype(np.float64)
    return np.repeat(w[:, None], nsrc, axis=1)


@pytest.mark.parametrize("bc,kern", [(mm.BC_SPONGE, 0), (mm.BC_CPML, mm.CPML_LAYER), (mm.BC_CPML, mm.CPML_FUSED),
                                     (mm.BC_NONE, 0)])
def test_two_layer_64_full_run(bc, kern):
    """64^3 two-layer model, Ricker 15 Hz at the centre, 200 steps at cfl 0.5:
    final field and the 64 x 64 receiver plane within 1e-5 of the oracle
    (CPML: either forward strategy)."""
    wl = W.two_layer_64()
    s = wl.shots[0]
    p = params(s.vel.shape, bc=bc, nb=wl.nb, cfl=wl.cfl, f0=wl.f0, sigma=wl.sigma, cpml_kernel=kern)
    T = wl.nsteps
    dt = mm.dt_for(p, float(s.vel.max()))
    w = _ricker_rows(wl.f0, wl.t0, dt, T)
    tr, pc, pm, dt_gpu = gpu_forward(p, s.vel, s.src, s.rec, w, T)
    assert dt_gpu == dt
    rtr, rpc, rpm = oracle_forward(p, dt, s.vel, s.src, s.rec, w, T)
    e_tr, e_pc, e_pm = rel(tr, rtr), rel(pc, rpc), rel(pm, rpm)
    print(f"bc={bc}: traces {e_tr:.2e} p^T {e_pc:.2e} p^(T-1) {e_pm:.2e}")
    assert e_tr <= 1e-5 and e_pc <= 1e-5 and e_pm <= 1e-5


_RAGGED = (23, 29, 37)  # (nz, ny, nx): not a multiple of any tile size


def _ragged_case(bc, seed=3):
    rng = np.random.default_rng(seed)
    nz, ny, nx = _RAGGED
    vel = rng.uniform(1500.0, 3200.0, _RAGGED).astype(np.float32)
    src = np.array([[18, 14, 11], [3, 5, 7], [18, 14, 11], [0, 0, 0], [36, 28, 22]], dtype=np.int32)
    rec = np.concatenate([W.plane(nx, ny, 2, inc=3), [[18, 14, 11], [36, 28, 22], [0, 28, 0]]]).astype(np.int32)
    p = params(_RAGGED, h=(10.0, 12.0, 9.0), bc=bc, nb=5, f0=25.0, sigma=0.05)
    T = 70
    dt = mm.dt_for(p, float(vel.max()))
    w = rng.standard_normal((T, len(src)))
    return p, vel, src, rec, w, T, dt


_CPML_BOTH = [mm.CPML_LAYER, mm.CPML_FUSED]


@pytest.mark.parametrize("bc,fs,kern", [(mm.BC_NONE, 0, 0), (mm.BC_SPONGE, 0, 0), (mm.BC_CPML, 0, mm.CPML_LAYER),
                                        (mm.BC_CPML, 0, mm.CPML_FUSED), (mm.BC_NONE, 1, 0), (mm.BC_SPONGE, 1, 0),
                                        (mm.BC_CPML, 1, mm.CPML_LAYER), (mm.BC_CPML, 1, mm.CPML_FUSED)])
def test_ragged_every_tile_variant(bc, fs, kern):
    """A ragged grid (partial tiles in x, y and z), duplicate sources,
    receivers on sources and on corners: every tile variant matches the oracle
    and all variants agree bitwise (tiling does not change the arithmetic),
    in either forward CPML strategy.  With a free surface a source and a
    receiver sit on the surface plane."""
    p, vel, src, rec, w, T, dt = _ragged_case(bc)
    p.free_surface = fs
    p.cpml_kernel = kern
    rtr, rpc, _ = oracle_forward(p, dt, vel, src, rec, w, T)
    first = None
    for t in range(mm.num_tiles()):
        tr, pc, pm, _ = gpu_forward(p, vel, src, rec, w, T, tile=t)
        assert rel(tr, rtr) <= 1e-5, (t, rel(tr, rtr))
        assert rel(pc, rpc) <= 1e-5, (t, rel(pc, rpc))
        if first is None:
            first = (tr, pc, pm)
        else:
            assert np.array_equal(first[0], tr) and np.array_equal(first[1], pc) and np.array_equal(first[2], pm), t


@pytest.mark.parametrize("bc,fs,kern", [(mm.BC_NONE, 0, 0), (mm.BC_SPONGE, 0, 0), (mm.BC_CPML, 0, mm.CPML_LAYER),
                                        (mm.BC_CPML, 0, mm.CPML_FUSED), (mm.BC_CPML, 1, mm.CPML_LAYER),
                                        (mm.BC_CPML, 1, mm.CPML_FUSED)])
def test_graph_and_chunked_runs_are_bitwise_equal(bc, fs, kern):
    p, vel, src, rec, w, T, dt = _ragged_case(bc, seed=4)
    p.free_surface = fs
    p.cpml_kernel = kern
    a = gpu_forward(p, vel, src, rec, w, T)
    b = gpu_forward(p, vel, src, rec, w, T, graph=True)
    c = gpu_forward(p, vel, src, rec, w, T, chunks=[1, 20, 0, 33, 16])
    d = gpu_forward(p, vel, src, rec, w, T, graph=True, chunks=[35, 35])
    for other in (b, c, d):
        for x, y in zip(a[:3], other[:3]):
            assert np.array_equal(x, y)


@pytest.mark.parametrize("bc,fs,kern", [(mm.BC_NONE, 0, 0), (mm.BC_SPONGE, 0, 0), (mm.BC_CPML, 0, mm.CPML_LAYER),
                                        (mm.BC_CPML, 0, mm.CPML_FUSED), (mm.BC_CPML, 1, mm.CPML_FUSED)])
def test_cache_hints_do_not_change_results(bc, fs, kern):
    """Non-temporal loads (forced on, forced off) change only where data is
    cached: traces and fields are bitwise the same, and the same as auto."""
    p, vel, src, rec, w, T, dt = _ragged_case(bc, seed=5)
    p.free_surface = fs
    p.cpml_kernel = kern
    out = []
    for h in (0, 1, 2):
        p.cache_hints = h
        out.append(gpu_forward(p, vel, src, rec, w, T))
    for other in out[1:]:
        for x, y in zip(out[0][:3], other[:3]):
            assert np.array_equal(x, y)


def test_minimal_and_degenerate_grids():
    """Smallest grids the damping allows (n = 2 nb + 1, CPML 2 nb + 4), a one-cell-thick
    grid with bc none, and runs with no receivers or no sources."""
    rng = np.random.default_rng(8)
    cases = [((11, 11, 11), mm.BC_SPONGE, 5), ((14, 15, 17), mm.BC_CPML, 5), ((1, 5, 9), mm.BC_NONE, 0),
             ((7, 1, 6), mm.BC_NONE, 0), ((6, 5, 1), mm.BC_NONE, 0)]
    for shape, bc, nb in cases:
        nz, ny, nx = shape
        vel = rng.uniform(1800, 2500, shape).astype(np.float32)
        p = params(shape, bc=bc, nb=nb)
        dt = mm.dt_for(p, float(vel.max()))
        T = 25
        src = np.array([[nx // 2, ny // 2, nz // 2]], dtype=np.int32)
        rec = np.array([[0, 0, 0], [nx - 1, ny - 1, nz - 1], [nx // 2, ny // 2, nz // 2]], dtype=np.int32)
        w = rng.standard_normal((T, 1))
        tr, pc, _, _ = gpu_forward(p, vel, src, rec, w, T)
        rtr, rpc, _ = oracle_forward(p, dt, vel, src, rec, w, T)
        assert rel(tr, rtr) <= 1e-5 and rel(pc, rpc) <= 1e-5, (shape, rel(tr, rtr), rel(pc, rpc))
        # no receivers: the field is the same
        _, pc2, _, _ = gpu_forward(p, vel, src, np.zeros((0, 3), np.int32), w, T)
        assert np.array_equal(pc, pc2)
        # no sources: the field stays exactly zero
        _, pc3, _, _ = gpu_forward(p, vel, np.zeros((0, 3), np.int32), rec, np.zeros((T, 0)), T)
        assert not np.any(pc3)


def test_zero_steps_and_determinism():
    p, vel, src, rec, w, T, dt = _ragged_case(mm.BC_CPML, seed=5)
    a = gpu_forward(p, vel, src, rec, w, T)
    b = gpu_forward(p, vel, src, rec, w, T)
    for x, y in zip(a[:3], b[:3]):
        assert np.array_equal(x, y)
    z = gpu_forward(p, vel, src, rec, w[:0], 0)
    assert not np.any(z[1]) and not np.any(z[2])


def test_state_save_restore_resume_bitwise():
    """100 steps, save, 100 more == 100 steps, restore into a fresh context,
    100 more (CPML memory included)."""
    p, vel, src, rec, w, T, dt = _ragged_case(mm.BC_CPML, seed=6)
    T = 60
    vt = torch.from_numpy(vel).to(DEV)
    wt = torch.from_numpy(np.asarray(w[:T], dtype=np.float32)).to(DEV)
    a = mm.Context.single(p, vt, src, rec)
    a.forward(30, wt[:30])
    st = a.get_state().clone()
    a.forward(30, wt[30:])
    b = mm.Context.single(p, vt, src, rec)
    b.set_state(st, 30)
    b.forward(30, wt[30:])
    sa, sb = a.get_state(), b.get_state()
    torch.cuda.synchronize()
    assert torch.equal(sa, sb)
    assert a.info()["step"] == b.info()["step"] == 60


def _batch_traces(p, vels, srcs, recs, ws, T, graph):
    ctx = mm.Context(p, [(torch.from_numpy(v).to(DEV), s, r) for v, s, r in zip(vels, srcs, recs)])
    wcat = torch.from_numpy(np.concatenate(ws, axis=1)).to(DEV)
    tr = torch.zeros((T, ctx.nrec), dtype=torch.float32, device=DEV)
    if graph:
        for j in range(0, T, 10):
            ctx.forward(10, wcat[j:j + 10], tr[j:j + 10], graph=True)
    else:
        ctx.forward(T, wcat, tr)
    out = tr.cpu().numpy()
    ng = ctx.info()["groups"]
    ctx.close()
    return out, ng


@pytest.mark.parametrize("group_kb,graph,many_src,kern",
                         [(-1, False, False, mm.CPML_LAYER), (1, False, False, mm.CPML_LAYER),
                          (1, True, False, mm.CPML_LAYER), (0, True, False, mm.CPML_LAYER),
                          (1, False, True, mm.CPML_LAYER), (700, True, True, mm.CPML_LAYER),
                          (-1, False, False, mm.CPML_FUSED), (1, True, False, mm.CPML_FUSED),
                          (700, True, True, mm.CPML_FUSED)])
def test_batched_shots_equal_single_shot_runs(group_kb, graph, many_src, kern):
    """Three uneven sub-volumes in one context give bitwise the single-shot
    results, whether all shots advance together (group_kb -1 or the default
    budget), one shot at a time (1 KiB budget) or two and one (700 KiB),
    eagerly or from captured graphs, in either forward CPML strategy.  With a
    shot of six sources every source goes through the injection kernel; then
    the reference is the same batch advanced as one group."""
    rng = np.random.default_rng(9)
    shapes = [(20, 26, 33), (31, 17, 22), (18, 18, 41)]
    p = params(shapes[0], bc=mm.BC_CPML, nb=4, f0=25.0, cpml_kernel=kern)
    vels = [rng.uniform(1500, 3000, s).astype(np.float32) for s in shapes]
    p.vmax = float(max(v.max() for v in vels))
    T = 40
    srcs = [np.array([[s[2] // 2, s[1] // 2, s[0] // 2]], np.int32) for s in shapes]
    if many_src:
        srcs[1] = W.random_points(rng, 6, shapes[1], margin=1)
    recs = [W.plane(s[2], s[1], 3, inc=2) for s in shapes]
    ws = [rng.standard_normal((T, len(s))).astype(np.float32) for s in srcs]
    p.group_kb = group_kb
    trb, ng = _batch_traces(p, vels, srcs, recs, ws, T, graph)
    assert ng == {-1: 1, 0: 1, 1: 3, 700: 2}[group_kb]
    if many_src:
        p.group_kb = -1
        ref, _ = _batch_traces(p, vels, srcs, recs, ws, T, False)
        assert np.array_equal(trb, ref)
        return
    off = 0
    for v, s, r, w in zip(vels, srcs, recs, ws):
        q = mm.default_params(**{k: getattr(p, k) for k, _ in mm.Params._fields_})
        q.nz, q.ny, q.nx = v.shape
        q.group_kb = 0
        t1, _, _, _ = gpu_forward(q, v, s, r, w, T)
        assert np.array_equal(t1, trb[:, off:off + len(r)])
        off += len(r)


def test_errors_leave_context_usable():
    vel = np.full((16, 16, 16), 2000.0, np.float32)
    src = np.array([[8, 8, 8]], np.int32)
    vt = torch.from_numpy(vel).to(DEV)
    p = params(vel.shape, bc=mm.BC_SPONGE, nb=4)
    p.cfl = 1.01
    with pytest.raises(mm.MinimodError) as e:
        mm.Context.single(p, vt, src, src)
    assert e.value.status == mm.MM_ERR_UNSTABLE
    p.cfl = 0.5
    bad = vel.copy()
    bad[3, 4, 5] = np.nan
    with pytest.raises(mm.MinimodError) as e:
        mm.Context.single(p, torch.from_numpy(bad).to(DEV), src, src)
    assert e.value.status == mm.MM_ERR_NONFINITE
    bad[3, 4, 5] = -1.0
    with pytest.raises(mm.MinimodError) as e:
        mm.Context.single(p, torch.from_numpy(bad).to(DEV), src, src)
    assert e.value.status == mm.MM_ERR_NONFINITE
    with pytest.raises(mm.MinimodError) as e:
        mm.Context.single(p, vt, np.array([[16, 0, 0]], np.int32), src)
    assert e.value.status == mm.MM_ERR_ARG
    ctx = mm.Context.single(p, vt, src, src)
    with pytest.raises(mm.MinimodError) as e:
        ctx.forward(3, None)
    assert e.value.status == mm.MM_ERR_ARG
    with pytest.raises(mm.MinimodError) as e:
        ctx.adjoint(1, torch.zeros((1, 1), device=DEV))
    assert e.value.status == mm.MM_ERR_STATE  # made without adjoint storage
    w = torch.ones((3, 1), device=DEV)
    ctx.forward(3, w)
    assert ctx.info()["step"] == 3


def test_autotune_then_forward_matches_default_tile():
    """The autotuner's trial steps (no wavelet) leave a zero state; the tuned
    context then reproduces the default-tile run bitwise (the CPML strategy
    held fixed: the two sum the layer terms in different orders)."""
    p, vel, src, rec, w, T, dt = _ragged_case(mm.BC_CPML, seed=12)
    p.cpml_kernel = mm.CPML_LAYER
    src, w = src[:3], w[:, :3]  # few enough sources to be added inside the stencil kernel
    a = gpu_forward(p, vel, src, rec, w, T)
    ctx = mm.Context.single(p, torch.from_numpy(vel).to(DEV), src, rec)
    t = ctx.autotune(2)
    assert 0 <= t < mm.num_tiles()
    assert ctx.info()["step"] == 0
    st = ctx.get_state()
    torch.cuda.synchronize()
    assert not torch.any(st)
    tr = torch.zeros((T, len(rec)), dtype=torch.float32, device=DEV)
    ctx.forward(T, torch.from_numpy(np.asarray(w, dtype=np.float32)).to(DEV), tr)
    assert np.array_equal(tr.cpu().numpy(), a[0])
    q = mm.default_params(**{k: getattr(p, k) for k, _ in mm.Params._fields_})
    q.tile = -1  # autotune inside init
    b = gpu_forward(q, vel, src, rec, w, T)
    assert np.array_equal(b[0], a[0]) and np.array_equal(b[1], a[1])


def test_cpml_strategy_choice_and_tuning():
    """The forward CPML strategy: the layer pass by default on a grid whose
    layers hold most of the cells, each strategy when forced, none reported
    for a sponge; the autotuner settles on one of the two, and the tuned
    context reproduces a fresh run forced to that strategy bitwise."""
    p, vel, src, rec, w, T, dt = _ragged_case(mm.BC_CPML, seed=13)
    src, w = src[:3], w[:, :3]
    v = torch.from_numpy(vel).to(DEV)

    def with_(**kw):
        q = mm.default_params(**{k: getattr(p, k) for k, _ in mm.Params._fields_})
        for k, x in kw.items():
            setattr(q, k, x)
        return q

    assert mm.Context.single(p, v, src, rec).cpml_kernel() == mm.CPML_LAYER
    for k in (mm.CPML_LAYER, mm.CPML_FUSED):
        assert mm.Context.single(with_(cpml_kernel=k), v, src, rec).cpml_kernel() == k
    assert mm.Context.single(with_(bc=mm.BC_SPONGE), v, src, rec).cpml_kernel() == mm.CPML_AUTO
    ctx = mm.Context.single(p, v, src, rec)
    t = ctx.autotune(2)
    k = ctx.cpml_kernel()
    assert k in (mm.CPML_LAYER, mm.CPML_FUSED)
    tr = torch.zeros((T, len(rec)), dtype=torch.float32, device=DEV)
    ctx.forward(T, torch.from_numpy(np.asarray(w, dtype=np.float32)).to(DEV), tr)
    ref = gpu_forward(with_(cpml_kernel=k), vel, src, rec, w, T, tile=t)
    assert np.array_equal(tr.cpu().numpy(), ref[0])


@pytest.mark.parametrize("bc", [mm.BC_NONE, mm.BC_SPONGE, mm.BC_CPML])
def test_step_timing_stamps_every_bc(bc):
    """mm_profile stamps whole time steps (the first launch's start, the last
    launch's end) for every boundary kind, CPML included where the CPML
    kernel takes the start stamp; timing leaves the results bitwise alone."""
    p, vel, src, rec, w, T, dt = _ragged_case(bc, seed=6)
    ref = gpu_forward(p, vel, src, rec, w, T)
    ctx = mm.Context.single(p, torch.from_numpy(vel).to(DEV), src, rec)
    tr = torch.zeros((T, len(rec)), dtype=torch.float32, device=DEV)
    ctx.profile(3)
    ctx.forward(T, torch.from_numpy(np.asarray(w, dtype=np.float32)).to(DEV), tr)
    ms, n = ctx.profile_read()
    ctx.profile(0)
    assert n == (T + 2) // 3 and ms > 0.0, (n, ms)
    assert np.array_equal(tr.cpu().numpy(), ref[0])
    ctx.close()
