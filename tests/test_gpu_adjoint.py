"""GPU adjoint and FWI gradient: dot-product test, parity with the FP64
oracle's adjoint and gradient (FP32 and BF16 checkpoints; sponge, CPML and
no boundary), the autograd binding, chunked and batched adjoint runs."""
import numpy as np
import pytest
import torch

from oracle import c_oracle as C
from paper_2007_06048_amd import minimod as mm

from .gpu_util import DEV, grid_for, params, rel

pytestmark = pytest.mark.gpu


def _case(bc, nsrc, seed, shape=(26, 30, 34), T=80):
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    vel = rng.uniform(1600.0, 3000.0, shape).astype(np.float32)
    src = np.stack([rng.integers(0, nx, nsrc), rng.integers(0, ny, nsrc), rng.integers(0, nz, nsrc)], 1).astype(np.int32)
    rec = np.stack([rng.integers(0, nx, 9), rng.integers(0, ny, 9), rng.integers(0, nz, 9)], 1).astype(np.int32)
    rec[2] = src[0]
    rec[5] = rec[4]  # a duplicated receiver
    p = params(shape, h=(10.0, 11.0, 9.0), bc=bc, nb=5, sigma=0.05)
    return rng, vel, src, rec, p, T


@pytest.mark.parametrize("bc,nsrc,fs", [(mm.BC_SPONGE, 1, 0), (mm.BC_SPONGE, 6, 0), (mm.BC_NONE, 3, 0),
                                        (mm.BC_CPML, 1, 0), (mm.BC_CPML, 6, 0), (mm.BC_SPONGE, 1, 1),
                                        (mm.BC_CPML, 6, 1)])
def test_dot_product_and_adjoint_parity(bc, nsrc, fs):
    """<F s, r> = <s, F^T r> on the GPU (FP32), and the GPU adjoint seismograms
    at the sources match the FP64 oracle's adjoint (with a free surface: a
    receiver on the surface plane and one just below it)."""
    rng, vel, src, rec, p, T = _case(bc, nsrc, seed=10 + nsrc)
    p.free_surface = fs
    if fs:
        rec[0, 2] = 0
        rec[1, 2] = 1
    p.ckpt_every = 16
    p.nsteps_max = T
    w = rng.standard_normal((T, nsrc)).astype(np.float32)
    r = rng.standard_normal((T, len(rec))).astype(np.float32)
    ctx = mm.Context.single(p, torch.from_numpy(vel).to(DEV), src, rec)
    tr = torch.zeros((T, len(rec)), device=DEV)
    ctx.forward(T, torch.from_numpy(w).to(DEV), tr)
    adj = torch.zeros((T, nsrc), device=DEV)
    ctx.adjoint(T, torch.from_numpy(r).to(DEV), adj)
    torch.cuda.synchronize()
    h = (p.dx, p.dy, p.dz)
    lhs = float(np.sum(tr.cpu().numpy().astype(np.float64) * r))
    rhs = float(np.sum(w.astype(np.float64) / (h[0] * h[1] * h[2]) * adj.cpu().numpy()))
    print(f"dot product: {lhs:.6e} vs {rhs:.6e}, rel {abs(lhs - rhs) / abs(lhs):.2e}")
    assert abs(lhs - rhs) <= 1e-5 * abs(lhs)
    g = grid_for(p, ctx.dt, float(vel.max()))
    ref = C.adjoint(g, vel.astype(np.float64), rec, r.astype(np.float64), T, src)
    assert rel(adj.cpu().numpy(), ref) <= 1e-5, rel(adj.cpu().numpy(), ref)


@pytest.mark.parametrize("bc", [mm.BC_SPONGE, mm.BC_CPML])
def test_adjoint_in_chunks_is_bitwise_one_call(bc):
    rng, vel, src, rec, p, T = _case(bc, 2, seed=21)
    p.ckpt_every = 16
    p.nsteps_max = T
    w = torch.from_numpy(rng.standard_normal((T, 2)).astype(np.float32)).to(DEV)
    r = torch.from_numpy(rng.standard_normal((T, len(rec))).astype(np.float32)).to(DEV)
    out = []
    for chunks in ([T], [30, 1, 49]):
        ctx = mm.Context.single(p, torch.from_numpy(vel).to(DEV), src, rec)
        ctx.forward(T, w)
        adj = torch.zeros((T, 2), device=DEV)
        g = torch.zeros(vel.shape, device=DEV)
        hi = T
        for cnum in chunks:  # adjoint walks backward: rows [hi - cnum, hi)
            ctx.adjoint(cnum, r[hi - cnum:hi], adj[hi - cnum:hi], g)
            hi -= cnum
        out.append((adj.cpu().numpy(), g.cpu().numpy()))
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])


@pytest.mark.parametrize("bc,snap,tol,fs,kern", [(mm.BC_SPONGE, mm.SNAP_FP32, 1e-4, 0, 0),
                                                  (mm.BC_SPONGE, mm.SNAP_BF16, 1e-2, 0, 0),
                                                  (mm.BC_CPML, mm.SNAP_FP32, 1e-4, 0, mm.CPML_LAYER),
                                                  (mm.BC_CPML, mm.SNAP_FP32, 1e-4, 0, mm.CPML_FUSED),
                                                  (mm.BC_CPML, mm.SNAP_BF16, 1e-2, 0, mm.CPML_LAYER),
                                                  (mm.BC_CPML, mm.SNAP_BF16, 1e-2, 0, mm.CPML_FUSED),
                                                  (mm.BC_CPML, mm.SNAP_FP32, 1e-4, 1, mm.CPML_LAYER),
                                                  (mm.BC_CPML, mm.SNAP_FP32, 1e-4, 1, mm.CPML_FUSED)])
def test_gradient_matches_oracle(bc, snap, tol, fs, kern):
    """FWI gradient w.r.t. m = 1/v^2 with checkpoints every 16 steps (a partial
    last segment included) against the oracle's exact FP64 gradient; CPML
    checkpoints carry the layer memory, with either forward strategy in the
    forward run and the replays; with a free surface the receivers sit just
    below it."""
    rng = np.random.default_rng(30)
    shape = (28, 32, 36)
    nz, ny, nx = shape
    k = np.arange(nz)[:, None, None]
    v0 = ((2000.0 + 30.0 * k) * np.ones(shape)).astype(np.float32)
    vt = v0.copy()
    vt[6:16, 10:22, 12:26] += 400.0
    p = params(shape, bc=bc, nb=6, sigma=0.05, f0=25.0)
    p.vmax = float(vt.max())
    p.ckpt_every = 16
    p.snap = snap
    p.free_surface = fs
    p.cpml_kernel = kern
    T = 140
    p.nsteps_max = T
    dt = mm.dt_for(p, p.vmax)
    src = np.array([[18, 16, 4]], np.int32)
    rec = np.array([[i, j, 1 if fs else 3] for i in range(2, nx - 2, 3) for j in range(2, ny - 2, 3)], np.int32)
    w = mm.ricker(25.0, 0.06, dt, T).reshape(T, 1)
    g = grid_for(p, dt, p.vmax)
    d_obs, _, _, _ = C.forward(g, vt.astype(np.float64), src, w.astype(np.float64), rec, T)
    d_obs32 = d_obs.astype(np.float32)
    ref, ref_tr, ref_J = C.gradient(g, v0.astype(np.float64), src, w.astype(np.float64), rec,
                                    d_obs32.astype(np.float64), T, ckpt=16)
    ctx = mm.Context.single(p, torch.from_numpy(v0).to(DEV), src, rec)
    assert ctx.dt == dt
    grad = torch.empty(shape, device=DEV)
    tr = torch.empty((T, len(rec)), device=DEV)
    J = ctx.gradient(T, torch.from_numpy(w).to(DEV), torch.from_numpy(d_obs32).to(DEV), grad, tr)
    gg = grad.cpu().numpy()
    e = rel(gg, ref)
    cos = float(np.sum(gg * ref) / (np.linalg.norm(gg) * np.linalg.norm(ref)))
    print(f"bc={bc} snap={snap}: gradient rel L2 {e:.2e}, cosine {cos:.8f}, J {J:.6e} vs {ref_J:.6e}")
    assert rel(tr.cpu().numpy(), ref_tr) <= 1e-5
    assert abs(J - ref_J) <= 1e-4 * ref_J
    assert e <= tol
    if snap == mm.SNAP_BF16:
        assert cos >= 0.9999


def test_gradient_is_independent_of_cache_hints():
    """The CPML gradient (forward with checkpoints, replay, adjoint and
    imaging) with non-temporal loads forced on equals the one with them off,
    bitwise."""
    rng = np.random.default_rng(31)
    shape = (24, 28, 30)
    nz, ny, nx = shape
    v0 = rng.uniform(1800.0, 2600.0, shape).astype(np.float32)
    p = params(shape, bc=mm.BC_CPML, nb=5, f0=25.0)
    p.vmax = float(v0.max())
    p.ckpt_every = 8
    T = 60
    p.nsteps_max = T
    dt = mm.dt_for(p, p.vmax)
    src = np.array([[15, 14, 12]], np.int32)
    rec = np.array([[i, j, 3] for i in range(2, nx - 2, 4) for j in range(2, ny - 2, 4)], np.int32)
    w = torch.from_numpy(mm.ricker(25.0, 0.06, dt, T).reshape(T, 1)).to(DEV)
    d_obs = torch.from_numpy(rng.standard_normal((T, len(rec))).astype(np.float32) * 1e-3).to(DEV)
    res = []
    for h in (1, 2):
        p.cache_hints = h
        ctx = mm.Context.single(p, torch.from_numpy(v0).to(DEV), src, rec)
        grad = torch.empty(shape, device=DEV)
        tr = torch.empty((T, len(rec)), device=DEV)
        J = ctx.gradient(T, w, d_obs, grad, tr)
        res.append((J, grad.cpu().numpy(), tr.cpu().numpy()))
        ctx.close()
    assert res[0][0] == res[1][0]
    assert np.array_equal(res[0][1], res[1][1]) and np.array_equal(res[0][2], res[1][2])
    assert np.abs(res[0][1]).max() > 0


def test_autograd_binding_matches_library_gradient():
    """traces_from_slowness(m).backward(r) gives the library's gradient for
    J = 1/2 |traces - d_obs|^2 when r = traces - d_obs."""
    rng = np.random.default_rng(40)
    shape = (22, 24, 26)
    vel = rng.uniform(1800.0, 2600.0, shape).astype(np.float32)
    p = params(shape, bc=mm.BC_SPONGE, nb=5, sigma=0.05)
    p.ckpt_every = 8
    T = 50
    p.nsteps_max = T
    src = np.array([[13, 12, 4]], np.int32)
    rec = np.array([[i, 12, 3] for i in range(1, 25, 2)], np.int32)
    dt = mm.dt_for(p, float(vel.max()))
    w = torch.from_numpy(mm.ricker(25.0, 0.06, dt, T).reshape(T, 1)).to(DEV)
    d_obs = torch.from_numpy(rng.standard_normal((T, len(rec))).astype(np.float32) * 1e-7).to(DEV)
    m = (1.0 / torch.from_numpy(vel).to(DEV) ** 2).requires_grad_(True)
    with pytest.raises(ValueError):  # dt and vmax must be pinned
        mm.traces_from_slowness(m, w, p, src, rec)
    p.dt = dt
    p.vmax = float(vel.max())
    tr = mm.traces_from_slowness(m, w, p, src, rec)
    loss = 0.5 * ((tr - d_obs) ** 2).sum()
    loss.backward()
    ctx = mm.Context.single(p, torch.rsqrt(m.detach()).contiguous(), src, rec)
    grad = torch.empty(shape, device=DEV)
    tr2 = torch.empty((T, len(rec)), device=DEV)
    ctx.gradient(T, w, d_obs, grad, tr2)
    torch.cuda.synchronize()
    assert torch.equal(tr.detach(), tr2)
    assert rel(m.grad.cpu().numpy(), grad.cpu().numpy()) <= 1e-6


def test_batched_adjoint_equals_single_shot_adjoints():
    """Adjoint seismograms of a two-shot CPML context (one adjoint CPML and
    stencil launch per step for both shots) equal the single-shot runs."""
    rng = np.random.default_rng(50)
    shapes = [(24, 27, 30), (22, 26, 21)]
    p = params(shapes[0], bc=mm.BC_CPML, nb=5, f0=25.0)
    vels = [rng.uniform(1600.0, 2800.0, sh).astype(np.float32) for sh in shapes]
    p.vmax = float(max(v.max() for v in vels))
    T = 40
    p.ckpt_every = 8
    p.nsteps_max = T
    srcs = [np.array([[sh[2] // 2, sh[1] // 2, sh[0] // 2]], np.int32) for sh in shapes]
    recs = [np.array([[1, 2, 3], [sh[2] - 2, sh[1] - 3, 2], [6, 7, 8]], np.int32) for sh in shapes]
    ws = [rng.standard_normal((T, 1)).astype(np.float32) for _ in shapes]
    rs = [rng.standard_normal((T, 3)).astype(np.float32) for _ in shapes]
    ctx = mm.Context(p, [(torch.from_numpy(v).to(DEV), s_, r_) for v, s_, r_ in zip(vels, srcs, recs)])
    ctx.forward(T, torch.from_numpy(np.concatenate(ws, 1)).to(DEV))
    adj = torch.zeros((T, 2), device=DEV)
    ctx.adjoint(T, torch.from_numpy(np.concatenate(rs, 1)).to(DEV), adj)
    both = adj.cpu().numpy()
    for i, (v, s_, r_, w, r) in enumerate(zip(vels, srcs, recs, ws, rs)):
        q = mm.default_params(**{k: getattr(p, k) for k, _ in mm.Params._fields_})
        q.nz, q.ny, q.nx = v.shape
        c1 = mm.Context.single(q, torch.from_numpy(v).to(DEV), s_, r_)
        c1.forward(T, torch.from_numpy(w).to(DEV))
        a1 = torch.zeros((T, 1), device=DEV)
        c1.adjoint(T, torch.from_numpy(r).to(DEV), a1)
        assert np.array_equal(a1.cpu().numpy()[:, 0], both[:, i])


def test_cpml_adjoint_limits():
    """With adjoint storage, CPML needs nb <= 64 and n >= 2 nb + 8 per axis
    (its adjoint correction reaches 4 cells past each layer)."""
    vel = np.full((24, 24, 24), 2000.0, np.float32)
    vt = torch.from_numpy(vel).to(DEV)
    p = params(vel.shape, bc=mm.BC_CPML, nb=9)
    p.ckpt_every = 8
    p.nsteps_max = 10
    with pytest.raises(mm.MinimodError) as e:
        mm.Context.single(p, vt, [[8, 8, 8]], [[4, 4, 4]])
    assert e.value.status == mm.MM_ERR_ARG and "2*nb+8" in str(e.value)
    p.nb = 8
    ctx = mm.Context.single(p, vt, [[8, 8, 8]], [[4, 4, 4]])
    ctx.forward(4, torch.ones((4, 1), device=DEV))
    ctx.adjoint(4, torch.zeros((4, 1), device=DEV))
    ctx.close()
    p.ckpt_every = 0
    p.nb = 10  # forward only: 2 nb + 4 suffices
    mm.Context.single(p, vt, [[8, 8, 8]], [[4, 4, 4]]).close()


def test_graph_captured_without_checkpoints_is_not_reused_for_a_checkpointed_run():
    """A graph captured for steps that store no checkpoints (a run starting
    at step 2 that would overrun nsteps_max) is not replayed for a run from
    step 0, which must store them: after reset, the graph run's checkpoints
    give the same gradient as mm_gradient."""
    rng = np.random.default_rng(41)
    shape = (20, 22, 24)
    vel = rng.uniform(1800.0, 2600.0, shape).astype(np.float32)
    p = params(shape, bc=mm.BC_CPML, nb=4, f0=25.0)
    p.ckpt_every = 8
    T = 40
    p.nsteps_max = T
    src = np.array([[12, 11, 10]], np.int32)
    rec = np.array([[i, 11, 3] for i in range(1, 23, 3)], np.int32)
    vt = torch.from_numpy(vel).to(DEV)
    ctx = mm.Context.single(p, vt, src, rec)
    dt = ctx.dt
    w = torch.from_numpy(mm.ricker(25.0, 0.06, dt, T + 2).reshape(T + 2, 1)).to(DEV)
    d_obs = torch.from_numpy(rng.standard_normal((T, len(rec))).astype(np.float32) * 1e-6).to(DEV)
    tr = torch.empty((T, len(rec)), device=DEV)
    ctx.forward(2, w[:2])
    ctx.forward(T, w[:T], tr, graph=True)  # steps 2 .. T + 1: past nsteps_max, no checkpoints
    ctx.reset()
    ctx.forward(T, w[:T], tr, graph=True)  # from step 0: checkpoints stored
    g1 = torch.zeros(shape, device=DEV)
    ctx.adjoint(T, (tr - d_obs).contiguous(), None, g1)
    c2 = mm.Context.single(p, vt, src, rec)
    g2 = torch.empty(shape, device=DEV)
    tr2 = torch.empty_like(tr)
    c2.gradient(T, w[:T].contiguous(), d_obs, g2, tr2)
    torch.cuda.synchronize()
    assert torch.equal(tr, tr2)
    assert float(g2.abs().max()) > 0
    assert rel(g1.cpu().numpy(), g2.cpu().numpy()) <= 1e-6
