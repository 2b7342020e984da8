"""mm_init_static (contexts in the library's static per-GPU workspace, for
callers that cannot allocate) against mm_init with a caller workspace: the
same kernels on the same inputs, so traces and final state agree bit for bit;
two static contexts in a row on one GPU, the second on a smaller problem
(the array keeps the first call's contents, which the second must clear);
torch allocates nothing while the static context is made and run; the
earlier static context is refused once a later one took the array over;
problems larger than the array are refused."""
import numpy as np
import pytest
import torch

from paper_2007_06048_amd import minimod as mm

from .gpu_util import DEV, params

pytestmark = pytest.mark.gpu


def _case(shape, bc, seed):
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    vel = rng.uniform(1500.0, 3200.0, shape).astype(np.float32)
    src = np.array([[nx // 2, ny // 2, nz // 2], [3, 4, 5]], dtype=np.int32)
    rec = np.array([[i, j, 3] for i in range(1, nx, 4) for j in range(2, ny, 5)], dtype=np.int32)
    p = params(shape, h=(10.0, 11.0, 9.0), bc=bc, nb=6, f0=20.0)
    T = 50
    dt = mm.dt_for(p, float(vel.max()))
    w = rng.standard_normal((T, len(src))).astype(np.float32)
    return p, vel, src, rec, w, T


def _run(ctx, vel_shape, T, w, nrec):
    tr = torch.zeros((T, nrec), dtype=torch.float32, device=DEV)
    ctx.forward(T, torch.from_numpy(w).to(DEV), tr)
    st = ctx.get_state()
    torch.cuda.synchronize()
    return tr.cpu().numpy(), st.cpu().numpy()


def test_static_context_matches_workspace_context_twice():
    first = None
    for shape, bc, seed in (((36, 40, 44), mm.BC_CPML, 1), ((23, 29, 37), mm.BC_SPONGE, 2)):
        p, vel, src, rec, w, T = _case(shape, bc, seed)
        v = torch.from_numpy(vel).to(DEV)
        ref_ctx = mm.Context.single(p, v, src, rec)
        ref = _run(ref_ctx, shape, T, w, len(rec))
        nstate = ref_ctx.state_size() // 4
        ref_ctx.close()
        wt = torch.from_numpy(w).to(DEV)
        tr = torch.zeros((T, len(rec)), dtype=torch.float32, device=DEV)
        st = torch.empty(nstate, dtype=torch.float32, device=DEV)
        torch.cuda.synchronize()
        # cumulative count of torch allocator requests (frees of older tensors do not move it)
        before = torch.cuda.memory_stats(DEV)["allocation.all.allocated"]
        sctx = mm.Context.static(p, v, src, rec)
        sctx.forward(T, wt, tr)
        mm._check(mm.load().mm_get_state(sctx.h, mm._ptr(st)), sctx.h)
        torch.cuda.synchronize()
        # making and running the static context allocated nothing through torch
        assert torch.cuda.memory_stats(DEV)["allocation.all.allocated"] == before
        assert np.array_equal(tr.cpu().numpy(), ref[0])
        assert np.array_equal(st.cpu().numpy(), ref[1])
        # a second run from reset on the same static context
        sctx.reset()
        tr2 = torch.zeros_like(tr)
        sctx.forward(T, torch.from_numpy(w).to(DEV), tr2)
        torch.cuda.synchronize()
        assert np.array_equal(tr2.cpu().numpy(), ref[0])
        if first is not None:
            # the first static context lost the array to this one
            with pytest.raises(mm.MinimodError) as ei:
                first.forward(1, torch.from_numpy(w[:1]).to(DEV), None)
            assert ei.value.status == mm.MM_ERR_STATE
            first.close()
        first = sctx
    first.close()


def test_static_context_size_limit():
    shape = (256, 256, 256)  # 16.8 M points: three fields alone exceed 64 MiB
    p = params(shape, bc=mm.BC_SPONGE, nb=8)
    v = torch.full(shape, 2000.0, dtype=torch.float32, device=DEV)
    with pytest.raises(mm.MinimodError) as ei:
        mm.Context.static(p, v, [[1, 1, 1]], [[2, 2, 2]])
    assert ei.value.status == mm.MM_ERR_WORKSPACE
    assert "static workspace" in str(ei.value)
