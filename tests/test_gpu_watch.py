"""The optional watchdog (mm_params.watch_every): scanning the wavefield for
NaN or Inf every K steps leaves the run bitwise unchanged and reports
nothing on a finite run; a non-finite wavelet sample is reported as
MM_ERR_NONFINITE with the first scanned state that holds it (by mm_watch
and by mm_gradient); mm_reset clears the finding."""
import numpy as np
import pytest
import torch

from paper_2007_06048_amd import minimod as mm

from .gpu_util import DEV, params

pytestmark = pytest.mark.gpu


def _setup(bc, watch, seed=7, **kw):
    rng = np.random.default_rng(seed)
    shape = (26, 30, 34)
    vel = rng.uniform(1500.0, 3000.0, shape).astype(np.float32)
    src = np.array([[17, 15, 13]], np.int32)
    rec = np.array([[i, 9, 4] for i in range(2, 32, 3)], np.int32)
    p = params(shape, bc=bc, nb=6, f0=20.0, **kw)
    p.watch_every = watch
    ctx = mm.Context.single(p, torch.from_numpy(vel).to(DEV), src, rec)
    return ctx, rng, rec


@pytest.mark.parametrize("bc", [mm.BC_SPONGE, mm.BC_CPML])
def test_watchdog_leaves_a_finite_run_alone(bc):
    out = []
    T = 60
    for watch in (0, 7):
        ctx, rng, rec = _setup(bc, watch)
        w = torch.from_numpy(rng.standard_normal((T, 1)).astype(np.float32)).to(DEV)
        tr = torch.zeros((T, len(rec)), device=DEV)
        ctx.forward(T, w, tr)
        if watch:
            assert ctx.watch() is None
        else:
            with pytest.raises(mm.MinimodError) as e:
                ctx.watch()
            assert e.value.status == mm.MM_ERR_STATE
        out.append((tr.cpu().numpy(), ctx.get_state().cpu().numpy()))
        ctx.close()
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])


@pytest.mark.parametrize("bc", [mm.BC_SPONGE, mm.BC_CPML])
def test_watchdog_reports_the_first_scanned_bad_state(bc):
    ctx, rng, rec = _setup(bc, 4)
    T = 30
    w = rng.standard_normal((T, 1)).astype(np.float32)
    w[5, 0] = np.inf  # enters p^6; the states after steps 4, 8, ... are scanned
    ctx.forward(T, torch.from_numpy(w).to(DEV), None)
    assert ctx.watch() == 8
    ctx.reset()
    assert ctx.watch() is None
    ctx.forward(3, torch.from_numpy(w[:3]).to(DEV), None)
    assert ctx.watch() is None
    ctx.close()


def test_gradient_reports_a_non_finite_forward_run():
    ctx, rng, rec = _setup(mm.BC_SPONGE, 5, ckpt_every=8, nsteps_max=40)
    T = 40
    w = rng.standard_normal((T, 1)).astype(np.float32)
    d_obs = torch.zeros((T, len(rec)), device=DEV)
    g = torch.empty((26, 30, 34), device=DEV)
    ctx.gradient(T, torch.from_numpy(w).to(DEV), d_obs, g)  # finite: no error
    w[12, 0] = np.nan
    with pytest.raises(mm.MinimodError) as e:
        ctx.gradient(T, torch.from_numpy(w).to(DEV), d_obs, g)
    assert e.value.status == mm.MM_ERR_NONFINITE and "step 15" in str(e.value)
    ctx.close()
