"""C-ABI contract on the CPU: the library loads, exports every function the
header declares, and its host-only logic (argument checks, stability limit,
wavelet, workspace sizing) behaves as documented.  No kernel is launched."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import c_oracle as C
from paper_2007_06048_amd import minimod as mm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    with open(os.path.join(ROOT, "include", "minimod.h")) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mm_[a-z_0-9]+)\s*\(", text)))


def test_every_declared_symbol_is_exported_and_bound():
    lib = mm.load()
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(mm.SYMBOLS) == names


def test_status_strings():
    lib = mm.load()
    for s in range(8):
        assert lib.mm_status_str(s).decode() not in ("", "unknown status")
    assert lib.mm_status_str(99).decode() == "unknown status"


def test_dt_matches_stability_limit_and_rejects_unstable():
    p = mm.default_params(dx=10.0, dy=12.0, dz=8.0, cfl=0.5)
    for vmax in (1500.0, 4500.0):
        want = 0.5 * C.dt_stab(vmax, 10.0, 12.0, 8.0)
        assert mm.dt_for(p, vmax) == pytest.approx(want, rel=1e-15)
    p.cfl = 1.0
    assert mm.dt_for(p, 3000.0) == pytest.approx(C.dt_stab(3000.0, 10.0, 12.0, 8.0), rel=1e-15)
    p.cfl = 1.01
    with pytest.raises(mm.MinimodError) as e:
        mm.dt_for(p, 3000.0)
    assert e.value.status == mm.MM_ERR_UNSTABLE
    p.cfl = 0.5
    p.dt = 1.001 * C.dt_stab(3000.0, 10.0, 12.0, 8.0)
    with pytest.raises(mm.MinimodError) as e:
        mm.dt_for(p, 3000.0)
    assert e.value.status == mm.MM_ERR_UNSTABLE
    p.dt = 1e-4
    assert mm.dt_for(p, 3000.0) == 1e-4
    for bad in (dict(dx=0.0), dict(dy=-1.0), dict(dz=float("nan")), dict(bc=7), dict(nb=-1)):
        q = mm.default_params(**bad)
        with pytest.raises(mm.MinimodError) as e:
            mm.dt_for(q, 3000.0)
        assert e.value.status == mm.MM_ERR_ARG
    with pytest.raises(mm.MinimodError):
        mm.dt_for(mm.default_params(), 0.0)


def test_ricker_matches_oracle_wavelet():
    for f0, t0, dt in ((15.0, 0.1, 9.0571e-4), (20.0, 0.075, 5.0317e-4), (10.0, 0.15, 1e-3)):
        got = mm.ricker(f0, t0, dt, 500)
        want = C.ricker(f0, t0, dt, 500)
        assert np.array_equal(got, want.astype(np.float32))


def _shot(nx, ny, nz, src, rec, vel=1 << 12):
    s = np.ascontiguousarray(np.asarray(src, np.int32).reshape(-1, 3))
    r = np.ascontiguousarray(np.asarray(rec, np.int32).reshape(-1, 3))
    sh = mm.Shot(nx, ny, nz, vel, s.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), len(s),
                 r.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), len(r))
    return sh, (s, r)


def _ws(p, shots):
    arr = (mm.Shot * len(shots))(*shots)
    n = ctypes.c_size_t()
    st = mm.load().mm_workspace_size(ctypes.byref(p), len(shots), arr, ctypes.byref(n))
    return st, n.value


def test_workspace_size_and_argument_checks():
    p = mm.default_params(bc=mm.BC_CPML, nb=10)
    s, keep = _shot(64, 48, 40, [[5, 5, 5]], [[1, 2, 3], [63, 47, 39]])
    st, n = _ws(p, [s])
    assert st == mm.MM_OK and n % 256 == 0
    # three fields of 64*48*40 floats plus six CPML slab arrays at least
    assert n >= 3 * 4 * 64 * 48 * 40 + 6 * 4 * 20 * (48 * 40 + 64 * 40 + 64 * 48) // 3
    p2 = mm.default_params(bc=mm.BC_CPML, nb=10, ckpt_every=16, nsteps_max=100)
    st, n2 = _ws(p2, [s])
    assert st == mm.MM_OK and n2 > n + 16 * 4 * 64 * 48 * 40  # segment buffer and checkpoints
    # layer too wide for the grid
    p3 = mm.default_params(bc=mm.BC_CPML, nb=20)
    st, _ = _ws(p3, [s])
    assert st == mm.MM_ERR_ARG
    assert "2*nb+4" in mm.load().mm_last_error(None).decode()
    # with adjoint storage the CPML adjoint needs two stencil radii between the layers, and nb <= 64
    p4 = mm.default_params(bc=mm.BC_CPML, nb=17, ckpt_every=8, nsteps_max=10)
    st, _ = _ws(p4, [s])
    assert st == mm.MM_ERR_ARG and "2*nb+8" in mm.load().mm_last_error(None).decode()
    p4.nb = 16
    assert _ws(p4, [s])[0] == mm.MM_OK
    big, keep5 = _shot(200, 200, 200, [[5, 5, 5]], [[1, 2, 3]])
    p4.nb = 65
    st, _ = _ws(p4, [big])
    assert st == mm.MM_ERR_ARG and "64" in mm.load().mm_last_error(None).decode()
    # receiver outside the grid
    bad, keep2 = _shot(64, 48, 40, [[5, 5, 5]], [[64, 0, 0]])
    st, _ = _ws(p, [bad])
    assert st == mm.MM_ERR_ARG and "receiver" in mm.load().mm_last_error(None).decode()
    # zero shots, bad sizes
    st, _ = _ws(p, [])
    assert st == mm.MM_ERR_ARG
    zero, keep3 = _shot(0, 48, 40, [], [])
    st, _ = _ws(p, [zero])
    assert st == mm.MM_ERR_ARG
    # batch: size grows with every shot
    s2, keep4 = _shot(30, 30, 30, [[1, 1, 1]], [[2, 2, 2]])
    st, nb2 = _ws(p, [s, s2])
    assert st == mm.MM_OK and nb2 > n


def test_acoustic_iso_dt_workspace_and_argument_checks():
    """acoustic_iso on the host side: its dt uses the staggered scheme's
    limit (the oracle's, not the constant-density one), its workspace holds
    the ping-pong pressure, three face velocities, dt rho v^2 and rho / dt,
    with CPML also the memory of the face and cell derivatives (slabs one
    cell wider than the layer), and adjoint storage is refused."""
    p = mm.default_params(dx=10.0, dy=12.0, dz=8.0, cfl=0.5, model=mm.MODEL_ISO, bc=mm.BC_SPONGE, nb=4)
    assert mm.dt_for(p, 3000.0) == pytest.approx(0.5 * C.iso_dt_stab(3000.0, 10.0, 12.0, 8.0), rel=1e-15)
    assert mm.dt_for(p, 3000.0) < mm.dt_for(mm.default_params(dx=10.0, dy=12.0, dz=8.0, cfl=0.5), 3000.0)
    s, keep = _shot(40, 36, 32, [[5, 5, 5]], [[1, 2, 3]])
    st, n_iso = _ws(p, [s])
    assert st == mm.MM_OK and n_iso >= 7 * 4 * 40 * 36 * 32
    st, n_cd = _ws(mm.default_params(dx=10.0, dy=12.0, dz=8.0, cfl=0.5, bc=mm.BC_SPONGE, nb=4), [s])
    assert st == mm.MM_OK and n_iso - n_cd >= 4 * 4 * 40 * 36 * 32
    q = mm.default_params(dx=10.0, dy=12.0, dz=8.0, cfl=0.5, model=mm.MODEL_ISO, bc=mm.BC_CPML, nb=4)
    st, n_pml = _ws(q, [s])
    w2 = 2 * (4 + 1)
    slabs = 32 * 36 * w2 + 32 * w2 * 40 + w2 * 36 * 40
    assert st == mm.MM_OK and n_pml - n_iso >= 2 * 4 * slabs
    q = mm.default_params(model=mm.MODEL_ISO, bc=mm.BC_SPONGE, nb=4, nsteps_max=10, ckpt_every=8)
    st, _ = _ws(q, [s])
    assert st == mm.MM_ERR_UNSUPPORTED
    q = mm.default_params(model=2)
    assert _ws(q, [s])[0] == mm.MM_ERR_ARG
    for bad in (-1, 3):
        q = mm.default_params(cache_hints=bad)
        assert _ws(q, [s])[0] == mm.MM_ERR_ARG
        assert "cache_hints" in mm.load().mm_last_error(None).decode()


def test_init_rejects_bad_workspace_before_touching_the_device():
    p = mm.default_params(nx=32, ny=32, nz=32, bc=mm.BC_SPONGE, nb=8)
    s, keep = _shot(32, 32, 32, [[5, 5, 5]], [[1, 2, 3]])
    st, need = _ws(p, [s])
    assert st == mm.MM_OK
    lib = mm.load()
    arr = (mm.Shot * 1)(s)
    h = ctypes.c_void_p()
    for ptr, size in ((0, need), (4096 + 16, need), (4096, need - 256)):
        st = lib.mm_init_batch(ctypes.byref(h), ctypes.byref(p), 1, arr, ctypes.c_void_p(ptr), size, None)
        assert st == mm.MM_ERR_WORKSPACE, (ptr, size)
        assert not h.value
    p.cfl = 1.5
    st = lib.mm_init_batch(ctypes.byref(h), ctypes.byref(p), 1, arr, ctypes.c_void_p(4096), need, None)
    assert st == mm.MM_ERR_UNSTABLE


def test_tile_table():
    n = mm.num_tiles()
    assert n >= 6
    names = [mm.tile_name(t) for t in range(n)]
    assert len(set(names)) == n
    assert mm.tile_name(n) == "?"


def test_binding_never_reaches_the_oracle():
    """The product binding does not import or load the test oracle: there is
    no CPU path for it to fall back to."""
    import paper_2007_06048_amd.minimod as b
    src = open(b.__file__).read()
    assert "import oracle" not in src and "from oracle" not in src and "liboracle" not in src
