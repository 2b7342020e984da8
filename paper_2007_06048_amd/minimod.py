"""Thin ctypes binding of libminimod.so (C ABI in include/minimod.h).

Argument marshalling only: every step of the propagator runs in the
library's HIP kernels.  PyTorch supplies device memory (workspace, fields,
traces, gradients as CUDA tensors) and the stream (the current torch stream).
The library must be built (`__graft_entry__.build()`); loading fails loudly
otherwise, and nothing here falls back to a CPU implementation.
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libminimod.so")

MM_OK, MM_ERR_ARG, MM_ERR_UNSTABLE, MM_ERR_WORKSPACE, MM_ERR_DEVICE, MM_ERR_STATE, MM_ERR_NONFINITE, \
    MM_ERR_UNSUPPORTED = range(8)
BC_NONE, BC_SPONGE, BC_CPML = 0, 1, 2
MODEL_ISO_CD, MODEL_ISO = 0, 1
SNAP_FP32, SNAP_BF16 = 0, 1
CPML_AUTO, CPML_LAYER, CPML_FUSED = 0, 1, 2

# every symbol declared in include/minimod.h
SYMBOLS = [
    "mm_default_params", "mm_dt", "mm_ricker", "mm_workspace_size", "mm_init_batch", "mm_init",
    "mm_forward_steps", "mm_forward_steps_graph", "mm_adjoint_steps", "mm_gradient", "mm_reset",
    "mm_state_size", "mm_get_state", "mm_set_state", "mm_get_info", "mm_autotune", "mm_set_tile",
    "mm_num_tiles", "mm_tile_name", "mm_profile", "mm_profile_read", "mm_destroy", "mm_status_str",
    "mm_last_error", "mm_snap_blocks", "mm_snap_encode", "mm_snap_decode", "mm_init_static", "mm_watch",
    "mm_get_cpml_kernel",
]


class Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dz", ctypes.c_double),
        ("dt", ctypes.c_double), ("cfl", ctypes.c_double), ("vmax", ctypes.c_double),
        ("bc", ctypes.c_int32), ("nb", ctypes.c_int32),
        ("sponge_sigma", ctypes.c_double), ("cpml_R", ctypes.c_double), ("cpml_f0", ctypes.c_double),
        ("ckpt_every", ctypes.c_int32), ("snap", ctypes.c_int32), ("nsteps_max", ctypes.c_int32),
        ("tile", ctypes.c_int32), ("group_kb", ctypes.c_int32),
        ("free_surface", ctypes.c_int32), ("model", ctypes.c_int32), ("cache_hints", ctypes.c_int32),
        ("watch_every", ctypes.c_int32), ("cpml_kernel", ctypes.c_int32),
    ]


class Shot(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("vel", ctypes.c_void_p),
        ("src_ijk", ctypes.POINTER(ctypes.c_int32)), ("nsrc", ctypes.c_int32),
        ("rec_ijk", ctypes.POINTER(ctypes.c_int32)), ("nrec", ctypes.c_int32),
        ("rho", ctypes.c_void_p),
    ]


class MinimodError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_status_name(status)}: {msg}")
        self.status = status


_lib = None


def load():
    """Load libminimod.so and declare the signatures.  Raises if missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library not built: {LIB_PATH} (run __graft_entry__.build())")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
    pp = ctypes.POINTER(Params)
    st = ctypes.c_int
    sig = {
        "mm_default_params": (None, [pp]),
        "mm_dt": (st, [pp, dbl, ctypes.POINTER(dbl)]),
        "mm_ricker": (st, [dbl, dbl, dbl, i32, ctypes.POINTER(ctypes.c_float)]),
        "mm_workspace_size": (st, [pp, i32, ctypes.POINTER(Shot), ctypes.POINTER(ctypes.c_size_t)]),
        "mm_init_batch": (st, [ctypes.POINTER(vp), pp, i32, ctypes.POINTER(Shot), vp, ctypes.c_size_t, vp]),
        "mm_init": (st, [ctypes.POINTER(vp), pp, vp, ctypes.POINTER(i32), i32, ctypes.POINTER(i32), i32, vp,
                         ctypes.c_size_t, vp]),
        "mm_forward_steps": (st, [vp, i32, vp, vp]),
        "mm_forward_steps_graph": (st, [vp, i32, vp, vp]),
        "mm_adjoint_steps": (st, [vp, i32, vp, vp, vp]),
        "mm_gradient": (st, [vp, i32, vp, vp, vp, vp, ctypes.POINTER(dbl)]),
        "mm_reset": (st, [vp]),
        "mm_state_size": (st, [vp, ctypes.POINTER(ctypes.c_size_t)]),
        "mm_get_state": (st, [vp, vp]),
        "mm_set_state": (st, [vp, vp, i32]),
        "mm_get_info": (st, [vp, ctypes.POINTER(dbl), ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32)]),
        "mm_get_cpml_kernel": (st, [vp, ctypes.POINTER(i32)]),
        "mm_autotune": (st, [vp, i32, ctypes.POINTER(i32)]),
        "mm_set_tile": (st, [vp, i32]),
        "mm_profile": (st, [vp, i32]),
        "mm_profile_read": (st, [vp, ctypes.POINTER(dbl), ctypes.POINTER(i32)]),
        "mm_num_tiles": (i32, []),
        "mm_tile_name": (ctypes.c_char_p, [i32]),
        "mm_destroy": (None, [vp]),
        "mm_status_str": (ctypes.c_char_p, [st]),
        "mm_last_error": (ctypes.c_char_p, [vp]),
        "mm_snap_blocks": (ctypes.c_int64, [ctypes.c_int64]),
        "mm_watch": (st, [vp, ctypes.POINTER(i32)]),
        "mm_init_static": (st, [ctypes.POINTER(vp), pp, vp, ctypes.POINTER(i32), i32, ctypes.POINTER(i32), i32, vp]),
        "mm_snap_encode": (st, [vp, vp, ctypes.c_int64, vp, vp, vp, vp, vp]),
        "mm_snap_decode": (st, [vp, vp, vp, vp, ctypes.c_int64, vp, vp, vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _status_name(s):
    try:
        return load().mm_status_str(s).decode()
    except Exception:
        return f"status {s}"


def _check(status, ctx=None):
    if status != MM_OK:
        msg = load().mm_last_error(ctx).decode()
        raise MinimodError(status, msg)


def default_params(**kw):
    p = Params()
    load().mm_default_params(ctypes.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise AttributeError(k)
        setattr(p, k, v)
    return p


def dt_for(params, vmax):
    out = ctypes.c_double()
    _check(load().mm_dt(ctypes.byref(params), float(vmax), ctypes.byref(out)))
    return out.value


def ricker(f0, t0, dt, n):
    import numpy as np
    out = np.zeros(n, dtype=np.float32)
    _check(load().mm_ricker(f0, t0, dt, n, out.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
    return out


def _pts(a):
    import numpy as np
    a = np.ascontiguousarray(np.asarray(a, dtype=np.int32).reshape(-1, 3))
    return a


def _ptr(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


class Context:
    """A propagator over one or more shots (sub-volumes) sharing spacing, dt,
    boundary and width.  `shots` is a list of (vel, src, rec) or (vel, src,
    rec, rho) where vel (and rho, the density of an acoustic_iso model) is a
    float32 CUDA tensor [nz][ny][nx] and src/rec are (n, 3) int arrays of
    (i, j, k) cells."""

    def __init__(self, params, shots, stream=None):
        import torch
        lib = load()
        self.params = params
        self._keep = []
        arr = (Shot * len(shots))()
        self.nsrc = self.nrec = 0
        self.shapes = []
        for i, shot in enumerate(shots):
            vel, src, rec = shot[:3]
            rho = shot[3] if len(shot) > 3 else None
            assert vel.is_cuda and vel.dtype == torch.float32 and vel.is_contiguous() and vel.dim() == 3
            if rho is not None:
                assert rho.is_cuda and rho.dtype == torch.float32 and rho.is_contiguous() and rho.shape == vel.shape
            nz, ny, nx = vel.shape
            s, r = _pts(src), _pts(rec)
            self._keep += [vel, s, r, rho]
            arr[i] = Shot(nx, ny, nz, vel.data_ptr(), s.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), len(s),
                          r.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), len(r),
                          rho.data_ptr() if rho is not None else None)
            self.nsrc += len(s)
            self.nrec += len(r)
            self.shapes.append((nz, ny, nx))
        self.device = shots[0][0].device
        self.iso = params.model == MODEL_ISO
        nbytes = ctypes.c_size_t()
        _check(lib.mm_workspace_size(ctypes.byref(params), len(shots), arr, ctypes.byref(nbytes)))
        self.ws_bytes = nbytes.value
        self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        _check(lib.mm_init_batch(ctypes.byref(h), ctypes.byref(params), len(shots), arr,
                                 ctypes.c_void_p(self.workspace.data_ptr()), self.ws_bytes,
                                 ctypes.c_void_p(self.stream.cuda_stream)))
        self.h = h

    @classmethod
    def single(cls, params, vel, src, rec, stream=None, rho=None):
        return cls(params, [(vel, src, rec) if rho is None else (vel, src, rec, rho)], stream)

    @classmethod
    def static(cls, params, vel, src, rec, stream=None):
        """A single-shot context in the library's static per-GPU workspace
        (mm_init_static): no device allocation here or in the library."""
        import torch
        self = cls.__new__(cls)
        assert vel.is_cuda and vel.dtype == torch.float32 and vel.is_contiguous() and vel.dim() == 3
        s, r = _pts(src), _pts(rec)
        self.params = params
        self._keep = [vel, s, r]
        self.nsrc, self.nrec = len(s), len(r)
        self.shapes = [tuple(vel.shape)]
        self.device = vel.device
        self.iso = params.model == MODEL_ISO
        self.ws_bytes = 0
        self.workspace = None
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        _check(load().mm_init_static(ctypes.byref(h), ctypes.byref(params), ctypes.c_void_p(vel.data_ptr()),
                                     s.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), len(s),
                                     r.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), len(r),
                                     ctypes.c_void_p(self.stream.cuda_stream)))
        self.h = h
        return self

    def __del__(self):
        h = getattr(self, "h", None)
        if h and _lib is not None:
            _lib.mm_destroy(h)
            self.h = None

    def close(self):
        self.__del__()

    # --------------------------------------------------------------- steps
    def forward(self, nsteps, wavelet=None, traces=None, graph=False):
        f = load().mm_forward_steps_graph if graph else load().mm_forward_steps
        _check(f(self.h, nsteps, _ptr(wavelet), _ptr(traces)), self.h)

    def adjoint(self, nsteps, resid, adj_src=None, grad=None):
        _check(load().mm_adjoint_steps(self.h, nsteps, _ptr(resid), _ptr(adj_src), _ptr(grad)), self.h)

    def gradient(self, nsteps, wavelet, d_obs, grad, traces=None):
        loss = ctypes.c_double()
        _check(load().mm_gradient(self.h, nsteps, _ptr(wavelet), _ptr(d_obs), _ptr(grad), _ptr(traces),
                                  ctypes.byref(loss)), self.h)
        return loss.value

    def reset(self):
        _check(load().mm_reset(self.h), self.h)

    def state_size(self):
        n = ctypes.c_size_t()
        _check(load().mm_state_size(self.h, ctypes.byref(n)), self.h)
        return n.value

    def get_state(self):
        import torch
        out = torch.empty(self.state_size() // 4, dtype=torch.float32, device=self.device)
        _check(load().mm_get_state(self.h, _ptr(out)), self.h)
        return out

    def set_state(self, state, step):
        _check(load().mm_set_state(self.h, _ptr(state), step), self.h)

    def info(self):
        dt, step, tile, ng = ctypes.c_double(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(load().mm_get_info(self.h, ctypes.byref(dt), ctypes.byref(step), ctypes.byref(tile),
                                  ctypes.byref(ng)), self.h)
        return {"dt": dt.value, "step": step.value, "tile": tile.value, "groups": ng.value}

    @property
    def dt(self):
        return self.info()["dt"]

    def cpml_kernel(self):
        """The forward CPML strategy in use: CPML_LAYER or CPML_FUSED (CPML_AUTO
        for other boundaries and acoustic_iso)."""
        k = ctypes.c_int32()
        _check(load().mm_get_cpml_kernel(self.h, ctypes.byref(k)), self.h)
        return k.value

    def autotune(self, steps=3):
        t = ctypes.c_int32()
        _check(load().mm_autotune(self.h, steps, ctypes.byref(t)), self.h)
        return t.value

    def set_tile(self, t):
        _check(load().mm_set_tile(self.h, t), self.h)

    def watch(self):
        """Watchdog result: the first step whose wavefield held NaN or Inf, or
        None (mm_watch; synchronises)."""
        bad = ctypes.c_int32()
        st = load().mm_watch(self.h, ctypes.byref(bad))
        if st == MM_ERR_NONFINITE:
            return bad.value
        _check(st, self.h)
        return None

    def profile(self, stride):
        _check(load().mm_profile(self.h, stride), self.h)

    def profile_read(self):
        ms, n = ctypes.c_double(), ctypes.c_int32()
        _check(load().mm_profile_read(self.h, ctypes.byref(ms), ctypes.byref(n)), self.h)
        return ms.value, n.value


def num_tiles():
    return load().mm_num_tiles()


def tile_name(t):
    return load().mm_tile_name(t).decode()


# ----------------------------------------------------------------- autograd

def snap_encode(prev, cur):
    """BF16 snapshot codec (mm_snap_encode) of two float32 CUDA tensors of
    the same size: returns (c0, c1) as int16 tensors holding the bfloat16
    bit patterns and the block scales (s0, s1)."""
    import torch
    n = prev.numel()
    nb = load().mm_snap_blocks(n)
    c0 = torch.empty(n, dtype=torch.int16, device=prev.device)
    c1 = torch.empty_like(c0)
    s0 = torch.empty(max(nb, 1), dtype=torch.float32, device=prev.device)
    s1 = torch.empty_like(s0)
    st = ctypes.c_void_p(torch.cuda.current_stream(prev.device).cuda_stream)
    _check(load().mm_snap_encode(_ptr(prev), _ptr(cur), n, _ptr(c0), _ptr(c1), _ptr(s0), _ptr(s1), st))
    return c0, c1, s0[:nb], s1[:nb]


def snap_decode(c0, c1, s0, s1):
    """Inverse of snap_encode: returns (prev, cur) as float32 tensors."""
    import torch
    n = c0.numel()
    prev = torch.empty(n, dtype=torch.float32, device=c0.device)
    cur = torch.empty_like(prev)
    st = ctypes.c_void_p(torch.cuda.current_stream(c0.device).cuda_stream)
    _check(load().mm_snap_decode(_ptr(c0), _ptr(c1), _ptr(s0), _ptr(s1), n, _ptr(prev), _ptr(cur), st))
    return prev, cur


def _make_traces_fn():
    import torch

    class TracesFromSlowness(torch.autograd.Function):
        """traces = F(m), m = 1/v^2 (squared slowness), for a single shot.

        forward builds a gradient-capable context from v = m^{-1/2}, runs the
        checkpointed forward and returns the receiver traces [nsteps][nrec];
        backward runs the library's adjoint with the incoming trace gradient as
        the residual and returns dL/dm (the imaging condition).

        The gradient is taken at a fixed time step and fixed boundary
        profiles, so params.dt (> 0) and params.vmax (> 0, the velocity of the
        CPML damping and of the stability check) must be set: were they
        derived from max(m^{-1/2}), they would move with m under a wavelet
        sampled at the old dt, and the returned gradient would not include
        that dependence.  ValueError otherwise."""

        @staticmethod
        def forward(ctx, m, wavelet, params, src, rec):
            if not (params.dt > 0.0 and params.vmax > 0.0):
                raise ValueError("traces_from_slowness needs params.dt > 0 and params.vmax > 0: dt and the "
                                 "CPML profiles are held fixed while m changes")
            vel = torch.rsqrt(m).contiguous()
            nsteps = wavelet.shape[0]
            p = Params.from_buffer_copy(params)
            p.nsteps_max = max(p.nsteps_max, nsteps)
            if p.ckpt_every <= 0:
                p.ckpt_every = 32
            c = Context.single(p, vel, src, rec)
            traces = torch.empty((nsteps, c.nrec), dtype=torch.float32, device=m.device)
            c.forward(nsteps, wavelet.contiguous(), traces)
            ctx.c = c
            ctx.nsteps = nsteps
            ctx.shape = m.shape
            return traces

        @staticmethod
        def backward(ctx, gtr):
            c = ctx.c
            g = torch.zeros(ctx.shape, dtype=torch.float32, device=gtr.device)
            c.adjoint(ctx.nsteps, gtr.contiguous().float(), None, g)
            ctx.c = None
            return g, None, None, None, None

    return TracesFromSlowness


_traces_fn = None


def traces_from_slowness(m, wavelet, params, src, rec):
    """Differentiable forward modelling: receiver traces as a function of the
    squared slowness m (CUDA float32 [nz][ny][nx]); see TracesFromSlowness."""
    global _traces_fn
    if _traces_fn is None:
        _traces_fn = _make_traces_fn()
    return _traces_fn.apply(m, wavelet, params, src, rec)
