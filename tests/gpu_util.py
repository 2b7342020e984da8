"""Helpers shared by the GPU tests: run the HIP library and the FP64 oracle
on the same seeded inputs."""
import numpy as np
import torch

from oracle import c_oracle as C
from paper_2007_06048_amd import minimod as mm

DEV = torch.device("cuda:0")


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def params(shape, h=(10.0, 10.0, 10.0), bc=mm.BC_SPONGE, nb=8, cfl=0.5, f0=15.0, sigma=0.015, **kw):
    nz, ny, nx = shape
    return mm.default_params(nx=nx, ny=ny, nz=nz, dx=h[0], dy=h[1], dz=h[2], cfl=cfl, bc=bc, nb=nb,
                             sponge_sigma=sigma, cpml_f0=f0, **kw)


def grid_for(p, dt, vmax):
    return C.Grid(p.nx, p.ny, p.nz, p.dx, p.dy, p.dz, dt, bc=p.bc, nb=p.nb, sigma=p.sponge_sigma, R=p.cpml_R,
                  f0=p.cpml_f0, vmax=vmax, fs=p.free_surface)


def gpu_forward(p, vel, src, rec, wav, T, tile=None, graph=False, chunks=None):
    """Returns (traces [T][nrec] float32, final p^T, final p^{T-1}, dt)."""
    ctx = mm.Context.single(p, torch.from_numpy(np.ascontiguousarray(vel, dtype=np.float32)).to(DEV), src, rec)
    if tile is not None:
        ctx.set_tile(tile)
    nrec = len(np.asarray(rec).reshape(-1, 3))
    nsrc = len(np.asarray(src).reshape(-1, 3))
    tr = torch.zeros((max(T, 1), max(nrec, 1)), dtype=torch.float32, device=DEV)
    w = torch.from_numpy(np.ascontiguousarray(np.asarray(wav, dtype=np.float32).reshape(T, nsrc))).to(DEV)
    if chunks is None:
        ctx.forward(T, w if nsrc else None, tr if nrec else None, graph=graph)
    else:
        done = 0
        for c in chunks:
            ctx.forward(c, w[done:done + c] if nsrc else None, tr[done:done + c] if nrec else None, graph=graph)
            done += c
    st = ctx.get_state()
    torch.cuda.synchronize()
    n = vel.size
    s = st.cpu().numpy()
    dt = ctx.dt
    ctx.close()
    return tr.cpu().numpy()[:T, :nrec], s[n:2 * n].reshape(vel.shape), s[:n].reshape(vel.shape), dt


def oracle_forward(p, dt, vel, src, rec, wav, T):
    g = grid_for(p, dt, float(np.max(vel)))
    tr, pm, pc, mem = C.forward(g, np.asarray(vel, dtype=np.float64), src,
                                np.asarray(wav, dtype=np.float64).reshape(T, -1), rec, T)
    return tr, pc, pm
