"""Seeded synthetic inputs for the acoustic_iso_cd workloads.

This module only builds inputs: velocity models (float32, [nz][ny][nx], m/s),
source and receiver cell lists (int32 [n][3] as (i, j, k) = (x, y, z)) and the
scalar settings of each workload.  It holds none of the method's arithmetic
(no time step, wavelet, stencil or boundary formula), so both the GPU library
and the FP64 oracle can be fed from it.

The paper uses internal velocity models given only by vmin = 1500 m/s and
vmax = 4500 m/s (parameter echo of section "Compilation and usage"); the
models here are seeded synthetic stand-ins with those ranges and the shapes
of the workloads below.  Random numbers come from numpy's PCG64
(`numpy.random.default_rng(seed)`); models are generated in float64 and
rounded once to float32.
"""
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

BC_NONE, BC_SPONGE, BC_CPML = 0, 1, 2


@dataclass
class Shot:
    """One modeling experiment on its own (sub-)volume."""
    vel: np.ndarray                 # float32 [nz][ny][nx]
    src: np.ndarray                 # int32 [nsrc][3]
    rec: np.ndarray                 # int32 [nrec][3]
    origin: tuple = (0, 0, 0)       # (i, j, k) of the sub-volume in the big model
    rho: Optional[np.ndarray] = None  # float32 [nz][ny][nx] density (acoustic_iso)


@dataclass
class Workload:
    name: str
    nx: int
    ny: int
    nz: int
    h: float
    nsteps: int
    bc: int
    nb: int
    f0: float            # Ricker peak frequency, Hz
    t0: float            # Ricker delay, s
    cfl: float = 0.5
    sigma: float = 0.015  # sponge strength
    cpml_R: float = 1e-3
    shots: List[Shot] = field(default_factory=list)
    vel_true: Optional[np.ndarray] = None  # gradient workload: model that makes d_obs
    vmax: Optional[float] = None           # common vmax for all shots (dt and CPML)
    ckpt_every: int = 32

    @property
    def points(self):
        return sum(int(s.vel.size) for s in self.shots)


def smooth_random(shape, sigma, vmin, vmax, seed):
    """Standard normal noise, Gaussian-filtered (reflect, truncate 4), affinely
    rescaled to [vmin, vmax]."""
    from scipy.ndimage import gaussian_filter

    rng = np.random.default_rng(seed)
    x = rng.standard_normal(shape)
    x = gaussian_filter(x, sigma, mode="reflect", truncate=4.0)
    lo, hi = x.min(), x.max()
    x = vmin + (x - lo) * (vmax - vmin) / (hi - lo)
    return x


def _lin_weights(n_out, n_in, lo=0, count=None):
    """[count][n_in] weights of corner-aligned linear interpolation from n_in
    to n_out samples, rows lo .. lo+count-1 of the full n_out x n_in matrix."""
    count = n_out - lo if count is None else count
    pos = (np.arange(lo, lo + count) * (n_in - 1) / max(n_out - 1, 1)).astype(np.float64)
    i0 = np.minimum(np.floor(pos).astype(np.int64), n_in - 2) if n_in > 1 else np.zeros(count, np.int64)
    f = pos - i0
    W = np.zeros((count, n_in))
    r = np.arange(count)
    if n_in == 1:
        W[:, 0] = 1.0
        return W
    W[r, i0] = 1.0 - f
    W[r, i0 + 1] += f
    return W


def _upsample_trilinear(c, shape, origin=(0, 0, 0), full=None):
    """Trilinear interpolation (corner-aligned) of the coarse field c onto the
    box `shape` = (nz, ny, nx) starting at `origin` (k, j, i) of a full grid of
    shape `full` (default: the box itself).  Separable, so it is three small
    matrix products."""
    full = shape if full is None else full
    Wz = _lin_weights(full[0], c.shape[0], origin[0], shape[0])
    Wy = _lin_weights(full[1], c.shape[1], origin[1], shape[1])
    Wx = _lin_weights(full[2], c.shape[2], origin[2], shape[2])
    t = np.tensordot(c, Wx.T, axes=([2], [0]))          # [cz][cy][nx]
    t = np.tensordot(Wy, t, axes=([1], [1]))            # [ny][cz][nx]
    t = np.tensordot(Wz, t, axes=([1], [1]))            # [nz][ny][nx]
    return t.astype(np.float32)


def smooth_random_coarse(shape, sigma, vmin, vmax, seed, factor=8, box=None):
    """Large-model variant: noise on a grid `factor` times coarser, filtered
    with sigma/factor, rescaled, then trilinearly upsampled to `shape`.  With
    box = (origin, size) only that sub-box of the upsampled field is built."""
    cshape = tuple(max(2, -(-n // factor) + 1) for n in shape)
    c = smooth_random(cshape, sigma / factor, vmin, vmax, seed)
    if box is None:
        return _upsample_trilinear(c, shape)
    origin, size = box
    return _upsample_trilinear(c, size, origin, shape)


def plane(nx, ny, z, inc=1):
    jj, ii = np.meshgrid(np.arange(0, ny, inc), np.arange(0, nx, inc), indexing="ij")
    return np.stack([ii.ravel(), jj.ravel(), np.full(ii.size, z)], axis=1).astype(np.int32)


def two_layer_64():
    """64^3, h = 10 m, 1500 m/s above z = 32 and 2500 m/s from z = 32 down,
    Ricker 15 Hz at the centre, 12-cell sponge, 200 steps, receivers on the
    64 x 64 plane z = 12."""
    n = 64
    v = np.full((n, n, n), 1500.0, dtype=np.float32)
    v[32:] = 2500.0
    src = np.array([[32, 32, 32]], dtype=np.int32)
    return Workload("two_layer_64^3_sponge12_200steps", n, n, n, 10.0, 200, BC_SPONGE, 12, 15.0, 0.1,
                    shots=[Shot(v, src, plane(n, n, 12))])


def smooth_240():
    """240^3, h = 10 m, smooth random 1500-4500 m/s (seed 2, sigma 8 cells),
    20-cell CPML, Ricker 20 Hz at (120, 120, 20), 240 x 240 receivers at z = 10,
    1000 steps."""
    n = 240
    v = smooth_random((n, n, n), 8.0, 1500.0, 4500.0, seed=2).astype(np.float32)
    src = np.array([[120, 120, 20]], dtype=np.int32)
    return Workload("smooth_240^3_cpml20_1000steps", n, n, n, 10.0, 1000, BC_CPML, 20, 20.0, 0.075,
                    shots=[Shot(v, src, plane(n, n, 10))])


def layered_1024(nz=512, ny=1024, nx=1024, seed=3):
    """1024 x 1024 x 512, h = 12.5 m: 10 layers (9 seeded interfaces in
    [33, 479], sorted velocities in [1500, 5000]) times (1 + 0.05 xi) with xi a
    smooth seeded field scaled to max |xi| = 1; 32-cell CPML; Ricker 15 Hz at
    the centre; receivers every 4 cells on the plane z = 32; 500 steps."""
    rng = np.random.default_rng(seed)
    iface = np.sort(rng.choice(np.arange(33, 480), size=9, replace=False))
    iface = (iface * nz // 512).astype(np.int64)
    vel_layers = np.sort(rng.uniform(1500.0, 5000.0, size=10))
    xi = smooth_random_coarse((nz, ny, nx), 8.0, -1.0, 1.0, seed + 1000, factor=8)
    xi = xi / np.abs(xi).max()
    layer_of_z = np.searchsorted(iface, np.arange(nz), side="right")
    v = (vel_layers[layer_of_z].astype(np.float32)[:, None, None] * (1.0 + 0.05 * xi)).astype(np.float32)
    src = np.array([[nx // 2, ny // 2, nz // 2]], dtype=np.int32)
    return Workload(f"layered_{nx}x{ny}x{nz}_cpml32_500steps", nx, ny, nz, 12.5, 500, BC_CPML, 32, 15.0, 0.1,
                    shots=[Shot(v, src, plane(nx, ny, 32, inc=4))])


def batched_shots(nshots=32, big=(400, 1024, 1024), side=(128, 256), seed=4, nsteps=800):
    """`nshots` sub-volumes with sides uniform in [side] cut at uniform origins
    from a smooth random 1500-4500 m/s model of shape `big` ([nz][ny][nx]);
    16-cell CPML; Ricker 15 Hz at each sub-volume's centre; receivers on the
    full plane z = 16; 800 steps."""
    rng = np.random.default_rng(seed)
    cshape = tuple(max(2, -(-n // 8) + 1) for n in big)
    coarse = smooth_random(cshape, 1.0, 1500.0, 4500.0, seed)
    shots = []
    for _ in range(nshots):
        nx, ny, nz = (int(rng.integers(side[0], side[1] + 1)) for _ in range(3))
        ox = int(rng.integers(0, big[2] - nx + 1))
        oy = int(rng.integers(0, big[1] - ny + 1))
        oz = int(rng.integers(0, big[0] - nz + 1))
        v = _upsample_trilinear(coarse, (nz, ny, nx), (oz, oy, ox), big)
        shots.append(Shot(v, np.array([[nx // 2, ny // 2, nz // 2]], dtype=np.int32), plane(nx, ny, 16),
                          origin=(ox, oy, oz)))
    w = Workload(f"batched_{nshots}shots_cpml16_{nsteps}steps", 0, 0, 0, 10.0, nsteps, BC_CPML, 16, 15.0, 0.1,
                 shots=shots)
    w.vmax = float(coarse.max())  # trilinear interpolation never exceeds the coarse maximum
    return w


def fwi_200(n=200, nshots=8, seed=5, nsteps=1000):
    """200^3, h = 10 m: background v(z) = 2000 + 1500 k/(nz-1); true model =
    background + 6 Gaussian blobs (centres uniform in [40,160]^3 scaled to the
    grid, widths 8-16 cells, amplitude +-300 m/s); start model = background;
    20-cell sponge; Ricker 10 Hz; shots at z = 22 on {60,140} x {40,80,120,160}
    (scaled); receivers on the full plane z = 20; checkpoints every 32 steps."""
    rng = np.random.default_rng(seed)
    s = n / 200.0
    k = np.arange(n)
    bg = 2000.0 + 1500.0 * k / (n - 1)
    v0 = np.broadcast_to(bg[:, None, None], (n, n, n)).astype(np.float64)
    zz, yy, xx = np.meshgrid(k, k, k, indexing="ij")
    vt = v0.copy()
    for _ in range(6):
        c = rng.uniform(40 * s, 160 * s, size=3)
        sig = rng.uniform(8 * s, 16 * s)
        amp = 300.0 * (1.0 if rng.random() < 0.5 else -1.0)
        vt += amp * np.exp(-((xx - c[0]) ** 2 + (yy - c[1]) ** 2 + (zz - c[2]) ** 2) / (2 * sig * sig))
    xs = [int(round(60 * s)), int(round(140 * s))]
    ys = [int(round(y * s)) for y in (40, 80, 120, 160)]
    zs = int(round(22 * s))
    rec = plane(n, n, int(round(20 * s)))
    v0f = v0.astype(np.float32)
    shots = [Shot(v0f, np.array([[x, y, zs]], dtype=np.int32), rec) for x in xs for y in ys][:nshots]
    w = Workload(f"fwi_{n}^3_sponge20_{nsteps}steps_{nshots}shots", n, n, n, 10.0, nsteps, BC_SPONGE,
                 int(round(20 * s)), 10.0, 0.15, shots=shots)
    w.vel_true = vt.astype(np.float32)
    w.vmax = float(max(w.vel_true.max(), v0f.max()))
    return w


def random_points(rng, n, shape, margin=0):
    nz, ny, nx = shape
    return np.stack([rng.integers(margin, nx - margin, n), rng.integers(margin, ny - margin, n),
                     rng.integers(margin, nz - margin, n)], axis=1).astype(np.int32)


def smooth_iso(n=240, nsteps=1000):
    """acoustic_iso workload: the smooth 1500-4500 m/s model of smooth_240
    (seed 2, sigma 8 cells, at size n) with Gardner's density rho = 310 v^0.25
    (kg/m^3, v in m/s; the paper's models are internal, so this standard
    velocity-density relation stands in); 20-cell sponge; Ricker 20 Hz at
    (n/2, n/2, n/12); receivers on the full plane z = n/24; nsteps steps."""
    v = smooth_random((n, n, n), 8.0 * n / 240, 1500.0, 4500.0, seed=2)
    rho = 310.0 * v ** 0.25
    src = np.array([[n // 2, n // 2, n // 12]], dtype=np.int32)
    w = Workload(f"smooth_iso_{n}^3_sponge20_{nsteps}steps", n, n, n, 10.0, nsteps, BC_SPONGE, 20, 20.0, 0.075,
                 shots=[Shot(v.astype(np.float32), src, plane(n, n, n // 24), rho=rho.astype(np.float32))])
    return w
