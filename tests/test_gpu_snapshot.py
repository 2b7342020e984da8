"""The BF16 snapshot codec of the gradient's checkpoints against a rounding
fixed from outside the library: torch's float32 -> bfloat16 conversion
(round to nearest even) of the scaled values, bit for bit.

Layout under test (declared with mm_snap_encode): c0 = bf16(p^k / s0[b]),
c1 = bf16((p^k - p^{k-1}) / s1[b]), s the largest magnitude of the block
b of 4096 cells (1 for an all-zero block); decode p^k = f(c0) s0,
p^{k-1} = p^k - f(c1) s1, each operation rounded once in float32."""
import numpy as np
import pytest
import torch

from paper_2007_06048_amd import minimod as mm

from .gpu_util import DEV

pytestmark = pytest.mark.gpu

BLK = 4096


def _block_max(x):
    n = x.size
    nb = (n + BLK - 1) // BLK
    pad = np.zeros(nb * BLK, np.float32)
    pad[:n] = np.abs(x)
    m = pad.reshape(nb, BLK).max(axis=1)
    return np.where(m > 0, m, np.float32(1.0)).astype(np.float32)


def _fields(n, seed):
    rng = np.random.default_rng(seed)
    # a wide dynamic range across blocks, an all-zero block, denormal-sized and exact-tie values
    mag = np.float32(10.0) ** rng.uniform(-30, 5, n).astype(np.float32)
    cur = (rng.standard_normal(n).astype(np.float32) * mag).astype(np.float32)
    prev = (cur * np.float32(0.999) + rng.standard_normal(n).astype(np.float32) * mag * np.float32(1e-3))
    prev = prev.astype(np.float32)
    if n > 2 * BLK:
        cur[BLK:2 * BLK] = 0.0
        prev[BLK:2 * BLK] = 0.0
    # block 0 has largest magnitude exactly 1 (scale 1), so values halfway between two
    # bfloat16 numbers stay ties after scaling (round to even, both directions)
    m0 = min(n, BLK)
    cur[:m0] = rng.uniform(-0.5, 0.5, m0).astype(np.float32)
    ties = np.array([-1.0, 0.5 + 2.0 ** -9, 0.5 + 3 * 2.0 ** -9, -(0.5 + 2.0 ** -9)], np.float32)
    k = min(n, 4)
    cur[:k] = ties[:k]
    return prev, cur


@pytest.mark.parametrize("n", [1, 4095, 4096, 3 * 4096 + 1234, 1 << 20])
def test_snapshot_codec_is_torch_rounding(n):
    prev, cur = _fields(n, seed=n)
    assert mm.load().mm_snap_blocks(n) == (n + BLK - 1) // BLK
    c0, c1, s0, s1 = mm.snap_encode(torch.from_numpy(prev).to(DEV), torch.from_numpy(cur).to(DEV))
    torch.cuda.synchronize()
    d = (cur - prev).astype(np.float32)
    rs0, rs1 = _block_max(cur), _block_max(d)
    assert np.array_equal(s0.cpu().numpy(), rs0) and np.array_equal(s1.cpu().numpy(), rs1)
    b = np.arange(n) // BLK
    q0 = torch.from_numpy((cur / rs0[b]).astype(np.float32)).to(torch.bfloat16).view(torch.int16).numpy()
    q1 = torch.from_numpy((d / rs1[b]).astype(np.float32)).to(torch.bfloat16).view(torch.int16).numpy()
    g0, g1 = c0.cpu().numpy(), c1.cpu().numpy()
    assert np.array_equal(g0, q0), int(np.sum(g0 != q0))
    assert np.array_equal(g1, q1), int(np.sum(g1 != q1))
    # decode: widen exactly, one rounding per product and for the difference
    pv, cv = mm.snap_decode(c0, c1, s0, s1)
    torch.cuda.synchronize()
    w0 = torch.from_numpy(q0).view(torch.bfloat16).to(torch.float32).numpy()
    w1 = torch.from_numpy(q1).view(torch.bfloat16).to(torch.float32).numpy()
    rc = (w0 * rs0[b]).astype(np.float32)
    rp = (rc - (w1 * rs1[b]).astype(np.float32)).astype(np.float32)
    assert np.array_equal(cv.cpu().numpy(), rc)
    assert np.array_equal(pv.cpu().numpy(), rp)
    # the codec's precision: 8 significant bits of the block scale, for p^k and for the increment
    assert np.all(np.abs(rc - cur) <= rs0[b] * 2.0 ** -9)
    assert np.all(np.abs((rc - rp) - d) <= rs1[b] * 2.0 ** -9 * 1.01 + (np.abs(rc) + rs1[b]) * 2.0 ** -22)


def test_snapshot_codec_argument_errors():
    L = mm.load()
    assert L.mm_snap_encode(None, None, -1, None, None, None, None, None) == mm.MM_ERR_ARG
    assert L.mm_snap_decode(None, None, None, None, 5, None, None, None) == mm.MM_ERR_ARG
    assert L.mm_snap_encode(None, None, 0, None, None, None, None, None) == mm.MM_OK
