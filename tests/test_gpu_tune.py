"""The autotuner on the GPU: every pair operation gets a measured launch for
every size class, the written table loads back, and a context running the
tuned launches still matches the oracle."""
import numpy as np
import pytest
import torch

import oracle
from paper_2103_01983_amd import native
from paper_2103_01983_amd import workloads as W

pytestmark = pytest.mark.gpu


def test_autotune_writes_a_loadable_table(dev, tmp_path):
    path = tmp_path / "tuning.txt"
    h = native.make_context(0)
    try:
        native._check(h, native.lib().ptrom_autotune(h, str(path).encode()), "ptrom_autotune")
    finally:
        native.destroy_context(h)
    rows = [l.split() for l in path.read_text().splitlines() if l and not l.startswith("#")]
    seen = {(r[0], int(r[1])) for r in rows}
    for op in native.PAIR_OPS:
        for cls in (11, 13, 15, 16, 17):
            assert (op, cls) in seen, (op, cls)
    for cls in (11, 13, 14, 15):
        assert (native.BATCHED_OP[0], cls) in seen, cls
    h = native.make_context(0, str(path))
    try:
        c = W.gaussian_patch(3000, seed=8, delta=0.01)
        xy = np.asarray(c.xy, np.float32).astype(np.float64)
        g = np.asarray(c.gamma, np.float32).astype(np.float64)
        xd = torch.tensor(xy, dtype=torch.float32, device=dev)
        gd = torch.tensor(g, dtype=torch.float32, device=dev)
        f, B = native.velocity_block_jacobian(xd, gd, 0.01, ctx=h)
        o = oracle.velocity(xy, g, float(np.float32(0.01)))
        assert np.linalg.norm(f.cpu().numpy() - o) <= 1e-5 * np.linalg.norm(o)
        ob = oracle.block_jacobian(xy, g, float(np.float32(0.01)))
        assert np.linalg.norm(B.cpu().numpy() - ob) <= 1e-5 * np.linalg.norm(ob)
        # the tuned batched launch on three instances
        sizes = [700, 2500, 1300]
        off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
        cs = [W.gaussian_patch(m, seed=20 + m, delta=0.01) for m in sizes]
        bx = np.concatenate([np.asarray(c.xy, np.float32).astype(np.float64) for c in cs])
        bg = np.concatenate([np.asarray(c.gamma, np.float32).astype(np.float64) for c in cs])
        dl = np.float32([0.01, 0.02, 0.005])
        fb = native.velocity_batched(off, torch.tensor(bx, dtype=torch.float32, device=dev),
                                     torch.tensor(bg, dtype=torch.float32, device=dev), dl, ctx=h).cpu().numpy()
        for b in range(3):
            o0, o1 = off[b], off[b + 1]
            ref = oracle.velocity(bx[2 * o0:2 * o1], bg[o0:o1], float(dl[b]))
            assert np.linalg.norm(fb[2 * o0:2 * o1] - ref) <= 1e-5 * np.linalg.norm(ref)
    finally:
        native.destroy_context(h)
