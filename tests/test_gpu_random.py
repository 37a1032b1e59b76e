"""Randomized parity: hull2d, hull2d_async and hull2d_batched against the
oracle on seeded inputs of many shapes (the four distributions, small
lattices with many duplicates and collinear runs, points on one line,
heavy duplication, points on the bounding box), sizes log-uniform from 1
to 3M.  Each input prints its kind and size before its GPU calls."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import paper_1508_05488_amd as ch  # noqa: E402
from oracle import hull as oracle  # noqa: E402
from paper_1508_05488_amd import workloads as wl  # noqa: E402

M = (1 << 23) - 1
KINDS = ("square", "disk", "gaussian", "adversarial", "lattice", "line", "dups", "box")


def say(msg):
    print(msg, file=sys.stderr, flush=True)


def make(kind, n, rng):
    if kind == "lattice":
        return wl.small_lattice(n, int(rng.integers(2, 200)), rng)
    if kind == "line":  # every point on one line (or one point when a = b = 0)
        t = rng.integers(0, 1 << 20, size=n)
        a, b = int(rng.integers(0, 7)), int(rng.integers(0, 7))
        return np.stack([np.clip(t * a, 0, M), np.clip(t * b + 5, 0, M)], 1).astype(np.float32)
    if kind == "dups":  # about fifty copies of each point
        base = wl.generate("disk", max(1, n // 50), int(rng.integers(1 << 30)))
        return np.ascontiguousarray(base[rng.integers(0, base.shape[0], size=n)])
    if kind == "box":  # on the edges of the domain's bounding box
        side, t = rng.integers(0, 4, size=n), rng.integers(0, M + 1, size=n)
        x = np.where(side == 0, 0, np.where(side == 1, M, t))
        y = np.where(side == 2, 0, np.where(side == 3, M, t))
        return np.stack([x, y], 1).astype(np.float32)
    return wl.generate(kind, n, int(rng.integers(1 << 30)))


@pytest.mark.parametrize("block", range(4))
def test_random_inputs(block):
    rng = np.random.default_rng(7000 + block)
    out = torch.empty(3_000_000, dtype=torch.int32, device="cuda")
    cnt = torch.empty(1, dtype=torch.int32, device="cuda")
    for it in range(32):
        kind = KINDS[it % len(KINDS)]
        n = int(np.exp(rng.uniform(0, np.log(3_000_000))))
        pts = make(kind, n, rng)
        say(f"  block {block} input {it}: {kind} n={n}")
        d = torch.from_numpy(pts).cuda()
        want = oracle.hull(pts)
        assert np.array_equal(ch.hull2d(d).cpu().numpy(), want), (block, it, kind, n)
        assert ch.hull2d_async(d, out, cnt) == ch.CH_OK
        torch.cuda.synchronize()
        c = int(cnt.item())
        assert c == ch.CH_BATCH_REDO or np.array_equal(out[:c].cpu().numpy(), want), (block, it, kind, n, c)


@pytest.mark.parametrize("block", range(3))
def test_random_batches(block):
    rng = np.random.default_rng(7100 + block)
    for it in range(4):
        sets = [make(KINDS[k % len(KINDS)], int(np.exp(rng.uniform(0, np.log(200_000)))), rng)
                for k in range(int(rng.integers(1, 40)))]
        offs = np.zeros(len(sets) + 1, np.int64)
        offs[1:] = np.cumsum([s.shape[0] for s in sets])
        say(f"  block {block} batch {it}: {len(sets)} sets, {offs[-1]} points")
        hulls, _ = ch.hull2d_batched(torch.from_numpy(np.ascontiguousarray(np.concatenate(sets))).cuda(), offs)
        for k, s in enumerate(sets):
            assert np.array_equal(hulls[k].cpu().numpy(), oracle.hull(s)), (block, it, k, s.shape[0])
