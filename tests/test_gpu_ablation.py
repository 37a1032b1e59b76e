"""SPA in subsets (the paper's divide-and-conquer variant, Section 2.2.2;
the experiment its Section 4.3 asks for) on the GPU, against the oracle's
rule, and the discard effectiveness across subset sizes on tie-free
inputs.  Each case prints its name before its GPU calls; the experiment
prints its table."""
import sys
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import paper_1508_05488_amd as ch  # noqa: E402
from oracle import steps  # noqa: E402
from paper_1508_05488_amd import workloads as wl  # noqa: E402


def say(msg):
    print(msg, file=sys.stderr, flush=True)


def gpu_keep(k2, sigma, chunk):
    t = torch.from_numpy(np.ascontiguousarray(k2.astype(np.int32))).cuda()
    return ch.spa_chunked(t, sigma, chunk).cpu().numpy()


def test_chunked_spa_parity_with_ties():
    rng = np.random.default_rng(101)
    say("  spa_chunked on random sequences with ties")
    for m in (0, 1, 2, 63, 64, 65, 1000, 100_003):
        k2 = rng.integers(0, max(2, m // 3), size=m)
        sigma = int(rng.integers(0, max(3, m // 2)))
        for chunk in (1, 2, 31, 1024, max(m, 1)):
            want = steps.spa_keep_chunked(k2, sigma, chunk)
            got = gpu_keep(k2, sigma, chunk)
            assert np.array_equal(got, want), (m, chunk)


def test_chunked_spa_discard_effectiveness():
    chunks = [1, 4, 16, 64, 256, 1024, 4096]
    rows = []
    for dist, seed in (("square", 111), ("disk", 112), ("gaussian", 113)):
        pts = wl.tie_free(dist, 2_000_000, seed)
        seqs = steps.region_sequences(pts)
        s1 = sum(seqs[r][0].shape[0] for r in seqs)
        say(f"  spa_chunked {dist} tie-free 2M (s1 = {s1})")
        exact = 0
        counts = {c: 0 for c in chunks + ["paper"]}
        ms_paper = ms_exact = 0.0
        for r, (k2, sigma) in seqs.items():
            m = k2.shape[0]
            d = torch.from_numpy(np.ascontiguousarray(k2.astype(np.int32))).cuda()
            ex = steps.spa_keep(k2, sigma)
            exact += int(ex.sum())
            prev = None
            for c in chunks + ["paper"]:
                size = max(1, -(-m // 1024)) if c == "paper" else c
                got = ch.spa_chunked(d, sigma, size).cpu().numpy()
                want = steps.spa_keep_chunked(k2, sigma, size)
                assert np.array_equal(got, want), (dist, r, size)
                assert np.all(got[ex])  # a superset of the exact survivors
                if prev is not None and c != "paper":
                    assert np.all(prev[got])  # larger nested subsets keep fewer
                    prev = got
                elif c != "paper":
                    prev = got
                counts[c] += int(got.sum())
            # kernel time of the paper's configuration and of one subset
            for size, key in ((max(1, -(-m // 1024)), "paper"), (max(m, 1), "exact")):
                torch.cuda.synchronize()
                a = time.perf_counter()
                for _ in range(5):
                    ch.spa_chunked(d, sigma, size)
                torch.cuda.synchronize()
                dt = (time.perf_counter() - a) / 5 * 1e3
                if key == "paper":
                    ms_paper += dt
                else:
                    ms_exact += dt
        rows.append((dist, s1, exact, counts, ms_paper, ms_exact))
    print("\n| input (tie-free, 2M) | s1 | exact SPA | " + " | ".join(f"subsets of {c}" for c in chunks)
          + " | 1024 subsets per region (paper) | ms paper / one subset |", flush=True)
    for dist, s1, exact, counts, mp, me in rows:
        print(f"| {dist} | {s1} | {exact} | " + " | ".join(str(counts[c]) for c in chunks)
              + f" | {counts['paper']} | {mp:.3f} / {me:.3f} |", flush=True)


def test_discard_counts_per_config():
    # the analog of the paper's Figure 11: points left after each discard
    cases = [("square 100K", "square", 100_000, 1), ("square 20M", "square", 20_000_000, 2),
             ("disk 20M", "disk", 20_000_000, 3), ("gaussian 20M", "gaussian", 20_000_000, 4),
             ("adversarial 20M", "adversarial", 20_000_000, 5)]
    print("\n| input | n | open | sort records | s1 (round 1) | s2 (SPA) | polygon | hull |", flush=True)
    for name, dist, n, seed in cases:
        pts = wl.generate(dist, n, seed)
        say(f"  discard counts {name}")
        d = torch.from_numpy(pts).cuda()
        _, st = ch.polygon(d)
        h = ch.hull2d(d)
        hs = ch.last_stats()
        if n <= 100_000:
            r = steps.cudachain(pts)
            assert [st["s1"][q] for q in range(4)] == [r["s1"][q + 1] for q in range(4)]
            assert [st["s2"][q] for q in range(4)] == [r["s2"][q + 1] for q in range(4)]
        print(f"| {name} | {n} | {st['open']} | {st['candidates']} | {sum(st['s1'])} | {sum(st['s2'])} | "
              f"{hs['polygon']} | {h.numel()} |", flush=True)
