"""The autotuner's candidate launch shapes: every shape it may choose gives
exactly the oracle's hulls (single-hull path on each distribution, sizes
spanning one and several k_stream rounds and a large polygon; the batched
kernel's loads in flight and launch orders on a batch of sets), and a
tuning file applied by the binding changes no result.  Each case prints its
name before its GPU calls."""
import json
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import paper_1508_05488_amd as ch  # noqa: E402
from oracle import hull as oracle  # noqa: E402
from paper_1508_05488_amd import autotune  # noqa: E402
from paper_1508_05488_amd import workloads as wl  # noqa: E402


def say(msg):
    print(msg, file=sys.stderr, flush=True)


INPUTS = [("square", 300_001, 601), ("disk", 1_000_000, 602), ("gaussian", 777_777, 603),
          ("adversarial", 1_500_000, 604)]


@pytest.fixture(scope="module")
def inputs():
    out = []
    for dist, n, seed in INPUTS:
        pts = wl.generate(dist, n, seed)
        out.append((f"{dist} n={n}", torch.from_numpy(pts).cuda(), oracle.hull(pts)))
    return out


def test_every_single_hull_shape_matches_oracle(inputs):
    base = ch.get_tuning(-1)
    try:
        for cand in autotune.candidates():
            ch.clear_tuning()
            ch.set_tuning(2**40, autotune.shape(base, **cand))
            assert ch.get_tuning(1000)["stream_grid"] == cand["stream_grid"]
            for name, d, want in inputs:
                say(f"  shape {cand} on {name}")
                out = torch.full((d.shape[0],), -7, dtype=torch.int32, device="cuda")
                cnt = torch.full((1,), -7, dtype=torch.int32, device="cuda")
                assert ch.hull2d_async(d, out, cnt) == ch.CH_OK
                torch.cuda.synchronize()
                c = int(cnt.item())
                assert np.array_equal(out[:max(c, 0)].cpu().numpy(), want), (cand, name, c)
    finally:
        ch.clear_tuning()


def test_batched_shapes_match_oracle():
    pts, offs, _ = wl.batched_sets(48, 100, 300_000, seed=611)
    d = torch.from_numpy(pts).cuda()
    want = [oracle.hull(pts[offs[s]:offs[s + 1]]) for s in range(len(offs) - 1)]
    base = ch.get_tuning(-1)
    try:
        for u in (1, 2):
            for o in (0, 1):
                ch.clear_tuning()
                ch.set_tuning(2**40, autotune.shape(base, batch_unroll=u, batch_order=o))
                say(f"  batched unroll {u} order {o}")
                hulls, _ = ch.hull2d_batched(d, offs)
                for s, h in enumerate(hulls):
                    assert np.array_equal(h.cpu().numpy(), want[s]), (u, o, s)
    finally:
        ch.clear_tuning()


def test_tuning_file_applies_and_keeps_results(tmp_path, inputs):
    base = ch.get_tuning(-1)
    doc = {"device": "test", "classes": [
        {"n_max": 500_000, "tuning": autotune.shape(base, stream_grid=256, stream_unroll=2, cand_per_row=2048)},
        {"n_max": 2**31 - 1, "tuning": autotune.shape(base, stream_grid=512, cand_per_row=65536, wide_grid=2048)}]}
    path = tmp_path / "t.json"
    path.write_text(json.dumps(doc))
    try:
        assert ch.load_tuning(str(path)) == str(path)
        assert ch.get_tuning(300_001)["stream_grid"] == 256
        assert ch.get_tuning(1_000_000)["stream_grid"] == 512
        for name, d, want in inputs:
            say(f"  tuning file on {name}")
            assert np.array_equal(ch.hull2d(d).cpu().numpy(), want), name
    finally:
        ch.clear_tuning()
        ch.load_tuning()  # the device's own file, if any
