"""CPU checks of the C-ABI library: it loads, exports every declared entry
point, and its host finish (step 7, Melkman) agrees with the oracle when fed
the oracle's own simple polygons.  No GPU compute is called here."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1508_05488_amd as ch
from oracle import hull as oracle
from oracle import steps
from paper_1508_05488_amd import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "chainhull.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b([a-z_][a-z0-9_]*)\s*\(", src, flags=re.M)))


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert set(names) == set(ch.EXPORTS), names
    L = ctypes.CDLL(ch.LIB_PATH)
    for name in names:
        assert hasattr(L, name), name


def test_strerror_and_workspace_bound():
    for code in (ch.CH_OK, ch.CH_EINVAL, ch.CH_EDOMAIN, ch.CH_ENOMEM, ch.CH_EHIP, ch.CH_EADMIT, ch.CH_ECAPACITY):
        assert ch.strerror(code)
    assert ch.strerror(123) == "unknown status"
    assert ch.workspace_bytes(20_000_000) >= 20_000_000 * 24
    assert ch.workspace_bytes(10) > 0


def test_single_hull_entry_points_reject_bad_arguments():
    # checked on the host before any device call (no GPU is touched)
    L = ch.lib()
    buf = ctypes.create_string_buffer(64)
    base = ctypes.addressof(buf) + (-ctypes.addressof(buf)) % 16
    for fn in (L.hull2d, L.hull2d_async, L.hull2d_noalloc):
        assert fn(base, -1, base, base, None) == ch.CH_EINVAL          # n < 0
        assert fn(base, 1 << 31, base, base, None) == ch.CH_EINVAL     # n > 2^31 - 1
        assert fn(base, 5, base, None, None) == ch.CH_EINVAL           # no count
        assert fn(None, 5, base, base, None) == ch.CH_EINVAL           # no points
        assert fn(base, 5, None, base, None) == ch.CH_EINVAL           # no output
        assert fn(base + 4, 5, base, base, None) == ch.CH_EINVAL       # points not 8-byte aligned
    # beyond the fixed buffer of hull2d_noalloc
    assert L.hull2d_noalloc(base, ch.NOALLOC_MAX_POINTS + 1, base, base, None) == ch.CH_ECAPACITY


def test_noalloc_buffer_holds_the_largest_call():
    # the workspace layout for the most points hull2d_noalloc takes, plus
    # its header stand-in, fits the fixed device buffer declared in the header
    assert ch.workspace_bytes(ch.NOALLOC_MAX_POINTS) + 256 <= ch.NOALLOC_SCRATCH_BYTES
    hdr = open(os.path.join(ROOT, "include", "chainhull.h")).read()
    assert f"#define CH_NOALLOC_MAX_POINTS {ch.NOALLOC_MAX_POINTS}" in hdr
    assert "#define CH_NOALLOC_SCRATCH_BYTES (96u << 20)" in hdr and ch.NOALLOC_SCRATCH_BYTES == 96 << 20


def _finish_via_library(pts):
    res = steps.cudachain(pts)
    X, Y = steps.to_int(pts)
    poly = res["polygon"]
    xy = np.stack([X[poly], Y[poly]], axis=1).astype(np.int32)
    return ch.finish_host(xy, poly.astype(np.int32))


def test_host_finish_on_every_3x3_subset():
    rng = wl.rng_for(51)
    lattice = np.array([(x, y) for x in range(3) for y in range(3)], np.float32)
    for mask in range(1, 1 << 9):
        base = lattice[[i for i in range(9) if mask >> i & 1]]
        extra = base[rng.integers(0, base.shape[0], size=int(rng.integers(0, 4)))]
        pts = np.concatenate([base, extra])
        pts = pts[rng.permutation(pts.shape[0])]
        assert _finish_via_library(pts).tolist() == oracle.hull(pts).tolist()


@pytest.mark.parametrize("k", [3, 4, 5, 8, 16, 100, 1 << 23])
def test_host_finish_on_random_small_sets(k):
    rng = wl.rng_for(52 + k % 89)
    for _ in range(400):
        pts = wl.small_lattice(int(rng.integers(1, 40)), k, rng)
        assert _finish_via_library(pts).tolist() == oracle.hull(pts).tolist()


@pytest.mark.parametrize("dist", wl.DISTRIBUTIONS)
def test_host_finish_on_distributions(dist):
    pts = wl.generate(dist, 200_000, seed=53)
    assert _finish_via_library(pts).tolist() == oracle.hull(pts).tolist()


def test_host_finish_degenerate_inputs():
    assert ch.finish_host(np.zeros((0, 2)), np.zeros(0)).tolist() == []
    assert ch.finish_host([[3, 4]], [7]).tolist() == [7]
    # coincident vertices collapse; two distinct points start at the lowest
    assert ch.finish_host([[3, 4], [3, 4], [1, 9], [3, 4]], [5, 6, 2, 8]).tolist() == [5, 2]
    # collinear polygon: the two far ends
    assert ch.finish_host([[0, 0], [1, 1], [2, 2], [3, 3], [2, 2]], [0, 1, 2, 3, 4]).tolist() == [0, 3]
    with pytest.raises(ch.ChainHullError):
        ch.finish_host([[0, 0], [1 << 23, 0], [0, 1]], [0, 1, 2])


def test_tuning_table_on_the_host():
    # the launch-shape table is host state: set, looked up by size class,
    # validated, cleared (no GPU is touched)
    base = ch.get_tuning(-1)
    assert base == {"stream_grid": 1024, "stream_unroll": 4, "cand_per_row": 2048, "chain_grid": 1024,
                    "wide_grid": 1024, "batch_unroll": 2, "batch_order": 0, "serve_batch_max": 1 << 18,
                    "fused_max": 1 << 15, "list_max": 4096}
    try:
        ch.set_tuning(1000, dict(base, stream_grid=256, cand_per_row=2048))
        ch.set_tuning(10**6, dict(base, stream_unroll=2))
        assert ch.get_tuning(10)["stream_grid"] == 256
        assert ch.get_tuning(1000)["cand_per_row"] == 2048
        assert ch.get_tuning(1001)["stream_unroll"] == 2 and ch.get_tuning(1001)["stream_grid"] == 1024
        assert ch.get_tuning(10**6 + 1) == base
        for bad in (dict(stream_grid=300), dict(stream_unroll=3), dict(cand_per_row=512),
                    dict(chain_grid=10), dict(wide_grid=5000), dict(batch_unroll=4), dict(batch_order=2),
                    dict(serve_batch_max=-1)):
            with pytest.raises(ch.ChainHullError):
                ch.set_tuning(5, dict(base, **bad))
        for k in range(14):
            ch.set_tuning(2 * 10**6 + k, base)
        with pytest.raises(ch.ChainHullError):  # 16 classes at most
            ch.set_tuning(3 * 10**6, base)
    finally:
        ch.clear_tuning()
    assert ch.get_tuning(10) == base


def test_tuning_file_found_by_architecture(monkeypatch):
    # a process may see the device without its name (under rocprofv3 the
    # key reads "gfx950_"): the one tuning file of the architecture applies
    import torch
    files = [f for f in os.listdir(ch.TUNING_DIR) if f.startswith("gfx950_") and f.endswith(".json")]
    if len(files) != 1:
        pytest.skip("no single gfx950 tuning file")
    ch.lib()
    monkeypatch.setattr(torch.cuda, "is_available", lambda: True)
    monkeypatch.setattr(ch, "device_key", lambda: "gfx950_")
    try:
        path = ch.load_tuning()
        assert path is not None and os.path.basename(path) == files[0]
        assert ch.tuning_note() is None
        monkeypatch.setattr(ch, "device_key", lambda: "gfx000_Other")
        assert ch.load_tuning() is None and "no tuning file" in ch.tuning_note()
    finally:
        ch.clear_tuning()
