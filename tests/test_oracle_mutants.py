"""The oracle's pins catch plausible mistakes.

Each case plants one mistake in a copy of the C oracle's source (a flipped
comparison, a transposed operand, a dropped term, a wrong tie-break), builds
it with gcc into a temporary directory and runs a short selection of the
pins; at least one must fail.  Nothing here touches the GPU library.
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest

from paper_1508_05488_amd import workloads as wl
from hullcheck import brute_hull, check_hull, polygon_with_extras

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "andrew_hull.c")

MUTANTS = {
    "collinear_kept_lower": ("cross3(chain[h - 2], chain[h - 1], &p[i]) <= 0) --h;\n            chain[h++] = &p[i];\n        }\n        /* Upper",
                             "cross3(chain[h - 2], chain[h - 1], &p[i]) < 0) --h;\n            chain[h++] = &p[i];\n        }\n        /* Upper"),
    "collinear_kept_upper": ("while (h > lower && cross3(chain[h - 2], chain[h - 1], &p[i]) <= 0) --h;",
                             "while (h > lower && cross3(chain[h - 2], chain[h - 1], &p[i]) < 0) --h;"),
    "duplicate_keeps_max_index": ("if (a->idx != b->idx) return a->idx < b->idx ? -1 : 1;",
                                  "if (a->idx != b->idx) return a->idx < b->idx ? 1 : -1;"),
    "start_at_leftmost": ("if (a->y < b->y || (a->y == b->y && a->x < b->x)) start = k;",
                          "if (a->x < b->x || (a->x == b->x && a->y < b->y)) start = k;"),
    "cross_transposed": ("return ax * by - ay * bx;", "return ay * bx - ax * by;"),
    "dropped_origin_term": ("int64_t ax = (int64_t)a->x - o->x, ay = (int64_t)a->y - o->y;",
                            "int64_t ax = (int64_t)a->x, ay = (int64_t)a->y - o->y;"),
    "upper_pops_into_lower": ("while (h > lower && cross3", "while (h >= lower && h >= 2 && cross3"),
    "domain_admits_2p23": ("v < 8388608.0f", "v <= 8388608.0f"),
    "dedup_on_x_only": ("if (m > 0 && p[m - 1].x == p[i].x && p[m - 1].y == p[i].y) continue;",
                        "if (m > 0 && p[m - 1].x == p[i].x) continue;"),
    "wrong_rotation_offset": ("out_idx[k] = chain[(start + k) % h]->idx;", "out_idx[k] = chain[(start + k + 1) % h]->idx;"),
}


def _build(tmp_path, name, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} not found exactly once"
    path = tmp_path / f"{name}.c"
    path.write_text(src.replace(old, new))
    so = tmp_path / f"{name}.so"
    subprocess.run(["gcc", "-O1", "-std=c99", "-shared", "-fPIC", "-o", str(so), str(path), "-lm"], check=True)
    lib = ctypes.CDLL(str(so))
    lib.oracle_hull.restype = ctypes.c_int
    lib.oracle_hull.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)]
    return lib


def _run(lib, pts):
    pts = np.ascontiguousarray(pts, dtype=np.float32)
    out = np.empty(max(pts.shape[0], 1), np.int32)
    h = ctypes.c_int64(0)
    rc = lib.oracle_hull(pts.ctypes.data, pts.shape[0], out.ctypes.data, ctypes.byref(h))
    if rc != 0:
        raise ValueError(rc)
    return out[:h.value].tolist()


def _pins(lib):
    """Yield nothing if every pin passes; raise on the first failure."""
    rng = wl.rng_for(99)
    lattice = np.array([(x, y) for x in range(3) for y in range(3)], np.float32)
    for mask in range(1, 1 << 9):
        base = lattice[[i for i in range(9) if mask >> i & 1]]
        extra = base[rng.integers(0, base.shape[0], size=2)]
        pts = np.concatenate([base, extra])[rng.permutation(base.shape[0] + 2)]
        assert _run(lib, pts) == brute_hull(pts)
    for _ in range(5):
        pts, want = polygon_with_extras(50, 10, 10, rng)
        assert _run(lib, pts) == want.tolist()
    pts = wl.generate("disk", 5000, 3)
    check_hull(pts, _run(lib, pts))
    bad = np.array([[1, 2], [2.0 ** 23, 4], [5, 1]], np.float32)
    try:
        _run(lib, bad)
    except ValueError:
        return
    raise AssertionError("2**23 was not rejected")


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_reject_mutant(tmp_path, name):
    old, new = MUTANTS[name]
    lib = _build(tmp_path, name, old, new)
    with pytest.raises((AssertionError, ValueError, KeyError)):
        _pins(lib)


def test_unmutated_source_passes_the_same_pins(tmp_path):
    lib = _build(tmp_path, "original", "#include <stdint.h>", "#include <stdint.h>")
    _pins(lib)
