"""Host-side pieces of the launch-mapping autotuner and of the batched-round,
tuning and timing entry points (no GPU calls)."""
import ctypes
import json
import os

import pytest

pytest.importorskip("torch")
from paper_2609_22608_amd import autotune  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2609_22608_amd", "libfruitninja.so")


def test_cache_round_trip(tmp_path):
    path = str(tmp_path / "tune.json")
    c = autotune.Cache(path)
    assert c.get("k") is None
    ch = autotune.Choice(2048, 512, 1, 0.25)
    c.put("k", ch)
    again = autotune.Cache(path)
    got = again.get("k")
    assert got == ch
    assert json.load(open(path))["k"]["knn_target_waves"] == 2048
    mem = autotune.Cache(None)  # in memory only
    mem.put("x", ch)
    assert mem.get("x") == ch and not os.path.exists(str(tmp_path / "None"))


def test_candidates_are_valid_tunings():
    grid = list(autotune.knn_grid())
    assert {f for _, _, f in grid} == {1, 2, 3}
    for tw, mc, form in grid:
        assert 0 < tw <= 16384 and mc > 0 and mc % 64 == 0 and form in (1, 2, 3)
        if form == 3:
            assert tw <= 4096  # the matrix-core form caps its wavefront target


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_new_entry_points_reject_null_on_the_host():
    lib = ctypes.CDLL(LIB)
    lib.fn_last_error.restype = ctypes.c_char_p
    vp = ctypes.c_void_p
    for name, args in (("fn_batch_prepare", (vp(), vp())), ("fn_batch_launch", (vp(), vp())),
                       ("fn_graph_capture", (vp(), vp())), ("fn_graph_launch", (vp(), vp())),
                       ("fn_set_tuning", (vp(), vp())), ("fn_kernel_timing", (vp(), 1)),
                       ("fn_kernel_times", (vp(), vp(), 0, vp()))):
        rc = getattr(lib, name)(*args)
        assert rc < 0, name
        assert lib.fn_last_error() != b"", name
