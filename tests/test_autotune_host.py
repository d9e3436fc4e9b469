"""Launch-configuration space and autotuner cache (host only, no device calls)."""
import ctypes
import json

import pytest


def _ws(tile, batch, flags=0):
    from paper_2501_06838_amd import _native as N
    arr = (N.gs_image * 2)(N.gs_image(40, 30, 3.3, 0, 1200, 0),
                           N.gs_image(17, 90, 11.5, 1200, 1530, 3 * 132 * 99))
    cfg = N.gs_config(tile, batch, flags, 0, 0)
    b = ctypes.c_size_t()
    return N.lib().gs_workspace_size(ctypes.byref(cfg), arr, 2, 2730, ctypes.byref(b))


def test_every_candidate_is_accepted_and_others_are_not():
    from paper_2501_06838_amd import _native as N
    from paper_2501_06838_amd.autotune import TILE_BATCHES, candidates
    for c in candidates():
        assert _ws(c["tile"], c["lds_batch"], c["flags"]) == N.GS_OK, c
    assert len(candidates()) == 4 * len(TILE_BATCHES)
    assert {c["flags"] for c in candidates()} == {0, 0x1, 0x4, 0x5}
    for tile in (8, 16, 32):
        for batch in (16, 32, 48, 64, 96, 112, 128, 256, 512):
            ok = (tile, batch) in TILE_BATCHES
            assert (_ws(tile, batch) == N.GS_OK) == ok, (tile, batch)
        assert _ws(tile, 0) == N.GS_OK   # default batch
    assert _ws(16, 0, 0x4) == N.GS_OK  # radix-sort binning
    assert _ws(16, 0, 0x8) == N.GS_OK  # pixel-centre sampling
    assert _ws(16, 0, 0x10) == N.GS_OK  # elliptical supports
    assert _ws(16, 0, 0x18 | 0x1) == N.GS_OK
    assert _ws(16, 0, 0x20) == N.GS_E_INVALID  # unknown flag bit
    # the elliptical kernels exist at each tile size's default batch only
    for tile, dflt, other in ((8, 64, 32), (16, 96, 128), (32, 32, 64)):
        assert _ws(tile, dflt, 0x10) == N.GS_OK
        assert _ws(tile, other, 0x10) == N.GS_E_UNSUPPORTED


def test_ellipse_rejects_a_window():
    from paper_2501_06838_amd import _native as N
    arr = (N.gs_image * 1)(N.gs_image(40, 30, 3.3, 0, 1200, 0))
    b = ctypes.c_size_t()
    for flags, want in ((0x10, N.GS_E_INVALID), (0x8, N.GS_OK), (0, N.GS_OK)):
        cfg = N.gs_config(16, 0, flags, 0, 0, 0.1)
        assert N.lib().gs_workspace_size(ctypes.byref(cfg), arr, 1, 1200,
                                         ctypes.byref(b)) == want, flags


def test_layout_key_depends_on_layout_and_device():
    from paper_2501_06838_amd.autotune import layout_key
    a = [(64, 64, 3.7, 0, 4096)] * 3
    assert layout_key(a, "gfx950") == layout_key([tuple(x) for x in a], "gfx950")
    assert layout_key(a, "gfx950") != layout_key(a, "other")
    assert layout_key(a, "gfx950") == layout_key(a, "gfx950", "graph")
    assert layout_key(a, "gfx950", "graph") != layout_key(a, "gfx950", "eager")
    b = [(64, 64, 3.7000001, 0, 4096)] * 3
    assert layout_key(a, "gfx950") != layout_key(b, "gfx950")
    c = [(64, 64, 3.7, 0, 4096)] * 2
    assert layout_key(a, "gfx950") != layout_key(c, "gfx950")
    # the packing offset does not matter, the counts do
    d = [(64, 64, 3.7, 7, 4096)] * 3
    assert layout_key(a, "gfx950") == layout_key(d, "gfx950")


def test_cache_round_trip_and_rejects_bad_entries(tmp_path):
    from paper_2501_06838_amd.autotune import TuneCache
    p = tmp_path / "sub" / "tune.json"
    c = TuneCache(str(p))
    assert c.get("k") is None
    c.put("k", {"config": {"tile": 16, "lds_batch": 128, "flags": 1}, "ms": 1.5})
    c2 = TuneCache(str(p))
    assert c2.get("k")["config"] == {"tile": 16, "lds_batch": 128, "flags": 1}
    c2.put("bad", {"config": {"tile": 12, "lds_batch": 128, "flags": 0}, "ms": 1.0})
    assert TuneCache(str(p)).get("bad") is None
    p.write_text("not json")
    assert TuneCache(str(p)).get("k") is None
    p.write_text(json.dumps([1, 2]))
    assert TuneCache(str(p)).entries == {}


def test_tile_count_limit_and_workspace_growth():
    """2^24 tiles or more is refused (one workgroup of up to 256 threads per
    tile must keep a dispatch under 2^32 work-items); just below is accepted;
    the radix-sort binning needs a larger workspace than the default."""
    from paper_2501_06838_amd import _native as N

    def ws(lr, s, tile, flags=0):
        arr = (N.gs_image * 1)(N.gs_image(lr, lr, s, 0, 1, 0))
        cfg = N.gs_config(tile, 0, flags, 1 << 20, 0)
        b = ctypes.c_size_t()
        st = N.lib().gs_workspace_size(ctypes.byref(cfg), arr, 1, 1, ctypes.byref(b))
        return st, b.value
    # 4096 x 4096 LR at x8 -> 32768^2 HR: 4096^2 = 2^24 tiles of 8 x 8
    assert ws(4096, 8.0, 8)[0] == N.GS_E_UNSUPPORTED
    # the same at 16 x 16 tiles: 2^22 tiles
    st, b0 = ws(4096, 8.0, 16)
    assert st == N.GS_OK
    st, b1 = ws(4096, 8.0, 16, 0x4)
    assert st == N.GS_OK and b1 > b0


def test_pick_keeps_the_default_within_the_margin():
    from paper_2501_06838_amd.autotune import DEFAULT_LAUNCH, pick
    other = {"tile": 16, "lds_batch": 112, "flags": 0}
    t = [{"config": dict(DEFAULT_LAUNCH), "ms": 1.00}, {"config": other, "ms": 0.99}]
    assert pick(t)["config"] == DEFAULT_LAUNCH          # 1% faster: noise
    t[1]["ms"] = 0.97
    assert pick(t)["config"] == other                   # 3% faster: taken
    assert pick(t, margin=0.05)["config"] == DEFAULT_LAUNCH
    # without the default among the timings the fastest wins
    assert pick(t[1:] + [{"config": {"tile": 8, "lds_batch": 64, "flags": 0}, "ms": 0.5}])["ms"] == 0.5
    # the default is what the library uses for a zero batch at tile 16
    from paper_2501_06838_amd import _native as N
    assert _ws(16, DEFAULT_LAUNCH["lds_batch"]) == N.GS_OK
