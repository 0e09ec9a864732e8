"""Host logic of the autotuner: candidate shapes, cache keys, cache round trip,
choice of the fastest candidate (with an injected timer; no GPU)."""
import json

import numpy as np
import pytest

from paper_1510_07328_amd import autotune as A
from paper_1510_07328_amd import batch as B
from paper_1510_07328_amd import lbm


def tubes_of(nx, steps):
    n = len(nx)
    return B.make_tubes(np.array(nx), np.full(n, 0.7), np.ones(n), np.full(n, 0.8), np.array(steps))


def test_candidates_fit_the_lds_window():
    c = A.batch_candidates()
    assert len(c) == len(set(c)) > 10
    for s, h, b in c:
        assert s >= 1 and s + 2 * h <= A.MAX_WINDOW and b % 64 == 0 and 64 <= b <= 1024
    assert (448, 32, 1024) in c  # the library's default shape is among them


def test_batch_key_is_order_independent_and_discriminating():
    opt = B.make_options()
    t1 = tubes_of([300, 1000, 37], [1200, 4000, 148])
    t2 = tubes_of([1000, 37, 300], [4000, 148, 1200])
    k = A.batch_key("gfx950x256", t1, opt)
    assert k == A.batch_key("gfx950x256", t2, opt)
    assert k != A.batch_key("gfx950x304", t1, opt)
    assert k != A.batch_key("gfx950x256", tubes_of([300, 1000, 38], [1200, 4000, 148]), opt)
    assert k != A.batch_key("gfx950x256", tubes_of([300, 1000, 37], [1200, 4000, 149]), opt)
    assert k != A.batch_key("gfx950x256", t1, B.make_options(precision=lbm.LBM_FP64))
    assert k != A.batch_key("gfx950x256", t1, B.make_options(order=3))


def test_scaled_probe_keeps_the_schedule_shape():
    t = tubes_of([256, 8192, 50], [1024, 32768, 0])
    p = A._scaled_tubes(t, 0.125)
    assert [x.nx for x in p] == [256, 8192, 50]
    assert [x.steps for x in p] == [128, 4096, 0]
    assert [x.tau for x in p] == [x.tau for x in t]


def test_tune_batch_picks_fastest_and_caches(tmp_path):
    path = str(tmp_path / "cache.json")
    t = tubes_of([300, 1000], [1200, 4000])
    opt = B.make_options()
    calls = []

    def fake_timer(probe, o, shape):
        calls.append(shape)
        s, h, b = shape
        return 1.0 + abs(h - 24) / 10 + (1024 - b) / 1e4 + (512 - s - 2 * h) / 1e3

    shape, rec = A.tune_batch(t, opt, path=path, timer=fake_timer, device="dev0")
    assert shape == (464, 24, 1024) and not rec["cached"]
    assert len(calls) == len(A.batch_candidates())
    data = json.load(open(path))
    assert len(data) == 1 and list(data.values())[0]["halo"] == 24
    calls.clear()
    shape2, rec2 = A.tune_batch(t, opt, path=path, timer=fake_timer, device="dev0")
    assert shape2 == shape and rec2["cached"] and not calls
    o, _ = A.batch_options(t, opt, path=path, timer=fake_timer, device="dev0")
    assert (o.tile_cols, o.halo, o.block) == shape and opt.tile_cols == 0  # a copy, the input is unchanged


def test_pick_best_is_deterministic_on_ties():
    assert A.pick_best({(2, 1): 1.0, (1, 5): 1.0, (3, 0): 2.0}) == (1, 5)
    with pytest.raises(ValueError):
        A.pick_best({})


def test_tune_field_with_injected_timer(tmp_path):
    path = str(tmp_path / "c.json")
    cfg = lbm.make_config("d2v9", shape=(64, 64, 1))
    best, rec = A.tune_field(cfg, None, None, path=path, timer=lambda c, n, u, b: {128: 3, 256: 2, 512: 2.5, 1024: 4}[b],
                             device="dev0")
    assert best == 256 and not rec["cached"]
    best2, rec2 = A.tune_field(cfg, None, None, path=path, timer=None, device="dev0")
    assert best2 == 256 and rec2["cached"]


def test_corrupt_cache_is_ignored(tmp_path):
    path = tmp_path / "bad.json"
    path.write_text("{not json")
    assert A.load_cache(str(path)) == {}
