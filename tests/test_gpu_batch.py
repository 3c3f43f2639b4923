"""Ragged batches (persistent, graph-captured plan) and the tile autotuner,
through the C-ABI: the plan's per-pair scores equal the per-pair launches bit
for bit and match the FP64 oracle; graph replays interleaved with other GPU
work all agree."""
import numpy as np
import pytest
import torch

import oracle as O
import synth
from _helpers import MAP_TOL, SCORE_TOL, device, oparams, to_dev

pytestmark = pytest.mark.gpu

SMALL_LADDER = ((213, 120), (320, 180), (427, 240), (97, 61), (640, 360), (33, 29))


@pytest.fixture(scope="module")
def P():
    import paper_2101_06354_amd as P
    return P


@pytest.fixture(scope="module")
def dev():
    return device()


def _cfg(P, pr):
    return P.SSIMConfig(window=pr["window"], k=pr["k"], stride=pr["stride"])


def _make_plan(P, pairs, dev, with_maps=False):
    items, keep = [], []
    for pr in pairs:
        x, y = to_dev(pr["ref"], dev), to_dev(pr["dis"], dev)
        cfg = _cfg(P, pr)
        d = {"ref": x, "dis": y, "cfg": cfg}
        if with_maps:
            ho, wo = P.map_shape(cfg, *pr["ref"].shape)
            d["map"] = torch.full((ho, wo), float("nan"), dtype=torch.float32, device=dev)
        items.append(d)
        keep.append(d)
    return P.BatchPlan(items), keep


def test_small_ragged_plan_matches_unbatched_and_oracle(P, dev):
    pairs = synth.config3(pairs=24, ladder=SMALL_LADDER, stream=5)
    plan, items = _make_plan(P, pairs, dev, with_maps=True)
    n_items, n_blocks = plan.info()
    assert n_items > 0 and 1 <= n_blocks <= n_items
    s_b = plan.run()
    torch.cuda.synchronize()
    maps_b = [d["map"].clone() for d in items]
    s_u = plan.run_unbatched()
    torch.cuda.synchronize()
    assert torch.equal(s_b, s_u)
    for i, pr in enumerate(pairs):
        assert torch.equal(maps_b[i], items[i]["map"])
        ref = O.ssim_map(pr["ref"], pr["dis"], oparams(_cfg(P, pr)))["map"]
        assert np.abs(maps_b[i].cpu().numpy() - ref).max() <= MAP_TOL
        assert abs(float(s_b[i]) - O.mean_pool(ref)) <= SCORE_TOL
        # and the ordinary per-frame entry point
        s1 = P.ssim(items[i]["ref"], items[i]["dis"], _cfg(P, pr))
        assert abs(float(s1[0]) - float(s_b[i])) <= 1e-6
    plan.close()


def test_graph_replays_interleaved_with_eager_work(P, dev):
    pairs = synth.config3(pairs=12, ladder=SMALL_LADDER, stream=6)
    plan, items = _make_plan(P, pairs, dev)
    first = plan.run().clone()
    torch.cuda.synchronize()
    junk = torch.randn(1 << 20, device=dev)
    for r in range(5):
        # other GPU work between replays, including a large reduction
        junk = junk * 1.0001 + 1
        _ = float(junk.sum())
        out = plan.run()
        torch.cuda.synchronize()
        assert torch.equal(out, first), r
    plan.close()


def test_full_ragged_config(P, dev):
    """256 pairs drawn from the 426x240 .. 2560x1440 ladder, Gaussian 11 or
    box 8, stride 1 or 4."""
    pairs = synth.config3(pairs=256, workers=8)
    plan, items = _make_plan(P, pairs, dev)
    s_b = plan.run()
    s_u = plan.run_unbatched()
    torch.cuda.synchronize()
    assert torch.equal(s_b, s_u)
    # sampled pairs against the oracle: one of each (window, stride, size) kind
    seen = set()
    for i, pr in enumerate(pairs):
        key = (pr["window"], pr["stride"], pr["ref"].shape)
        if key in seen or len(seen) >= 10:
            continue
        seen.add(key)
        ref = O.ssim_map(pr["ref"], pr["dis"], oparams(_cfg(P, pr)))["map"]
        assert abs(float(s_b[i]) - O.mean_pool(ref)) <= SCORE_TOL, key
    plan.close()


def test_autotune_and_cache_roundtrip(P, dev, tmp_path):
    cfg = P.SSIMConfig()
    best = P.autotune(cfg, torch.uint8, 360, 640, 1)
    assert 0 <= best < P.num_tile_configs()
    box = P.SSIMConfig(window="box", k=8, stride=4)
    best2 = P.autotune(box, torch.uint8, 240, 426, 1)
    assert 0 <= best2 < P.num_tile_configs()
    # the timing frames of every dtype (pseudo-random samples over its range)
    for dt in (torch.uint16, torch.float32, torch.bfloat16):
        assert 0 <= P.autotune(P.SSIMConfig(L=1.0), dt, 120, 200, 2) < P.num_tile_configs()
    path = str(tmp_path / "tune.json")
    P.tune_cache_save(path)
    text = open(path).read()
    assert "entries" in text and "640x360" in text
    P.tune_cache_load(path)
    # tuned shapes give the same maps as the default shape
    x, y = synth.config1(frames=1, h=360, w=640)
    xt, yt = to_dev(x, dev), to_dev(y, dev)
    s_t, m_t = P.ssim(xt, yt, cfg, return_map=True)
    P.set_tile_override(0)
    try:
        s_0, m_0 = P.ssim(xt, yt, cfg, return_map=True)
    finally:
        P.set_tile_override(-1)
    assert torch.equal(m_t, m_0)
    assert abs(float(s_t[0]) - float(s_0[0])) <= 2e-7
