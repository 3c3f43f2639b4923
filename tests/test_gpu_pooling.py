"""GPU parity of the spatial pooling methods (ssimx_pool_map) against the
oracle's pooling functions, on SSIM maps the library computed and on
synthetic maps with ties, tiny maps and pitched batches."""
import numpy as np
import pytest
import torch

import oracle as O
import synth
from _helpers import SCORE_TOL, device, to_dev

pytestmark = pytest.mark.gpu

KINDS = [("mean", {}, lambda q: O.pool_mean(q)),
         ("cov", {}, lambda q: O.pool_cov(q)),
         ("mean_dev", {"p": 2, "o": 3}, lambda q: O.pool_md(q, 2, 3)),
         ("mean_dev", {"p": 4, "o": 1}, lambda q: O.pool_md(q, 4, 1)),
         ("mean_dev", {"p": 1.5, "o": 1}, lambda q: O.pool_md(q, 1.5, 1)),
         ("minkowski", {"p": 4}, lambda q: O.pool_minkowski(q, 4)),
         ("minkowski", {"p": 0.25}, lambda q: O.pool_minkowski(q, 0.25)),
         ("dist_weighted", {"p": 1}, lambda q: O.pool_distortion_weighted(q, 1)),
         ("dist_weighted", {"p": 8}, lambda q: O.pool_distortion_weighted(q, 8)),
         ("five_number", {}, lambda q: O.pool_five_number(q)),
         ("percentile", {"p": 6, "r": 4000}, lambda q: O.pool_percentile(q, 6, 4000)),
         ("percentile", {"p": 25, "r": 2}, lambda q: O.pool_percentile(q, 25, 2)),
         ("percentile", {"p": 0, "r": 2}, lambda q: O.pool_percentile(q, 0, 2)),
         ("percentile", {"p": 100, "r": 3}, lambda q: O.pool_percentile(q, 100, 3))]


@pytest.fixture(scope="module")
def P():
    import paper_2101_06354_amd as P
    return P


@pytest.fixture(scope="module")
def dev():
    return device()


@pytest.fixture(scope="module")
def ssim_maps(P, dev):
    x, y = synth.config1(frames=3, h=360, w=640)
    _, m = P.ssim(to_dev(x, dev), to_dev(y, dev), P.SSIMConfig(), return_map=True)
    return m


def _tol(want):
    return SCORE_TOL * max(1.0, abs(want))


@pytest.mark.parametrize("kind,kw,ref", KINDS, ids=[f"{k}-{'-'.join(map(str, v.values()))}" for k, v, _ in KINDS])
def test_pooling_of_ssim_maps(P, dev, ssim_maps, kind, kw, ref):
    got = P.pool(ssim_maps, kind, **kw).cpu().numpy()
    q = ssim_maps.cpu().numpy().astype(np.float64)
    for f in range(q.shape[0]):
        want = ref(q[f])
        assert abs(got[f] - want) <= _tol(want), (f, got[f], want)


@pytest.mark.parametrize("kind,kw,ref", KINDS, ids=[f"{k}-{'-'.join(map(str, v.values()))}" for k, v, _ in KINDS])
@pytest.mark.parametrize("shape", [(1, 1), (2, 3), (7, 300), (129, 65)])
def test_pooling_ties_and_small_maps(P, dev, kind, kw, ref, shape):
    rng = np.random.default_rng(shape[0] * 1000 + shape[1])
    # coarsely quantised values: many ties, including at the percentile cuts
    q = (np.round(rng.uniform(-0.2, 1.0, (2,) + shape) * 16) / 16).astype(np.float32)
    q[1, 0, 0] = 1.0
    got = P.pool(to_dev(q, dev), kind, **kw).cpu().numpy()
    for f in range(2):
        want = ref(q[f].astype(np.float64))
        if np.isnan(want):
            assert np.isnan(got[f])
        else:
            assert abs(got[f] - want) <= _tol(want), (f, got[f], want)


def test_pooling_pitched_batch_and_identity(P, dev):
    rng = np.random.default_rng(4)
    base = rng.uniform(0.3, 1.0, (3, 50, 90)).astype(np.float32)
    t = to_dev(base, dev)[:, 5:45, 7:80]  # row pitch 90, frame stride 4500
    q = base[:, 5:45, 7:80].astype(np.float64)
    for kind, kw, ref in KINDS:
        got = P.pool(t, kind, **kw).cpu().numpy()
        for f in range(3):
            want = ref(q[f])
            assert abs(got[f] - want) <= _tol(want), (kind, f)
    ones = torch.ones((2, 30, 40), dtype=torch.float32, device=dev)
    assert P.pool(ones, "cov").cpu().tolist() == [0.0, 0.0]
    assert P.pool(ones, "dist_weighted", p=2).cpu().tolist() == [1.0, 1.0]
    assert P.pool(ones, "five_number").cpu().tolist() == [1.0, 1.0]
