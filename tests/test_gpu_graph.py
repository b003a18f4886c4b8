"""Scoring batches captured into a HIP graph (ngs_score_graph_*) through the C ABI: every
replay, with eager library work and host synchronisations between replays, must reproduce the
eager ngs_score_batch result on the same inputs, including after the training store and the
normalisers change in place (a greedy step), and the first replay's gains must match the
oracle. Mixed resolutions, more views than buffer sets."""
import sys

import numpy as np
import pytest

import oracle
import scenegen
from parity_util import check_gain

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2602_08266_amd import binding
    binding.lib()
    return binding


@pytest.fixture(scope="module")
def ctx(B):
    return B.Context(0)


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def workload():
    scene = scenegen.make_scene(6000, 8, 16, seed=11)
    cfg = scenegen.SceneConfig("graph", 6000, 8, 16, 13, ((96, 64, 5), (160, 120, 4), (200, 150, 4)), 525.0,
                               (0.5, 0.7))
    cands, train = scenegen.make_cameras(cfg, 11)
    return scene, cands, train


def same_batch(a, b, what):
    """Gains of two runs of the same batch: equal up to the order of the FP32 atomic adds that
    accumulate the information blocks (far below the 1e-3 parity bar)."""
    sa, ba, ra = (t.cpu().numpy() for t in a)
    sb, bb, rb = (t.cpu().numpy() for t in b)
    assert np.allclose(ra, rb, rtol=1e-5, atol=0), f"{what}: raw gains differ {np.abs(ra - rb).max()}"
    assert np.allclose(sa, sb, rtol=1e-5, atol=0), f"{what}: scores differ"
    ia, ib = int(ba[0]), int(bb[0])
    assert ia == ib or abs(sa[ia, 3] - sa[ib, 3]) <= 1e-5 * abs(sa[ia, 3]), f"{what}: argmax differs"


def test_graph_replays_match_eager_and_oracle(B, ctx):
    import torch
    log("test_graph_replays_match_eager_and_oracle")
    scene, cands, train = workload()
    ds = B.DeviceScene(scene, "cuda")
    rp, ig = B.raster_params(), B.ig_params()
    scorer = B.NbvScorer(ctx, ds, rp, ig, max_pairs=1 << 20, max_slots=1 << 14, store_capacity=1 << 14,
                         views_in_flight=4)
    tcams = [B.camera(c) for c in train]
    cams = [B.camera(c) for c in cands]
    norm = scorer.setup(tcams)
    eager = [t.clone() for t in scorer.score(cams)]
    ref = oracle.score(scene, train, cands)
    for v in range(len(cands)):
        check_gain(eager[2][v].cpu().numpy(), ref.ig_cand[v], f"eager view {v}")
    ws = B.score_workspace(ds, 1 << 20, 1 << 14, views_in_flight=4)
    g = B.ScoreGraph(ctx, ds, scorer.h, cams, rp, ig, ws, normalisers=norm)
    for r in range(3):
        out = [t.clone() for t in g.replay()]
        torch.cuda.synchronize()
        log(f"  replay {r}: best {int(out[1].item())}")
        assert int(g.overflow.item()) == 0
        same_batch(out, eager, f"replay {r}")
        # eager library work and a host synchronisation between replays
        eager = [t.clone() for t in scorer.score(cams)]
        torch.cuda.synchronize()
    # a greedy step: the chosen view joins the training set; the store is rebuilt in place
    # and the normalisers change, the graph is replayed as it is
    pick = int(eager[1].item())
    norm2 = scorer.setup(tcams + [cams[pick]])
    eager2 = [t.clone() for t in scorer.score(cams)]
    for r in range(2):
        out = [t.clone() for t in g.replay(normalisers=norm2)]
        torch.cuda.synchronize()
        same_batch(out, eager2, f"after the greedy step, replay {r}")
    ref2 = oracle.score(scene, list(train) + [cands[pick]], cands)
    for v in range(len(cands)):
        check_gain(out[2][v].cpu().numpy(), ref2.ig_cand[v], f"graph after greedy step, view {v}")
    g.close()


def test_graph_reports_overflow(B, ctx):
    """A pair capacity below what the views need: every replay raises the device overflow flag."""
    import torch
    log("test_graph_reports_overflow")
    scene, cands, train = workload()
    ds = B.DeviceScene(scene, "cuda")
    rp, ig = B.raster_params(), B.ig_params()
    B.ngs_prepare_scene(ctx, ds, ig)
    ws = B.score_workspace(ds, 64, 1 << 14, views_in_flight=2)
    g = B.ScoreGraph(ctx, ds, None, [B.camera(c) for c in cands[:5]], rp, ig, ws)
    for r in range(2):
        g.overflow.fill_(0)
        g.replay()
        torch.cuda.synchronize()
        assert int(g.overflow.item()) == 1
    g.close()
