"""What the trained surrogate gains over scoring every candidate exactly.

Seeded 200k-Gaussian scenes with 512 candidates at 80x60: exact scores from ngs_score_batch
label four training scenes; the network is trained on the GPU by the library's BF16 kernels.
On a held-out scene the pipeline (feature maps and network for every candidate, exact
re-score of the surrogate's 64 best) must pick a view within 2% of the exact best while
running the exact scorer on 1/8 of the candidates and taking less time than exact scoring of
all of them. Controls: the same network untrained must rank the candidates worse, and exact
re-scoring of 64 random candidates (the same exact budget without the network) must on
average pick a worse view than the pipeline."""
import sys
import time

import numpy as np
import pytest

import scenegen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2602_08266_amd import binding
    binding.lib()
    return binding


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def workload(seed, nv=512):
    scene = scenegen.make_scene(200_000, 32, 32, seed=seed)
    cfg = scenegen.SceneConfig("gain", 200_000, 32, 32, nv, ((80, 60, nv),), 525.0, (0.6, 0.6))
    cands, train = scenegen.make_cameras(cfg, seed)
    return scene, cands, train


def test_trained_surrogate_gains_over_exact_scoring(B):
    import torch
    from scipy.stats import spearmanr
    from paper_2602_08266_amd import surrogate as SG
    log("test_trained_surrogate_gains_over_exact_scoring")
    ctx = B.Context(0)
    xs, ys = [], []
    for seed in range(4):
        scene, cands, train = workload(100 + seed)
        s = SG.scene_samples(ctx, scene, cands, train, views_in_flight=8, max_pairs=1 << 22, rescore=64)
        xs.append(s.x)
        ys.append((s.y - s.y.mean()) / s.y.std())
        log(f"  training scene {seed}: features {s.seconds_features:.2f} s, exact {s.seconds_exact:.2f} s")
    x = torch.cat(xs, dim=1).contiguous()
    y = torch.cat(ys).contiguous()
    net = B.Surrogate(ctx, seed=0, max_batch=256)
    untrained = B.Surrogate(ctx, seed=0, max_batch=256)
    hist = SG.train(net, x, y, epochs=12, lr=1e-3)
    log(f"  loss {hist[0]:.3f} -> {hist[-1]:.3f}")
    assert hist[-1] < 0.5 * hist[0]

    scene, cands, train = workload(999)
    s = SG.scene_samples(ctx, scene, cands, train, views_in_flight=8, max_pairs=1 << 22, rescore=64)
    exact = s.y.cpu().numpy()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pred = SG.predict(net, s.x).cpu().numpy()
    t_net = time.perf_counter() - t0
    pick = SG.pipeline_pick(pred, exact, 64)
    regret = (exact.max() - exact[pick]) / abs(exact.max())
    rho = spearmanr(pred, exact)[0]
    rho0 = spearmanr(SG.predict(untrained, s.x).cpu().numpy(), exact)[0]
    t_pipe = s.seconds_features + t_net + s.seconds_rescore
    log(f"  held out: spearman trained {rho:.3f} untrained {rho0:.3f}; pick rank "
        f"{int((exact > exact[pick]).sum())}, regret {regret:.4f}; pipeline {t_pipe:.3f} s vs exact "
        f"{s.seconds_exact:.3f} s")
    rng = np.random.default_rng(5)
    rand = np.mean([(exact.max() - exact[c].max()) / abs(exact.max())
                    for c in (rng.choice(len(exact), 64, replace=False) for _ in range(200))])
    log(f"  random 64 re-scored: mean regret {rand:.4f}")
    assert regret <= 0.02
    assert rho >= 0.6 and rho >= rho0 + 0.1
    assert regret < rand
    assert t_pipe < s.seconds_exact
