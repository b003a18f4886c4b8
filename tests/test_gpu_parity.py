"""GPU parity: the HIP path through the C ABI against the FP64 oracle on the same seeded
inputs (small configurations; the oracle runs live)."""
import sys

import numpy as np
import pytest

import oracle
import scenegen
from parity_util import check_gain, check_image

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


def device_scene(B, ctx, scene, target=-1):
    ds = B.DeviceScene(scene, "cuda")
    B.ngs_prepare_scene(ctx, ds, B.ig_params(target_id=target))
    return ds


def small_scene(k=4, n=40, seed=5, spread=0.06):
    rng = np.random.default_rng(seed)
    means = np.column_stack([rng.normal(0, spread, n), rng.normal(0, spread, n), rng.normal(0, 0.05, n)])
    ls = np.log(rng.uniform(0.004, 0.03, (n, 3)))
    return scenegen.tiny_scene(means, ls, rng.normal(size=(n, 4)), rng.normal(0, 1, n), rng.uniform(0, 1, (n, 3)),
                               rng.normal(0, 1.5, (n, k)))


def test_prepare_scene(B, ctx):
    log("test_prepare_scene")
    cfg, scene, cands, train = scenegen.make_workload("tiny", 0)
    for target in (-1, 3):
        ds = device_scene(B, ctx, scene, target)
        gt = oracle.gaussian_terms(scene, oracle.IGParams(target_id=target))
        assert np.allclose(ds.prob.cpu().numpy(), gt["p"], rtol=1e-5, atol=1e-7)
        assert np.allclose(ds.opacity.cpu().numpy(), gt["sigma"], rtol=1e-5)
        assert np.allclose(ds.kappa.cpu().numpy(), gt["kappa"], rtol=1e-5)
        assert np.allclose(ds.conf.cpu().numpy(), gt["conf"], rtol=1e-5)
        assert np.array_equal(ds.label.cpu().numpy(), gt["argmax"])


@pytest.mark.parametrize("wl,view", [("tiny", 0), ("tiny", 5)])
def test_project_bitexact_keys_and_rects(B, ctx, wl, view):
    log(f"test_project {wl} view {view}")
    cfg, scene, cands, train = scenegen.make_workload(wl, 0)
    cam = cands[view]
    ds = device_scene(B, ctx, scene)
    pr = B.ngs_project(ctx, ds, B.camera(cam), B.raster_params())
    ref = oracle.project(scene, cam)
    valid = ref["valid"].astype(bool)
    cnt = pr.count.cpu().numpy()
    assert np.array_equal(cnt > 0, valid)
    zk = pr.zkey.cpu().numpy().view(np.uint32)
    assert np.array_equal(zk[valid], ref["zkey"][valid])
    rect = pr.rect.cpu().numpy().astype(np.int32).T  # [n][4] -> [4][n]
    assert np.array_equal(rect[:, valid], ref["rect"][:, valid])
    area = (ref["rect"][2] - ref["rect"][0] + 1) * (ref["rect"][3] - ref["rect"][1] + 1)
    assert np.array_equal(cnt[valid], area[valid])
    m2 = pr.mean2d.cpu().numpy().astype(np.float64)
    assert np.allclose(m2[:, valid], ref["m"][:, valid], rtol=1e-6, atol=1e-4)
    con = pr.conic.cpu().numpy().astype(np.float64)
    assert np.allclose(con[:, valid], ref["conic"][:, valid], rtol=1e-6, atol=1e-9)


@pytest.mark.parametrize("wl,view", [("tiny", 0), ("tiny", 3)])
def test_bin_sort_bitexact(B, ctx, wl, view):
    log(f"test_bin_sort {wl} view {view}")
    cfg, scene, cands, train = scenegen.make_workload(wl, 0)
    cam = cands[view]
    ds = device_scene(B, ctx, scene)
    rp = B.raster_params()
    c = B.camera(cam)
    pr = B.ngs_project(ctx, ds, c, rp)
    lists = B.ngs_bin_sort(ctx, ds, pr, c, rp, capacity=16, want_keys=True)   # grows through CAPACITY
    ref = oracle.tile_lists(scene, cam)
    m = int(lists.n_pairs.item())
    assert m == ref["m"]
    assert np.array_equal(lists.gids[:m].cpu().numpy().view(np.uint32), ref["gids"])
    assert np.array_equal(lists.keys[:m].cpu().numpy().view(np.uint64), ref["keys"])
    assert np.array_equal(lists.ranges.cpu().numpy().view(np.uint32), ref["ranges"])


@pytest.mark.parametrize("chunk", [256, 2048, 8192])
def test_bin_sort_bitexact_every_chunk_size(B, ctx, chunk):
    """The second binning level's chunk size (a tuning knob) changes no list: 200k Gaussians
    at 640x480 against the oracle, bit for bit."""
    log(f"test_bin_sort chunk {chunk}")
    cfg, scene, cands, train = scenegen.make_workload("mid", 0, n_views=2)
    ds = device_scene(B, ctx, scene)
    rp = B.raster_params()
    c = B.camera(cands[1])
    pr = B.ngs_project(ctx, ds, c, rp)
    B.ngs_set_tuning(ctx, 0, 0, chunk)
    try:
        lists = B.ngs_bin_sort(ctx, ds, pr, c, rp, capacity=1 << 24)
    finally:
        B.ngs_set_tuning(ctx, 0)
    ref = oracle.tile_lists(scene, cands[1])
    m = int(lists.n_pairs.item())
    assert m == ref["m"]
    assert np.array_equal(lists.gids[:m].cpu().numpy().view(np.uint32), ref["gids"])
    assert np.array_equal(lists.ranges.cpu().numpy().view(np.uint32), ref["ranges"])


@pytest.mark.parametrize("groups", [1, 3, 4])
def test_score_batch_every_group_count(B, ctx, groups):
    """The number of view groups in flight (a tuning knob) changes no gain: a batch of 11
    views on 8 buffer sets (groups of 8 / groups views, a ragged last group) against the
    oracle (1e-3 relative), object-centric target."""
    log(f"test_score_batch groups {groups}")
    scene = scenegen.make_scene(3000, 8, 16, seed=23, object_centric=True)
    cfg = scenegen.SceneConfig("groups", 3000, 8, 16, 11, ((128, 96, 11),), 500.0, (0.6, 0.6))
    cands, train = scenegen.make_cameras(cfg, 23)
    target = scene.target
    assert target >= 1
    ds = B.DeviceScene(scene, "cuda")
    ig = oracle.IGParams(target_id=target)
    ref = oracle.score(scene, train, cands, ig=ig)
    assert ref.status == 0
    B.ngs_set_tuning(ctx, 0, 0, 0, groups)
    try:
        assert B.ngs_get_tuning(ctx)["groups_in_flight"] == groups
        scorer = B.NbvScorer(ctx, ds, B.raster_params(), B.ig_params(target_id=target), max_pairs=1 << 18,
                             max_slots=1 << 14, store_capacity=1 << 14, views_in_flight=8)
        scorer.setup([B.camera(c) for c in train])
        scores, best, raw = scorer.score([B.camera(c) for c in cands])
        for v in range(len(cands)):
            check_gain(raw[v].cpu().numpy(), ref.ig_cand[v], f"view {v}")
    finally:
        B.ngs_set_tuning(ctx, 0)


def test_tuning_rejects_bad_group_count(B, ctx):
    L = B.lib()
    for bad in (-1, 5):
        t = B.ngs_tuning(0, 0, 0, bad)
        assert L.ngs_set_tuning(ctx.handle, B._ref(t)) == B.NGS_INVALID_ARG


@pytest.mark.parametrize("w,h", [(2304, 64), (64, 1100), (64, 2100), (1300, 40)])
def test_bin_sort_bitexact_tile_grid_shapes(B, ctx, w, h):
    """Tile grids that take the other counter paths of the two-level partition: more than
    128 tiles per row (LDS counters), 65-128 rows and more than 128 rows (register pairs and
    LDS for the row level), 82 tiles per row (two registers per lane)."""
    log(f"test_bin_sort tile grid {w}x{h}")
    scene = scenegen.make_scene(20000, 8, 16, seed=31)
    cam = scenegen.look_at(np.array([0.55, -0.25, 0.35]), w, h, 0.9 * max(w, h))
    ds = device_scene(B, ctx, scene)
    rp = B.raster_params()
    c = B.camera(cam)
    pr = B.ngs_project(ctx, ds, c, rp)
    lists = B.ngs_bin_sort(ctx, ds, pr, c, rp, capacity=16, want_keys=True)
    ref = oracle.tile_lists(scene, cam)
    m = int(lists.n_pairs.item())
    assert m == ref["m"] and m > 0
    assert np.array_equal(lists.gids[:m].cpu().numpy().view(np.uint32), ref["gids"])
    assert np.array_equal(lists.keys[:m].cpu().numpy().view(np.uint64), ref["keys"])
    assert np.array_equal(lists.ranges.cpu().numpy().view(np.uint32), ref["ranges"])


def render_gpu(B, ctx, ds, cam, want_obj=True):
    rp = B.raster_params()
    c = B.camera(cam)
    pr = B.ngs_project(ctx, ds, c, rp)
    lists = B.ngs_bin_sort(ctx, ds, pr, c, rp, capacity=1 << 20)
    img = B.ngs_render(ctx, ds, pr, lists, c, rp, want_obj=want_obj)
    return {k: (v.cpu().numpy() if v is not None else None) for k, v in img.items()}, pr, lists


@pytest.mark.parametrize("view", [0, 2, 7])
def test_render_parity_tiny(B, ctx, view):
    log(f"test_render tiny view {view}")
    cfg, scene, cands, train = scenegen.make_workload("tiny", 0)
    ds = device_scene(B, ctx, scene)
    img, _, _ = render_gpu(B, ctx, ds, cands[view])
    ref = oracle.render(scene, cands[view])
    stats = check_image(img, ref, scene.k, depth_max=1.0)
    log(f"  {stats}")


def test_render_ragged_and_edge_cases(B, ctx):
    log("test_render ragged")
    sc = small_scene(k=4, n=60)
    # image size not a multiple of the tile; camera close enough for large footprints
    cam = scenegen.look_at(np.array([0.25, -0.2, 0.2]), 100, 70, 60.0)
    ds = device_scene(B, ctx, sc)
    img, _, lists = render_gpu(B, ctx, ds, cam)
    ref = oracle.render(sc, cam)
    check_image(img, ref, sc.k, depth_max=1.0)
    assert ref["ncontrib"].sum() > 0
    # a camera that looks away: nothing binned, empty image
    away = scenegen.look_at(np.array([3.0, 0.0, 0.2]), 100, 70, 60.0, target=(6.0, 0.0, 0.2))
    img, _, lists = render_gpu(B, ctx, ds, away)
    assert int(lists.n_pairs.item()) == 0
    assert np.all(img["t_final"] == 1.0) and np.all(img["rgb"] == 0.0) and np.all(img["argmax_id"] == 0)


def gpu_gain(B, ctx, ds, cam, ig, h=None, stats=None):
    rp = B.raster_params()
    c = B.camera(cam)
    pr = B.ngs_project(ctx, ds, c, rp)
    lists = B.ngs_bin_sort(ctx, ds, pr, c, rp, capacity=1 << 20)
    ws = B.IgWorkspace(ds, 1 << 14)
    return B.ngs_info_gain(ctx, ds, pr, lists, c, rp, ig, h, ws, stats).cpu().numpy()


@pytest.mark.parametrize("target", [-1, 2])
def test_info_gain_prior_only_tiny(B, ctx, target):
    """H_T = lambda I (no training information): gain of each candidate view."""
    log(f"test_info_gain prior-only target {target}")
    cfg, scene, cands, train = scenegen.make_workload("tiny", 0)
    ds = device_scene(B, ctx, scene, target)
    away = [scenegen.look_at(np.array([5.0, 0.0, 0.5]), 128, 96, 100.0, target=(10.0, 0.0, 0.5))]
    ref = oracle.score(scene, away, cands[:3], ig=oracle.IGParams(target_id=target))
    for v in range(3):
        g = gpu_gain(B, ctx, ds, cands[v], B.ig_params(target_id=target))
        r = check_gain(g, ref.ig_cand[v], f"view {v}")
        log(f"  view {v}: gpu {g} ref {ref.ig_cand[v]} rel {r:.2e}")


def test_info_gain_small_scene_all_outputs(B, ctx):
    log("test_info_gain small scene")
    sc = small_scene(k=4, n=30, seed=11)
    cam = scenegen.look_at(np.array([0.3, 0.1, 0.25]), 64, 48, 60.0)
    ds = device_scene(B, ctx, sc)
    away = [scenegen.look_at(np.array([5.0, 0.0, 0.5]), 64, 48, 60.0, target=(10.0, 0.0, 0.5))]
    for outputs in (1, 2, 4, 7):
        for eq2 in (1, 0):
            ref = oracle.score(sc, away, [cam], ig=oracle.IGParams(outputs=outputs, obj_eq2=eq2))
            g = gpu_gain(B, ctx, ds, cam, B.ig_params(outputs=outputs, obj_eq2=eq2))
            check_gain(g, ref.ig_cand[0], f"outputs {outputs} eq2 {eq2}")


@pytest.mark.parametrize("target", [-1, 3])
def test_score_pipeline_tiny(B, ctx, target):
    """Training setup (H_T, Eq. 10 normalisers) and batched scoring against the oracle."""
    log(f"test_score_pipeline tiny target {target}")
    cfg, scene, cands, train = scenegen.make_workload("tiny", 0)
    ds = B.DeviceScene(scene, "cuda")
    ig = B.ig_params(target_id=target)
    scorer = B.NbvScorer(ctx, ds, B.raster_params(), ig, max_pairs=1 << 18, max_slots=1 << 14,
                         store_capacity=1 << 14)
    norm = scorer.setup([B.camera(c) for c in train])
    ref = oracle.score(scene, train, cands, ig=oracle.IGParams(target_id=target))
    assert ref.status == 0
    check_gain(norm, ref.norm, "normalisers")
    for t in range(len(train)):
        check_gain(scorer.ig_train[t], ref.ig_train[t], f"train {t}")
    import torch
    stats = torch.zeros(B.STATS_LEN, dtype=torch.int64, device="cuda")
    scores, best, raw = scorer.score([B.camera(c) for c in cands], stats)
    raw = raw.cpu().numpy()
    for v in range(len(cands)):
        check_gain(raw[v], ref.ig_cand[v], f"candidate {v}")
    sc = scores.cpu().numpy().astype(np.float64)
    assert np.allclose(sc, ref.scores, rtol=2e-3)
    top = np.sort(ref.scores[:, 3])
    if (top[-1] - top[-2]) / abs(top[-1]) > 1e-3:
        assert int(best.item()) == ref.best
    st = stats.cpu().numpy()
    assert st[0] == len(cands) and st[5] == 0
    # contributing (tile, Gaussian) pairs: at least one per touched Gaussian, at most one per
    # contributing (pixel, Gaussian) pair and per emitted (tile, Gaussian) pair
    assert st[2] <= st[9] <= min(st[3], st[1])
    log(f"  best gpu {int(best.item())} oracle {ref.best}; stats {st}")


def opaque_workload(seed=4):
    """A tiny-sized scene with opacity logits N(7, 0.5) (sigma about 0.999) seen close up
    (f = 300 at 128x96), so that sigma exp(-q/2) passes the 0.99 clamp at many pixel centres."""
    scene = scenegen.make_scene(2000, 8, 16, seed=seed)
    rng = np.random.default_rng(seed + 100)
    scene.opacity_logit = rng.normal(7.0, 0.5, scene.n).astype(np.float32)
    cfg = scenegen.SceneConfig("opaque", 2000, 8, 16, 6, ((128, 96, 6),), 300.0 * 640 / 128, (0.6, 0.6))
    cands, train = scenegen.make_cameras(cfg, seed)
    return scene, cands, train


def clamped_pairs(scene, cam):
    """(pixel, Gaussian) pairs of the view where the unclamped opacity exceeds alpha_max."""
    pr = oracle.project(scene, cam)
    sig = 1.0 / (1.0 + np.exp(-scene.opacity_logit.astype(np.float64)))
    cnt = 0
    for g in np.flatnonzero(pr["valid"] & (sig > 0.99)):
        mx, my = pr["m"][:, g]
        a, b, c = pr["conic"][:, g]
        xs = np.arange(max(0, int(mx) - 2), min(cam.width, int(mx) + 3)) + 0.5
        ys = np.arange(max(0, int(my) - 2), min(cam.height, int(my) + 3)) + 0.5
        dx, dy = np.meshgrid(xs - mx, ys - my)
        q = a * dx * dx + 2 * b * dx * dy + c * dy * dy
        cnt += int((sig[g] * np.exp(-0.5 * q) > 0.99).sum())
    return cnt


def test_opaque_scene_alpha_clamp_render_and_gain(B, ctx):
    """Opacities on the 0.99 clamp (Eq. 1 with the 3DGS clamp): k_render's clamped alpha and
    k_ig_tile's zero opacity derivative at clamped contributors against the oracle."""
    log("test_opaque_scene_alpha_clamp")
    scene, cands, train = opaque_workload()
    ds = device_scene(B, ctx, scene)
    hits = [clamped_pairs(scene, c) for c in cands[:2]]
    assert min(hits) > 100, hits
    for v in range(2):
        img, _, _ = render_gpu(B, ctx, ds, cands[v])
        ref = oracle.render(scene, cands[v])
        st = check_image(img, ref, scene.k, depth_max=1.0)
        log(f"  view {v}: clamped (pixel, Gaussian) pairs {hits[v]}, {st}")
    for target in (-1, 3):
        ig = B.ig_params(target_id=target)
        scorer = B.NbvScorer(ctx, B.DeviceScene(scene, "cuda"), B.raster_params(), ig, max_pairs=1 << 18,
                             max_slots=1 << 14, store_capacity=1 << 14)
        norm = scorer.setup([B.camera(c) for c in train])
        ref = oracle.score(scene, train, cands, ig=oracle.IGParams(target_id=target))
        assert ref.status == 0
        check_gain(norm, ref.norm, f"normalisers target {target}")
        scores, best, raw = scorer.score([B.camera(c) for c in cands])
        raw = raw.cpu().numpy()
        for v in range(len(cands)):
            check_gain(raw[v], ref.ig_cand[v], f"target {target} candidate {v}")


@pytest.mark.parametrize("target", [3, 17])
def test_score_batch_filtered_lists_mid(B, ctx, target):
    """With a target object the batched scorer writes only the lists of tiles that a weighted
    Gaussian reaches; its gains must equal those of the stand-alone path over complete lists up
    to the order of FP32 atomic adds. A candidate that looks away from the scene gains exactly
    zero on both paths."""
    log(f"test_score_batch_filtered_lists mid target {target}")
    cfg, scene, cands, train = scenegen.make_workload("mid", 0)
    ds = B.DeviceScene(scene, "cuda")
    ig = B.ig_params(target_id=target)
    rp = B.raster_params()
    B.ngs_prepare_scene(ctx, ds, ig)
    away = scenegen.look_at(np.array([3.0, 0.0, 0.2]), 640, 480, 525.0, target=(6.0, 0.0, 0.2))
    views = [cands[0], cands[5], away, cands[9], cands[30]]
    scorer = B.NbvScorer(ctx, ds, rp, ig, max_pairs=1 << 24, max_slots=1 << 16, store_capacity=1 << 16,
                         views_in_flight=2)
    scorer.setup([B.camera(c) for c in train])
    _, _, raw = scorer.score([B.camera(c) for c in views])
    raw = raw.cpu().numpy()
    ws = B.IgWorkspace(ds, 1 << 16)
    seen = 0
    for i, cam in enumerate(views):
        c = B.camera(cam)
        pr = B.ngs_project(ctx, ds, c, rp)
        lists = B.ngs_bin_sort(ctx, ds, pr, c, rp, capacity=1 << 24)
        ref = B.ngs_info_gain(ctx, ds, pr, lists, c, rp, ig, scorer.h, ws).cpu().numpy()
        log(f"  view {i}: batch {raw[i]} stand-alone {ref}")
        if cam is away:
            assert np.all(raw[i] == 0.0) and np.all(ref == 0.0)
        else:
            seen += int(np.all(ref > 0.0))
            assert np.allclose(raw[i], ref, rtol=1e-4, atol=0.0)
    assert seen >= 2  # the target is in view of most candidates


def test_count_pairs_prepass_matches_oracle(B, ctx):
    """The capacity pre-pass (ngs_count_pairs) gives every view's pair count M exactly."""
    log("test_count_pairs_prepass")
    cfg, scene, cands, train = scenegen.make_workload("tiny", 0)
    ds = device_scene(B, ctx, scene)
    rp = B.raster_params()
    away = scenegen.look_at(np.array([3.0, 0.0, 0.2]), 128, 96, 100.0, target=(6.0, 0.0, 0.2))
    views = list(cands) + [away]
    got = B.ngs_count_pairs(ctx, ds, [B.camera(c) for c in views], rp).cpu().numpy()
    ref = [oracle.tile_lists(scene, c)["m"] for c in views]
    log(f"  pairs {got.tolist()}")
    assert got.tolist() == ref and ref[-1] == 0


def test_surrogate_pick_rescores_the_network_choice(B, ctx):
    """ngs_sur_pick: the candidates ranked by the given predictions (descending, lower index on
    ties), the best `rescore` of them scored exactly as ngs_score_batch scores them, and the
    exact argmax among those returned as an index into the full candidate list."""
    import torch
    log("test_surrogate_pick")
    cfg, scene, cands, train = scenegen.make_workload("tiny", 0)
    ds = B.DeviceScene(scene, "cuda")
    rp, ig = B.raster_params(), B.ig_params()
    scorer = B.NbvScorer(ctx, ds, rp, ig, max_pairs=1 << 18, max_slots=1 << 14, store_capacity=1 << 14)
    norm = scorer.setup([B.camera(c) for c in train])
    cams = [B.camera(c) for c in cands]
    full_scores, full_best, _ = scorer.score(cams)
    full_scores = full_scores.cpu().numpy()
    rng = np.random.default_rng(3)
    pred_np = rng.normal(size=len(cams)).astype(np.float32)
    pred_np[5] = pred_np[2]  # a tie: the lower index goes first
    pred = torch.tensor(pred_np, device="cuda")
    order = sorted(range(len(cams)), key=lambda i: (-pred_np[i], i))
    for r in (1, 3, len(cams), len(cams) + 4):
        best, chosen, scores, raw = B.ngs_sur_pick(ctx, ds, scorer.h, norm, cams, pred, r, rp, ig, scorer.workspace())
        rr = min(r, len(cams))
        assert chosen == order[:rr]
        sc = scores.cpu().numpy()
        assert np.allclose(sc, full_scores[chosen], rtol=1e-4, atol=0.0)
        assert best == chosen[int(np.argmax(sc[:, 3]))]
    assert best == int(full_best.item())


def test_training_setup_degenerate_and_capacity(B, ctx):
    """ngs_training_setup reports a training set that sees nothing (all Eq. 10 normalisers
    zero) as NGS_DEGENERATE, and a store smaller than the touched Gaussians as NGS_CAPACITY."""
    log("test_training_setup errors")
    cfg, scene, cands, train = scenegen.make_workload("tiny", 0)
    ds = B.DeviceScene(scene, "cuda")
    away = scenegen.look_at(np.array([3.0, 0.0, 0.2]), 128, 96, 100.0, target=(6.0, 0.0, 0.2))
    scorer = B.NbvScorer(ctx, ds, B.raster_params(), B.ig_params(), max_pairs=1 << 18, max_slots=1 << 14,
                         store_capacity=1 << 14)
    with pytest.raises(B.NgsError) as e:
        scorer.setup([B.camera(away)])
    assert e.value.status == B.NGS_DEGENERATE
    small = B.NbvScorer(ctx, ds, B.raster_params(), B.ig_params(), max_pairs=1 << 18, max_slots=1 << 14,
                        store_capacity=8)
    with pytest.raises(B.NgsError) as e:
        small.setup([B.camera(c) for c in train])
    assert e.value.status == B.NGS_CAPACITY
    # the context and a correct store still work afterwards
    norm = scorer.setup([B.camera(c) for c in train])
    assert np.all(norm > 0)


def test_view_slot_overflow_then_recovers(B, ctx):
    """More weighted Gaussians reach a view than its workspace has statistic slots: the front
    pass's slot claims stop at the capacity and the call reports NGS_CAPACITY; a scorer with
    enough slots on the same context and scene then matches the oracle (the claimed slots and
    the refused ones leave no stale entries behind)."""
    log("test_view_slot_overflow_then_recovers")
    cfg, scene, cands, train = scenegen.make_workload("tiny", 0)
    cands = cands[:4]
    ds = B.DeviceScene(scene, "cuda")
    small = B.NbvScorer(ctx, ds, B.raster_params(), B.ig_params(), max_pairs=1 << 18, max_slots=8,
                        store_capacity=1 << 14)
    with pytest.raises(B.NgsError) as e:
        small.setup([B.camera(c) for c in train])
    assert e.value.status == B.NGS_CAPACITY
    ref = oracle.score(scene, train, cands)
    assert ref.status == 0
    scorer = B.NbvScorer(ctx, ds, B.raster_params(), B.ig_params(), max_pairs=1 << 18, max_slots=1 << 14,
                         store_capacity=1 << 14)
    scorer.setup([B.camera(c) for c in train])
    for rep in range(2):  # the second call reuses the workspace after the first call's claims
        scores, best, raw = scorer.score([B.camera(c) for c in cands])
        for v in range(len(cands)):
            check_gain(raw[v].cpu().numpy(), ref.ig_cand[v], f"call {rep} view {v}")


@pytest.mark.parametrize("target", [-1, 3])
def test_greedy_nbv_sequence_tiny(B, ctx, target):
    """Three greedy steps: each chosen view joins the training set (H_T and normalisers are
    rebuilt) before the remaining candidates are rescored; the GPU follows the oracle's picks
    so that every step compares the same candidate set."""
    log(f"test_greedy_nbv_sequence tiny target {target}")
    cfg, scene, cands, train = scenegen.make_workload("tiny", 0)
    ds = B.DeviceScene(scene, "cuda")
    scorer = B.NbvScorer(ctx, ds, B.raster_params(), B.ig_params(target_id=target), max_pairs=1 << 18,
                         max_slots=1 << 14, store_capacity=1 << 14)
    oig = oracle.IGParams(target_id=target)
    chosen, remaining, picks, refs = [], list(range(len(cands))), [], []
    for step in range(3):
        ref = oracle.score(scene, list(train) + [cands[i] for i in chosen], [cands[i] for i in remaining], ig=oig)
        assert ref.status == 0
        refs.append((list(remaining), ref))
        pick = remaining[ref.best]
        picks.append(pick)
        chosen.append(pick)
        remaining.remove(pick)
    seq = scorer.greedy([B.camera(c) for c in train], [B.camera(c) for c in cands], 3, follow=picks)
    for step, (rem, ref) in enumerate(refs):
        got = seq[step]
        assert got["remaining"] == rem
        check_gain(got["norm"], ref.norm, f"step {step} normalisers")
        for v in range(len(rem)):
            check_gain(got["raw"][v], ref.ig_cand[v], f"step {step} candidate {rem[v]}")
        assert np.allclose(got["scores"].astype(np.float64), ref.scores, rtol=2e-3)
        top = np.sort(ref.scores[:, 3])
        if len(top) > 1 and (top[-1] - top[-2]) / abs(top[-1]) > 1e-3:
            assert got["best"] == picks[step]
        log(f"  step {step}: pick {picks[step]} gpu best {got['best']}")


def test_abi_errors(B, ctx):
    log("test_abi_errors")
    import ctypes as C
    L = B.lib()
    cfg, scene, cands, train = scenegen.make_workload("tiny", 0)
    ds = device_scene(B, ctx, scene)
    cam = B.camera(cands[0])
    rp = B.raster_params()
    pr = B.ngs_project(ctx, ds, cam, rp)
    sc, pc = ds.c(), pr.c()
    bad_rp = B.raster_params(tile=8)
    assert L.ngs_project(ctx.handle, C.byref(sc), C.byref(cam), C.byref(bad_rp), C.byref(pc), None) == B.NGS_UNSUPPORTED
    assert L.ngs_project(ctx.handle, None, C.byref(cam), C.byref(rp), C.byref(pc), None) == B.NGS_INVALID_ARG
    big = B.ngs_camera(cam.R, cam.t, cam.fx, cam.fy, cam.cx, cam.cy, 4096, 4096)
    assert L.ngs_project(ctx.handle, C.byref(sc), C.byref(big), C.byref(rp), C.byref(pc), None) == B.NGS_UNSUPPORTED
    sc_bad = ds.c()
    sc_bad.k = 65
    assert L.ngs_project(ctx.handle, C.byref(sc_bad), C.byref(cam), C.byref(rp), C.byref(pc), None) == B.NGS_UNSUPPORTED
    # degenerate normalisers
    import torch
    ws = B.score_workspace(ds, 1 << 16, 1 << 12)
    with pytest.raises(B.NgsError) as e:
        B.ngs_score_batch(ctx, ds, None, [1.0, 0.0, 1.0], [cam], rp, B.ig_params(), ws)
    assert e.value.status == B.NGS_DEGENERATE
    # too small a workspace for the IG slots
    tiny_ws = B.IgWorkspace.__new__(B.IgWorkspace)
    tiny_ws.buf = torch.empty(64, dtype=torch.uint8, device="cuda")
    lists = B.ngs_bin_sort(ctx, ds, pr, cam, rp, capacity=1 << 16)
    with pytest.raises(B.NgsError) as e:
        B.ngs_info_gain(ctx, ds, pr, lists, cam, rp, B.ig_params(), None, tiny_ws)
    assert e.value.status == B.NGS_WORKSPACE_TOO_SMALL
    assert L.ngs_render_backward(ctx.handle, None, None, None, None, None, 0, None, None, None, 0, None) == B.NGS_INVALID_ARG


@pytest.mark.parametrize("k,lpp,waves", [(4, 1, 0), (4, 2, 0), (8, 1, 0), (8, 2, 0), (16, 1, 0), (16, 2, 0),
                                         (16, 4, 0), (32, 1, 0), (32, 2, 0), (32, 2, 4), (32, 4, 0), (64, 1, 0),
                                         (64, 2, 0), (64, 2, 4)])
def test_info_gain_every_launch_shape(B, ctx, k, lpp, waves):
    """Every lanes-per-pixel shape the autotuner may pick (ngs_set_tuning) scores a small
    scene with a training store to the oracle's gains (1e-3 relative)."""
    log(f"test_info_gain_every_launch_shape k={k} lpp={lpp} waves={waves}")
    clusters = min(8, k)
    scene = scenegen.make_scene(3000, clusters, k, seed=21)
    cfg = scenegen.SceneConfig("shape", 3000, clusters, k, 4, ((128, 96, 4),), 500.0, (0.6, 0.6))
    cands, train = scenegen.make_cameras(cfg, 21)
    ds = B.DeviceScene(scene, "cuda")
    ref = oracle.score(scene, train, cands)
    assert ref.status == 0
    B.ngs_set_tuning(ctx, lpp, waves)
    try:
        assert B.ngs_get_tuning(ctx) == {"ig_lanes_per_pixel": lpp, "ig_waves_per_simd": waves, "bin_chunk": 0,
                                         "groups_in_flight": 0}
        scorer = B.NbvScorer(ctx, ds, B.raster_params(), B.ig_params(), max_pairs=1 << 18, max_slots=1 << 14,
                             store_capacity=1 << 14, views_in_flight=2)
        norm = scorer.setup([B.camera(c) for c in train])
        check_gain(norm, ref.norm, "normalisers")
        scores, best, raw = scorer.score([B.camera(c) for c in cands])
        for v in range(len(cands)):
            check_gain(raw[v].cpu().numpy(), ref.ig_cand[v], f"view {v}")
    finally:
        B.ngs_set_tuning(ctx, 0)


def test_tuning_rejects_shapes_the_width_does_not_allow(B, ctx):
    log("test_tuning_rejects_shapes")
    scene = scenegen.make_scene(500, 8, 64, seed=3)
    ds = B.DeviceScene(scene, "cuda")
    with pytest.raises(B.NgsError):
        B.ngs_set_tuning(ctx, 3)
    with pytest.raises(B.NgsError):
        B.ngs_set_tuning(ctx, 2, 3)
    cam = scenegen.look_at(np.array([0.6, 0.0, 0.3]), 64, 48, 60.0)
    for lpp, waves in ((4, 0), (1, 4)):  # four lanes at k = 64; the 4-wave build with one lane
        B.ngs_set_tuning(ctx, lpp, waves)
        try:
            scorer = B.NbvScorer(ctx, ds, B.raster_params(), B.ig_params(), max_pairs=1 << 16, max_slots=1 << 12,
                                 store_capacity=1 << 12)
            with pytest.raises(B.NgsError):
                scorer.setup([B.camera(cam)])
        finally:
            B.ngs_set_tuning(ctx, 0)


@pytest.mark.parametrize("wl,target", [("tiny", -1), ("tiny", 3), ("k64", -1)])
def test_trace_criterion_matches_oracle(B, ctx, wl, target):
    """The trace-based f of Sec. III-B (criterion 1): training totals S, the raw covariance-
    trace reductions, the Eq. 10 normalisers of the converted gains, the scores and the argmax
    against the oracle. k64 takes the factored object block at k = 64."""
    log(f"test_trace_criterion {wl} target {target}")
    if wl == "tiny":
        cfg, scene, cands, train = scenegen.make_workload("tiny", 0)
    else:
        scene = scenegen.make_scene(3000, 8, 64, seed=23)
        cfg = scenegen.SceneConfig("k64", 3000, 8, 64, 4, ((128, 96, 4),), 500.0, (0.6, 0.6))
        cands, train = scenegen.make_cameras(cfg, 23)
    cands = cands[:5]
    ds = B.DeviceScene(scene, "cuda")
    ig = B.ig_params(target_id=target, criterion=1)
    ref = oracle.score(scene, train, cands, ig=oracle.IGParams(target_id=target, criterion=1))
    assert ref.status == 0
    scorer = B.NbvScorer(ctx, ds, B.raster_params(), ig, max_pairs=1 << 18, max_slots=1 << 14,
                         store_capacity=1 << 14)
    norm = scorer.setup([B.camera(c) for c in train])
    assert np.allclose(scorer.trace_total, ref.trace_total, rtol=1e-6)
    for t in range(len(train)):
        check_gain(scorer.ig_train[t], ref.ig_train[t], f"training view {t}")
    check_gain(norm, ref.norm, "normalisers")
    scores, best, raw = scorer.score([B.camera(c) for c in cands])
    for v in range(len(cands)):
        check_gain(raw[v].cpu().numpy(), ref.ig_cand[v], f"candidate {v}")
    assert np.allclose(scores.cpu().numpy().astype(np.float64), ref.scores, rtol=2e-3)
    top = np.sort(ref.scores[:, 3])
    if (top[-1] - top[-2]) / abs(top[-1]) > 1e-3:
        assert int(best.item()) == ref.best
