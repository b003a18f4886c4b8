"""ngs_info_gain_static (the entry point that allocates nothing: its workspace is the
library's fixed device scratch array) against ngs_info_gain on the same inputs, through the C
ABI: two calls in a row, the second on a smaller input, so that the second reads the array
after the first has left its contents there. Named to be collected last."""
import sys

import numpy as np
import pytest

import scenegen
from parity_util import check_gain

pytestmark = pytest.mark.gpu


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def B():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2602_08266_amd import binding
    binding.lib()
    return binding


def _gain_both(B, ctx, scene, cam, ig, h, target):
    import torch
    ds = B.DeviceScene(scene, "cuda")
    B.ngs_prepare_scene(ctx, ds, B.ig_params(target_id=target))
    rp = B.raster_params()
    c = B.camera(cam)
    pr = B.ngs_project(ctx, ds, c, rp)
    lists = B.ngs_bin_sort(ctx, ds, pr, c, rp, capacity=1 << 20)
    ws = B.IgWorkspace(ds, 1 << 14)
    ref = B.ngs_info_gain(ctx, ds, pr, lists, c, rp, ig, h, ws).cpu().numpy()
    out = torch.full((3,), float("nan"), dtype=torch.float64, device="cuda")
    st = torch.zeros(B.STATS_LEN, dtype=torch.int64, device="cuda")
    got = B.ngs_info_gain_static(ctx, ds, pr, lists, c, rp, ig, h, out, st).cpu().numpy()
    return ref, got, st.cpu().numpy()


def test_static_entry_matches_workspace_entry_twice(B):
    ctx = B.Context(0)
    # call 1: 2,000 Gaussians at 128 x 96 with a training store (H_T from four views)
    cfg, scene, cands, train = scenegen.make_workload("tiny", 0)
    log("no-alloc call 1: tiny workload, view 2, training store, whole scene")
    ds = B.DeviceScene(scene, "cuda")
    scorer = B.NbvScorer(ctx, ds, B.raster_params(), B.ig_params(), max_pairs=1 << 18, max_slots=1 << 14,
                         store_capacity=1 << 14)
    scorer.setup([B.camera(c) for c in train])
    ref, got, st = _gain_both(B, ctx, scene, cands[2], B.ig_params(), scorer.h, -1)
    check_gain(got, ref, "call 1")
    assert st[2] > 0 and st[5] == 0
    log(f"  workspace entry {ref}, static entry {got}")
    # call 2: a smaller input (500 Gaussians at 64 x 48, object-centric, no store)
    small = scenegen.make_scene(500, 4, 8, seed=7)
    cam = scenegen.look_at(np.array([0.45, 0.2, 0.35]), 64, 48, 50.0)
    log("no-alloc call 2: 500 Gaussians at 64 x 48, target 2, no store")
    ig2 = B.ig_params(target_id=2)
    ref2, got2, st2 = _gain_both(B, ctx, small, cam, ig2, None, 2)
    check_gain(got2, ref2, "call 2")
    assert np.all(ref2 > 0)
    log(f"  workspace entry {ref2}, static entry {got2}")
    ctx.close()


def test_static_entry_rejects_scenes_beyond_the_array(B):
    """A scene whose per-Gaussian slot table alone exceeds the fixed array is refused before
    any device work (no pointer of the struct is read)."""
    import ctypes as C
    ctx = B.Context(0)
    big = B.ngs_scene()
    big.n, big.k = 64 << 20, 16
    st = B.lib().ngs_info_gain_static(ctx.handle, C.byref(big), None, None, None, None, None, None, None, None,
                                      None)
    assert st == B.NGS_WORKSPACE_TOO_SMALL
    ctx.close()
