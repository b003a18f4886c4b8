"""GPU parity of the backward rasterizer: parameter gradients through the C ABI against the
FP64 oracle's gradient (sum over pixels of image gradient times Jacobian rows), on seeded
scenes and seeded image gradients. Image gradients are zeroed at pixels whose oracle walk
came within 1e-5 of a threshold decision, where FP32 and FP64 may legitimately composite
different sets (the same exclusion as the image parity)."""
import sys

import numpy as np
import pytest

import oracle
import scenegen

pytestmark = pytest.mark.gpu

GROUPS = (("mean", slice(0, 3)), ("log_scale", slice(3, 6)), ("rot", slice(6, 10)), ("opacity_logit", slice(10, 11)),
          ("rgb", slice(11, 14)))
REL = 1e-3  # per entry, relative to the largest |gradient| of its parameter group, plus 1e-3 of itself


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


def image_grads(scene, cam, seed, eq2=1):
    """Seeded image gradients, zero at ambiguous pixels of the oracle's walk."""
    rng = np.random.default_rng(seed)
    H, W, k = cam.height, cam.width, scene.k
    ref = oracle.render(scene, cam, ig=oracle.IGParams(obj_eq2=eq2))
    keep = (ref["ambiguous"] == 0).astype(np.float64)
    g = dict(rgb=rng.normal(size=(3, H, W)) * keep, depth=rng.normal(size=(H, W)) * keep,
             obj=rng.normal(size=(k, H, W)) * keep)
    return {x: v.astype(np.float32) for x, v in g.items()}, int((keep == 0).sum())


def gpu_grads(B, ctx, scene, cam, g, eq2=1):
    import torch
    ds = B.DeviceScene(scene, "cuda")
    B.ngs_prepare_scene(ctx, ds, B.ig_params())
    c = B.camera(cam)
    rp = B.raster_params()
    pr = B.ngs_project(ctx, ds, c, rp)
    ls = B.ngs_bin_sort(ctx, ds, pr, c, rp, capacity=1 << 22)
    t = lambda a: torch.as_tensor(a, device="cuda")
    out = B.ngs_render_backward(ctx, ds, pr, ls, c, rp, t(g["rgb"]), t(g["depth"]), t(g["obj"]), obj_eq2=bool(eq2))
    torch.cuda.synchronize()
    n = scene.n
    flat = np.concatenate([out["mean"].cpu().numpy().T, out["log_scale"].cpu().numpy().T, out["rot"].cpu().numpy().T,
                           out["opacity_logit"].cpu().numpy().reshape(n, 1), out["rgb"].cpu().numpy().T,
                           out["obj_logit"].cpu().numpy().T], axis=1)
    return flat.astype(np.float64)


def check_grads(got, ref, label):
    k = ref.shape[1] - 14
    groups = list(GROUPS) + [("obj_logit", slice(14, 14 + k))]
    for name, sl in groups:
        r, gv = ref[:, sl], got[:, sl]
        scale = np.abs(r).max()
        assert scale > 0, (label, name)
        err = np.abs(gv - r)
        tol = REL * scale + REL * np.abs(r)
        bad = err > tol
        assert not bad.any(), (label, name, int(bad.sum()), float(err.max() / scale))
        log(f"  {label} {name}: max err / scale {err.max() / scale:.2e}")


@pytest.mark.parametrize("view,eq2", [(0, 1), (3, 1), (5, 0)])
def test_backward_tiny_matches_oracle(B, ctx, view, eq2):
    log(f"test_backward_tiny view {view} eq2 {eq2}")
    cfg, scene, cands, train = scenegen.make_workload("tiny", 0)
    cam = cands[view]
    g, amb = image_grads(scene, cam, seed=100 + view, eq2=eq2)
    ref = oracle.render_grad(scene, cam, g["rgb"], g["depth"], g["obj"], ig=oracle.IGParams(obj_eq2=eq2))
    got = gpu_grads(B, ctx, scene, cam, g, eq2)
    log(f"  ambiguous pixels zeroed: {amb}")
    check_grads(got, ref, f"tiny view {view}")


def test_backward_ragged_view(B, ctx):
    """A 100 x 70 view: partial tiles on both edges."""
    log("test_backward_ragged_view")
    cfg, scene, cands, train = scenegen.make_workload("tiny", 0)
    c0 = cands[1]
    cam = scenegen.Camera(R=c0.R, t=c0.t, fx=c0.fx * 100 / 128, fy=c0.fy * 100 / 128, cx=50.0, cy=35.0, width=100,
                          height=70)
    g, _ = image_grads(scene, cam, seed=7)
    ref = oracle.render_grad(scene, cam, g["rgb"], g["depth"], g["obj"])
    got = gpu_grads(B, ctx, scene, cam, g)
    check_grads(got, ref, "ragged")


def test_backward_diff_workload_view(B, ctx):
    """500k Gaussians (k = 32) at 640 x 480, one view, every parameter compared."""
    log("test_backward_diff_workload_view")
    cfg, scene, cands, train = scenegen.make_workload("diff", 0, n_views=1)
    cam = cands[0]
    g, amb = image_grads(scene, cam, seed=9)
    ref = oracle.render_grad(scene, cam, g["rgb"], g["depth"], g["obj"])
    got = gpu_grads(B, ctx, scene, cam, g)
    log(f"  ambiguous pixels zeroed: {amb}; Gaussians with gradient {int((np.abs(ref).sum(1) > 0).sum())}")
    check_grads(got, ref, "diff view 0")


def test_autograd_function_matches_direct_call(B, ctx):
    """torch autograd through RenderFunction (an L1 + L1 + cross-entropy loss) gives the same
    parameter gradients as ngs_render_backward called with torch's image gradients."""
    import torch
    log("test_autograd_function")
    cfg, scene, cands, train = scenegen.make_workload("tiny", 0)
    cam = B.camera(cands[2])
    t = lambda a: torch.as_tensor(np.asarray(a, np.float32), device="cuda").contiguous().requires_grad_(True)
    params = [t(scene.mean), t(scene.log_scale), t(scene.rot), t(scene.opacity_logit), t(scene.rgb), t(scene.obj_logit)]
    rgb, depth, obj = B.render(*params, ctx, cam)
    rng = np.random.default_rng(4)
    tgt_rgb = torch.as_tensor(rng.uniform(0, 1, rgb.shape).astype(np.float32), device="cuda")
    tgt_d = torch.as_tensor(rng.uniform(0, 1, depth.shape).astype(np.float32), device="cuda")
    labels = torch.as_tensor(rng.integers(0, scene.k, depth.shape), device="cuda")
    loss = (rgb - tgt_rgb).abs().sum() + (depth - tgt_d).abs().sum() + \
        torch.nn.functional.nll_loss(torch.log(obj.clamp_min(1e-6)).unsqueeze(0), labels.unsqueeze(0), reduction="sum")
    loss.backward()
    # the same image gradients through the direct entry
    rgb2, depth2, obj2 = [x.detach().requires_grad_(True) for x in (rgb, depth, obj)]
    l2 = (rgb2 - tgt_rgb).abs().sum() + (depth2 - tgt_d).abs().sum() + \
        torch.nn.functional.nll_loss(torch.log(obj2.clamp_min(1e-6)).unsqueeze(0), labels.unsqueeze(0), reduction="sum")
    l2.backward()
    ds = B.DeviceScene(scene, "cuda")
    B.ngs_prepare_scene(ctx, ds, B.ig_params())
    rp = B.raster_params()
    pr = B.ngs_project(ctx, ds, cam, rp)
    ls = B.ngs_bin_sort(ctx, ds, pr, cam, rp)
    direct = B.ngs_render_backward(ctx, ds, pr, ls, cam, rp, rgb2.grad, depth2.grad, obj2.grad)
    for name, p in zip(("mean", "log_scale", "rot", "opacity_logit", "rgb", "obj_logit"), params):
        assert p.grad is not None and torch.isfinite(p.grad).all()
        a, b = p.grad.cpu().numpy(), direct[name].cpu().numpy()
        assert np.allclose(a, b, rtol=1e-4, atol=1e-5 * max(1.0, np.abs(b).max())), name
