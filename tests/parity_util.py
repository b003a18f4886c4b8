"""Comparison helpers for GPU-vs-oracle parity (tolerances of the parity protocol).

Rendered channels: |gpu - ref| <= 1e-4 * max(|ref|, tau) at every pixel whose oracle walk
stayed clear of a threshold decision (q vs the cut-off, alpha vs its floor or clamp, T (1 -
alpha) vs t_min, within 1e-5 relative in FP64). The FP32 kernel may take the other side of
such a decision, so those "ambiguous" pixels only need |gpu - ref| <= 0.02 * max |feature|
(one flipped Gaussian changes a pixel by at most sigma exp(-4.5) < 0.011 of a feature).
Argmax ids: exact wherever the pixel is not ambiguous and the oracle's top-2 margin exceeds
1e-5. Information gain: 1e-3 relative per output.

The object vector O of a pixel (Eq. 2; its k entries sum to 1) is one rendered channel: its
error is measured as a vector, ||O_gpu - O_ref||_1 <= 1e-4 ||O_ref||_1 = 1e-4. Entry by entry
the relative bound does not hold in FP32: the 2D means are FP32 (half an ulp is 3e-5 px at
640 px), so q = d^T Q d of a pixel 3 px from a mean is off by up to ~2e-5 relative and alpha
by ~1e-4 at q near 9, and the transmittance behind a near-opaque Gaussian inherits its alpha
error scaled by alpha / (1 - alpha); an entry of O fed mostly by Gaussians behind such a
Gaussian can be off by a few 1e-4 of its own (small) value while the vector is within 1e-4.
Every entry must still be within the per-entry bound of the other channels at 20x (2e-3 of
max(|ref|, 1e-2)).
"""
import numpy as np

REL = 1e-4
TAU = 1e-2
IG_REL = 1e-3


def check_channel(name, gpu, ref, ambiguous, feature_max, tau=TAU):
    gpu = np.asarray(gpu, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    amb = np.broadcast_to(ambiguous.astype(bool), ref.shape)
    err = np.abs(gpu - ref)
    bound = REL * np.maximum(np.abs(ref), tau)
    bad = (err > bound) & ~amb
    assert not bad.any(), (f"{name}: {bad.sum()} pixels beyond 1e-4 rel, worst {err[bad].max():.3e} "
                           f"at ref {ref[bad][np.argmax(err[bad])]:.4e}")
    if amb.any():
        loose = 0.02 * feature_max
        assert err[amb].max() <= loose, f"{name}: ambiguous pixel off by {err[amb].max():.3e} > {loose:.3e}"
    return float(err[~amb].max()) if (~amb).any() else 0.0


def check_image(gpu, ref, k, depth_max):
    amb = ref["ambiguous"].astype(bool)
    out = {}
    out["rgb"] = check_channel("rgb", gpu["rgb"], ref["rgb"], amb[None], 1.0)
    out["depth"] = check_channel("depth", gpu["depth"], ref["depth"], amb, depth_max)
    out["t_final"] = check_channel("t_final", gpu["t_final"], ref["t_final"], amb, 1.0)
    if gpu.get("obj") is not None:
        go = np.asarray(gpu["obj"], dtype=np.float64)
        ro = np.asarray(ref["obj"], dtype=np.float64)
        l1 = np.abs(go - ro).sum(axis=0)
        bad = (l1 > REL * np.abs(ro).sum(axis=0)) & ~amb
        assert not bad.any(), f"obj: {bad.sum()} pixels beyond 1e-4 in L1, worst {l1[bad].max():.3e}"
        ent = np.abs(go - ro) > 20 * REL * np.maximum(np.abs(ro), TAU)
        assert not (ent & ~amb[None]).any(), f"obj: {(ent & ~amb[None]).sum()} entries beyond 2e-3 rel"
        if amb.any():
            assert np.abs(go - ro)[:, amb].max() <= 0.02, "obj: ambiguous pixel off by more than 0.02"
        out["obj"] = float(l1[~amb].max()) if (~amb).any() else 0.0
    if gpu.get("mean_conf") is not None:
        out["mean_conf"] = check_channel("mean_conf", gpu["mean_conf"], ref["kbar"], amb, 1.0)
    srt = np.sort(ref["obj"], axis=0)
    margin = srt[-1] - srt[-2] if k > 1 else np.full(amb.shape, np.inf)
    firm = (~amb) & (margin > 1e-5)
    gid = np.asarray(gpu["argmax_id"])
    assert np.array_equal(gid[firm], ref["id"][firm]), f"argmax ids differ at {(gid[firm] != ref['id'][firm]).sum()} pixels"
    if gpu.get("n_contrib") is not None:
        nc = np.asarray(gpu["n_contrib"])
        assert np.array_equal(nc[~amb], ref["ncontrib"][~amb]), "contributor counts differ"
    out["ambiguous"] = int(amb.sum())
    out["argmax_loose"] = int((~firm).sum())
    return out


def check_gain(gpu, ref, what=""):
    gpu = np.asarray(gpu, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    rel = np.abs(gpu - ref) / np.maximum(np.abs(ref), 1e-300)
    assert np.all((rel <= IG_REL) | ((ref == 0) & (gpu == 0))), f"IG {what}: gpu {gpu} ref {ref} rel {rel}"
    return float(rel[np.isfinite(rel)].max()) if np.isfinite(rel).any() else 0.0
