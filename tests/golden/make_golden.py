"""Writes the FP64 oracle's information gains for the full-size workloads.

Every value in the JSON files this script writes comes from ``oracle.score`` (FP64 CPU
oracle) on scenes and cameras regenerated from their seeds by ``scenegen``; nothing is taken
from the GPU path. Run from the repository root:

    python tests/golden/make_golden.py [mid|batched640|batched ...]
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import scenegen  # noqa: E402

SPECS = {
    # whole-scene scoring (Eq. 7), 200k Gaussians, k = 32, 640x480
    "mid": dict(seed=0, views=[0, 1, 40]),
    # object-centric scoring of the seeded target (Eq. 12), 1M Gaussians, k = 64, 640x480
    "batched640": dict(seed=0, views=[0, 17, 60]),
    # the mixed-resolution batch: one view from each third (320x240, 640x480, 1280x720; view
    # 200 is the batch's largest, 85M pairs)
    "batched": dict(seed=0, views=[5, 120, 200]),
}


def make(name):
    spec = SPECS[name]
    cfg, scene, cands, train = scenegen.make_workload(name, spec["seed"])
    ig = oracle.IGParams(target_id=scene.target)
    sel = [cands[v] for v in spec["views"]]
    t0 = time.time()
    r = oracle.score(scene, train, sel, ig=ig)
    out = {
        "_source": "FP64 oracle (oracle.score) on scenegen workload %r, seed %d; written by "
                   "tests/golden/make_golden.py" % (name, spec["seed"]),
        "workload": name, "seed": spec["seed"], "target_id": scene.target, "views": spec["views"],
        "status": r.status, "ig_train": r.ig_train.tolist(), "norm": r.norm.tolist(),
        "ig_cand": r.ig_cand.tolist(), "scores": r.scores.tolist(), "best_of_views": r.best,
        "touched": r.stats[:, 0].tolist(), "contrib_pairs": r.stats[:, 1].tolist(),
        "oracle_seconds": round(time.time() - t0, 1),
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"ig_{name}_seed{spec['seed']}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(path, out["oracle_seconds"], "s", flush=True)


if __name__ == "__main__":
    for n in (sys.argv[1:] or list(SPECS)):
        make(n)
