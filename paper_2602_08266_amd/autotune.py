"""Autotuner of the batched scorer's launch shapes.

It times ngs_score_batch on a sample of the real candidate set for every combination of
views_in_flight (buffer sets and context streams kept busy at once), lanes per pixel of the
information-gain back pass (which sets its workgroup size and the packed rows it stages in LDS
per reduction round) and, where the library has both builds, its waves per SIMD (one or two
workgroups per CU), then at the fastest of those the chunk size of the second binning level and
the number of view groups in flight; keeps the fastest, and applies it to the context
(ngs_set_tuning) and to the scorer's workspace. Results may be cached in a JSON file keyed by the device, the scene
size and the resolution mix of the sample.
"""
from __future__ import annotations

import json
import os
import time
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence, Tuple

import torch

from . import binding as B

VIEWS_IN_FLIGHT = (2, 4, 8, 12, 16, 24, 32)
BIN_CHUNKS = (1024, 2048, 4096)  # tried at the best shape after the default (512)
GROUPS = (1, 3, 4)  # groups in flight tried at the best shape after the default (2) ...
GROUP_SHAPES = ((48, 3), (64, 4))  # ... and (views in flight, groups) with full groups of 16
CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning_cache.json")


def lpp_choices(k: int) -> Tuple[int, ...]:
    """Lanes per pixel the library accepts for object vectors of length k."""
    if k <= 8:
        return (1, 2)
    if k <= 32:
        return (1, 2, 4)
    return (1, 2)


def waves_choices(k: int, lpp: int) -> Tuple[int, ...]:
    """Waves per SIMD of the back pass the library accepts (0 = the default build)."""
    return (0, 4) if lpp == 2 and k > 16 else (0,)


@dataclass
class TuneResult:
    views_in_flight: int
    ig_lanes_per_pixel: int
    ms_per_view: float
    table: List[Dict] = field(default_factory=list)
    cached: bool = False
    ig_waves_per_simd: int = 0
    bin_chunk: int = 0
    groups_in_flight: int = 0


def _key(scene: B.DeviceScene, cams: Sequence[B.ngs_camera], max_pairs: int, max_slots: int) -> str:
    res: Dict[str, int] = {}
    for c in cams:
        r = f"{c.width}x{c.height}"
        res[r] = res.get(r, 0) + 1
    dev = (torch.cuda.get_device_properties(torch.cuda.current_device()).gcnArchName.split(":")[0]
           if torch.cuda.is_available() else "none")
    return json.dumps({"dev": dev, "n": scene.n, "k": scene.k, "res": sorted(res.items()), "pairs": max_pairs,
                       "slots": max_slots}, sort_keys=True)


def tune_score(ctx: B.Context, scorer: B.NbvScorer, cams: Sequence[B.ngs_camera], sample: int = 64,
               reps: int = 2, vif: Sequence[int] = VIEWS_IN_FLIGHT, lpps: Optional[Sequence[int]] = None,
               cache: Optional[str] = None, write_cache: bool = True, log=None) -> TuneResult:
    """Times every (views_in_flight, lanes per pixel) pair on `sample` evenly spaced candidates
    (after one untimed batch), best of `reps`; applies the winner to ctx and scorer. With a
    cache file, a stored result for the same device, scene size and resolution mix is applied
    without timing; new results are added to it when write_cache is set."""
    step = max(1, len(cams) // sample)
    sub = list(cams[::step][:sample])
    key = _key(scorer.scene, sub, scorer.max_pairs, scorer.max_slots)
    if cache and os.path.exists(cache):
        with open(cache) as f:
            hit = json.load(f).get(key)
        if hit:
            res = TuneResult(hit["views_in_flight"], hit["ig_lanes_per_pixel"], hit["ms_per_view"], hit["table"],
                             cached=True, ig_waves_per_simd=hit.get("ig_waves_per_simd", 0),
                             bin_chunk=hit.get("bin_chunk", 0), groups_in_flight=hit.get("groups_in_flight", 0))
            apply(ctx, scorer, res)
            return res
    lpps = tuple(lpps) if lpps else lpp_choices(scorer.scene.k)
    table = []
    best = None
    for lpp in lpps:
        for waves in waves_choices(scorer.scene.k, lpp):
            B.ngs_set_tuning(ctx, lpp, waves)
            for v in vif:
                scorer.views_in_flight = v
                scorer.ws = None  # resized for v buffer sets on the next score()
                scorer.score(sub)
                torch.cuda.synchronize()
                t = float("inf")
                for _ in range(reps):
                    t0 = time.perf_counter()
                    scorer.score(sub)
                    torch.cuda.synchronize()
                    t = min(t, time.perf_counter() - t0)
                ms = t / len(sub) * 1e3
                table.append({"views_in_flight": v, "ig_lanes_per_pixel": lpp, "ig_waves_per_simd": waves,
                              "ms_per_view": round(ms, 4)})
                if log:
                    log(f"autotune: views_in_flight {v:2d}, lanes per pixel {lpp}, waves per SIMD {waves}: "
                        f"{ms:.3f} ms/view")
                if best is None or ms < best[0]:
                    best = (ms, v, lpp, waves)
    # then the binning chunk size at the best shape
    best_chunk = 0
    scorer.views_in_flight = best[1]
    scorer.ws = None
    for chunk in BIN_CHUNKS:
        B.ngs_set_tuning(ctx, best[2], best[3], chunk)
        scorer.score(sub)
        torch.cuda.synchronize()
        t = float("inf")
        for _ in range(reps):
            t0 = time.perf_counter()
            scorer.score(sub)
            torch.cuda.synchronize()
            t = min(t, time.perf_counter() - t0)
        ms = t / len(sub) * 1e3
        table.append({"views_in_flight": best[1], "ig_lanes_per_pixel": best[2], "ig_waves_per_simd": best[3],
                      "bin_chunk": chunk, "ms_per_view": round(ms, 4)})
        if log:
            log(f"autotune: binning chunk {chunk}: {ms:.3f} ms/view")
        if ms < best[0]:
            best = (ms, best[1], best[2], best[3])
            best_chunk = chunk
    # then the number of view groups in flight (with more buffer sets for more groups)
    best_groups = 0
    # shapes whose buffer sets would take more than 40 % of the device are not tried (a
    # whole-scene workload keeps a statistic row per Gaussian in every set)
    budget = 0.4 * torch.cuda.get_device_properties(torch.cuda.current_device()).total_memory
    for v, groups in [(best[1], gr) for gr in GROUPS] + list(GROUP_SHAPES):
        if groups > v:
            continue
        if B.workspace_size(2, scorer.scene.n, scorer.scene.k, max_pairs=scorer.max_pairs,
                            max_slots=scorer.max_slots, views_in_flight=v) > budget:
            continue
        scorer.views_in_flight = v
        scorer.ws = None
        B.ngs_set_tuning(ctx, best[2], best[3], best_chunk, groups)
        scorer.score(sub)
        torch.cuda.synchronize()
        t = float("inf")
        for _ in range(reps):
            t0 = time.perf_counter()
            scorer.score(sub)
            torch.cuda.synchronize()
            t = min(t, time.perf_counter() - t0)
        ms = t / len(sub) * 1e3
        table.append({"views_in_flight": v, "ig_lanes_per_pixel": best[2], "ig_waves_per_simd": best[3],
                      "bin_chunk": best_chunk, "groups_in_flight": groups, "ms_per_view": round(ms, 4)})
        if log:
            log(f"autotune: {v} views in flight, groups in flight {groups}: {ms:.3f} ms/view")
        if ms < best[0]:
            best = (ms, v, best[2], best[3])
            best_groups = groups
    scorer.ws = None
    res = TuneResult(best[1], best[2], best[0], table, ig_waves_per_simd=best[3], bin_chunk=best_chunk,
                     groups_in_flight=best_groups)
    apply(ctx, scorer, res)
    if cache and write_cache:
        data = {}
        if os.path.exists(cache):
            with open(cache) as f:
                data = json.load(f)
        data[key] = {k: v for k, v in res.__dict__.items() if k != "cached"}
        with open(cache, "w") as f:
            json.dump(data, f, indent=1)
    return res


def apply(ctx: B.Context, scorer: B.NbvScorer, res: TuneResult):
    B.ngs_set_tuning(ctx, res.ig_lanes_per_pixel, res.ig_waves_per_simd, res.bin_chunk, res.groups_in_flight)
    scorer.views_in_flight = res.views_in_flight
    scorer.ws = None
