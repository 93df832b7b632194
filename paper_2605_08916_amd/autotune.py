"""Launch-configuration autotuner for the fused persistent chain-step kernel.

It sweeps the kernel form (straight-line or ray-refill), the threads per
block, the resident blocks per compute unit of the persistent grid, the number
of chains a lane takes per queue pop, lanes per chain, the ordering of chains
(none, by path length, by screen tile) and the refill thresholds, times
`dr_step(n)` (n steps per launch, as the caller will issue them) for each
candidate with HIP events on the launch stream, and caches the fastest configuration in a JSON file keyed by device name, path
length, chain count and triangle count.  The chain state is saved before and
restored after the sweep, so tuning does not advance the chains.
"""
from __future__ import annotations

import json
import os

from . import dr

CACHE = os.environ.get("DR_AUTOTUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "drestore_autotune.json"))

BLOCKS = (64, 128, 256)
BLOCKS_PER_CU = (1, 2, 3, 4, 6, 8)
GRABS = (1,)
LANES = (1, 2)
# chain ordering before a launch: (sort_by_length, sort_by_tile), 1 on, 2 off
ORDERS = ((2, 2), (1, 2), (2, 1))
REFILL_PCTS = ((50, 50),)  # (event, advance) thresholds of the ray-refill form


def candidates():
    """Every launch configuration the sweep times: the straight-line form
    over block x blocks-per-CU x grab x lanes x ordering, and the ray-refill
    form (one lane per chain) over block x blocks-per-CU x ordering x
    thresholds."""
    out = []
    for block in BLOCKS:
        for bpc in BLOCKS_PER_CU:
            for by_len, by_tile in ORDERS:
                for grab in GRABS:
                    for lanes in LANES:
                        out.append(dict(block=block, blocks_per_cu=bpc, grab=grab, lanes_per_chain=lanes,
                                        sort_by_length=by_len, sort_by_tile=by_tile, refill=2))
                for ev, adv in REFILL_PCTS:
                    out.append(dict(block=block, blocks_per_cu=bpc, sort_by_length=by_len, sort_by_tile=by_tile,
                                    refill=1, refill_event_pct=ev, refill_advance_pct=adv))
    return out


def _key(ch: "dr.Chains") -> str:
    import torch
    name = torch.cuda.get_device_name()
    return f"{name}|L{ch.L}|N{ch.N}|T{int(ch.scene.sc['indices'].shape[0])}"


def _load() -> dict:
    try:
        with open(CACHE) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _time(ch: "dr.Chains", reps: int, per_launch: int) -> float:
    import torch
    s = torch.cuda.current_stream()
    ch.step(per_launch)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        ch.step(per_launch)
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / (reps * per_launch)


def tune(ch: "dr.Chains", reps: int = 3, use_cache: bool = True, verbose: bool = False, per_launch: int = 8) -> dict:
    """Pick and apply the fastest launch configuration for this chain set
    (time per chain-step with `per_launch` steps per launch)."""
    key = _key(ch) + f"|F{per_launch}"
    cache = _load() if use_cache else {}
    if key in cache:
        cfg = cache[key]["cfg"]
        ch.set_launch(**cfg)
        return cache[key]
    snap = ch.read_state()
    results = []
    for cfg in candidates():
        ch.set_launch(**cfg)
        ms = _time(ch, reps, per_launch)
        results.append((ms, cfg))
        if verbose:
            print(f"autotune {cfg}: {ms:.3f} ms/step")
    results.sort(key=lambda r: r[0])
    best_ms, best = results[0]
    ch.set_launch(**best)
    ch.write_state(x=snap["x"], score=snap["score"], killed=snap["killed"], accum=snap["accum"], step=snap["step"],
                   tour_count=snap["tour_count"], k0=snap["k0"])
    entry = {"cfg": best, "ms": best_ms, "sweep": [(ms, c) for ms, c in results]}
    cache[key] = entry
    try:
        os.makedirs(os.path.dirname(CACHE), exist_ok=True)
        with open(CACHE, "w") as f:
            json.dump(cache, f, indent=1)
    except OSError:
        pass
    return entry
