"""Launch-configuration autotuner for the fused persistent chain-step kernel.

It searches the kernel form (straight-line or ray-refill), the threads per
block, the resident blocks per compute unit of the persistent grid, the number
of consecutive chains a lane (or lane pair) takes per pop of the device work
queue (the queue's batch depth), lanes per chain, the ordering of chains
(none, by path length, by screen tile) and the refill thresholds.  Each candidate is timed on the live chain set
as `dr_step(n)` launches (n steps per launch, as the caller will issue them)
with HIP events on the launch stream.  The default search is staged
(coordinate descent: block x blocks per CU first, then each other dimension
in turn from the best so far, about 28 candidates); `exhaustive=True` times
the full product.  The fastest configuration is cached in a JSON file keyed
by device name, path length, chain count, triangle count and steps per
launch.  The chain state is saved before and restored after the sweep
(unless the caller re-initialises the chains anyway), so tuning does not
advance the chains.
"""
from __future__ import annotations

import json
import os

from . import dr

CACHE = os.environ.get("DR_AUTOTUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "drestore_autotune.json"))

BLOCKS = (64, 128, 256)
BLOCKS_PER_CU = (1, 2, 3, 4, 6, 8)
GRABS = (1, 2, 4)          # chains per lane per queue pop
LANES = (1, 2)
# chain ordering before a launch: (sort_by_length, sort_by_tile), 1 on, 2 off
ORDERS = ((2, 2), (1, 2), (2, 1))
REFILL_PCTS = ((50, 50), (75, 50), (75, 75), (90, 75))  # (event, advance) thresholds of the ray-refill form


def candidates():
    """Every launch configuration the exhaustive sweep times: the
    straight-line form over block x blocks-per-CU x grab x lanes x ordering,
    and the ray-refill
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
    # the leading tag changes whenever the launch fields do, so entries that
    # name fields the library no longer has are never applied
    return f"launch2|{name}|L{ch.L}|N{ch.N}|T{int(ch.scene.sc['indices'].shape[0])}"


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


def staged_candidates(ch: "dr.Chains", timer) -> list:
    """Coordinate descent over the launch dimensions; timer(cfg) -> ms per
    step.  Returns [(ms, cfg)] of every configuration timed."""
    results = []

    def run(cfgs):
        for c in cfgs:
            results.append((timer(c), c))
        return min(results, key=lambda r: r[0])[1]

    base = dict(sort_by_length=2, sort_by_tile=2, refill=2, grab=1)
    best = run([dict(base, block=b, blocks_per_cu=k) for b in BLOCKS for k in BLOCKS_PER_CU])
    best = run([dict(best, lanes_per_chain=n) for n in LANES])
    best = run([dict(best, sort_by_length=a, sort_by_tile=b) for a, b in ORDERS[1:]])
    best = run([dict(best, grab=g) for g in GRABS[1:]])
    run([dict(best, refill=1, refill_event_pct=ev, refill_advance_pct=adv) for ev, adv in REFILL_PCTS])
    return results


def tune_init(ch: "dr.Chains", reps: int = 2, frame0: int = 1 << 20) -> dict:
    """Time the initialise pass in its straight-line and ray-refill forms on
    the live chains (it re-initialises them) and apply the faster."""
    import torch
    s = torch.cuda.current_stream()
    out = {}
    for rf in (2, 1):
        ch.set_launch(init_refill=rf)
        ch.reinit(frame0)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for r in range(reps):
            ch.reinit(frame0 + 1 + r)
        e1.record(s)
        torch.cuda.synchronize()
        out["refill" if rf == 1 else "straight"] = e0.elapsed_time(e1) / reps
    best = 1 if out["refill"] < out["straight"] else 2
    ch.set_launch(init_refill=best)
    out["init_refill"] = best
    return out


def tune(ch: "dr.Chains", reps: int = 3, use_cache: bool = True, verbose: bool = False, per_launch: int = 8,
         exhaustive: bool = False, restore: bool = True, keep_within: float = 0.0) -> dict:
    """Pick and apply the fastest launch configuration for this chain set
    (time per chain-step with `per_launch` steps per launch).  restore=False
    skips saving and restoring the chain state (for callers that
    re-initialise the chains afterwards).  keep_within: keep the chain set's
    current configuration unless the best is faster by more than this
    fraction (timing noise does not flip the choice)."""
    key = _key(ch) + f"|F{per_launch}"
    cache = _load() if use_cache else {}
    if key in cache:
        cfg = cache[key]["cfg"]
        ch.set_launch(**cfg)
        return cache[key]
    snap = ch.read_state() if restore else None
    full = dict(sort_by_length=2, sort_by_tile=2, refill=2, grab=1, refill_event_pct=50, refill_advance_pct=50)
    flags = ("sort_by_length", "sort_by_tile", "refill", "wavefront", "init_refill")  # read back 1/0, requested 1 on / 2 off
    current = {k: ((1 if v else 2) if k in flags else v) for k, v in ch.get_launch().items()}
    ch.set_launch(**current)
    current_ms = _time(ch, reps, per_launch)

    def timer(cfg):
        ch.set_launch(**dict(full, **cfg))
        ms = _time(ch, reps, per_launch)
        if verbose:
            print(f"autotune {cfg}: {ms:.3f} ms/step")
        return ms

    if exhaustive:
        results = [(timer(c), c) for c in candidates()]
    else:
        results = staged_candidates(ch, timer)
    results.sort(key=lambda r: r[0])
    best_ms, best = results[0]
    if best_ms >= current_ms * (1.0 - keep_within):
        best_ms, best = current_ms, current
    ch.set_launch(**dict(full, **best))
    if snap is not None:
        ch.write_state(x=snap["x"], score=snap["score"], killed=snap["killed"], accum=snap["accum"],
                       step=snap["step"], tour_count=snap["tour_count"], k0=snap["k0"])
    entry = {"cfg": dict(full, **best), "ms": best_ms, "current_ms": current_ms,
             "sweep": [(ms, c) for ms, c in results]}
    cache[key] = entry
    try:
        os.makedirs(os.path.dirname(CACHE), exist_ok=True)
        with open(CACHE, "w") as f:
            json.dump(cache, f, indent=1)
    except OSError:
        pass
    return entry
