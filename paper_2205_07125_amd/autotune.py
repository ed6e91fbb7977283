"""Launch-shape autotuner: picks, per network shape, the snn_tuning values
(persistent update blocks, receive-side blocks per destination node, the
receive side as one launch or two) that run whole steps fastest on this GPU,
and caches the choice.

None of the choices changes a result (the GPU tests check each against the
default), so the tuner only times: for every candidate it replays whole
steps from HIP graphs on the simulation's stream, bracketed by HIP events,
and keeps the candidate with the least time per step.  Tuning runs the
simulation forward by (warmup + steps) steps per candidate.

The cache is a JSON file keyed by the shape (neurons, partitions, group
size, tiles, synapses, weight type, drive) and the device name; a later run
of the same shape on the same kind of device reuses the entry without
timing anything.
"""
from __future__ import annotations

import json
import os
import time

from . import _abi

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "paper_2205_07125_amd",
                             "tuning.json")


def shape_key(sim) -> str:
    import torch
    wl = sim.wl
    tiles = -(-wl.n_neurons // sim.tile_neurons)
    nnz = int(sim.host.nnz) if sim.host is not None else -1
    dev = torch.cuda.get_device_name(sim.device)
    return (f"{dev}|N={wl.n_neurons}|P={wl.n_partitions}|G={wl.gpus_per_node}|tiles={tiles}|"
            f"K={wl.k_in}|nnz={nnz}|w={wl.weight_type}|topo={wl.topology}|"
            f"rate={wl.rate_on_hz if wl.forced else 'lif'}")


def candidates(sim, cu_count: int | None = None) -> list[dict]:
    """update_blocks: one block per tile, or persistent grids of 1, 2 and 3
    blocks per CU where that is fewer than the tiles; recv_split: one block
    per destination node up to as many as the 256 receive-side blocks allow;
    recv_merged: both forms of the receive side."""
    import torch
    wl = sim.wl
    tiles = -(-wl.n_neurons // sim.tile_neurons)
    if cu_count is None:
        cu_count = torch.cuda.get_device_properties(sim.device).multi_processor_count
    ub = [0] + [k * cu_count for k in (1, 2, 3) if k * cu_count < tiles]
    nodes = wl.n_nodes
    rs = [0]
    if nodes < 256:
        rs += [s for s in (1, 2, 4, 8, 16, 32, 64) if s < 256 // nodes]
    return [{"update_blocks": u, "recv_split": r, "recv_merged": m}
            for u in ub for r in rs for m in (0, 1)]


def time_candidate(sim, cand: dict, steps: int, warmup: int, mode: int) -> float:
    """ms per whole step with tuning `cand` (HIP events on the sim's stream)."""
    import torch
    sim.set_tuning(**cand)
    sim.run(warmup, mode, use_graph=True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    sim.sync()
    e0.record(sim.stream)
    sim.run(steps, mode, use_graph=True)
    e1.record(sim.stream)
    sim.stream.synchronize()
    return e0.elapsed_time(e1) / steps


def tune(sim, mode: int = _abi.SNN_ROUTE_TWO_LEVEL, steps: int = 64, warmup: int = 16,
         cache: str | None = DEFAULT_CACHE, force: bool = False, log=None) -> dict:
    """Picks and applies the fastest tuning for sim's shape; -> {"tuning",
    "ms_per_step", "timings", "cached"}."""
    key = shape_key(sim) + f"|mode={mode}"
    db = {}
    if cache and os.path.exists(cache):
        with open(cache) as fh:
            db = json.load(fh)
    if not force and key in db:
        ent = db[key]
        sim.set_tuning(**ent["tuning"])
        return dict(ent, cached=True)
    timings = []
    t0 = time.time()
    for cand in candidates(sim):
        ms = time_candidate(sim, cand, steps, warmup, mode)
        timings.append({"tuning": cand, "ms_per_step": ms})
        if log:
            log(f"autotune {cand}: {ms * 1e3:.1f} us/step")
    best = min(timings, key=lambda x: x["ms_per_step"])
    ent = {"tuning": best["tuning"], "ms_per_step": best["ms_per_step"], "timings": timings,
           "seconds": time.time() - t0}
    sim.set_tuning(**best["tuning"])
    if cache:
        os.makedirs(os.path.dirname(cache), exist_ok=True)
        db[key] = ent
        tmp = cache + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(db, fh, indent=1, sort_keys=True)
        os.replace(tmp, cache)
    return dict(ent, cached=False)
