"""Benchmark of one GPU's share of the simulation step on an MI355X.

One step = neuron update + compaction, routing (two-level by default, with
mask expansion) and synaptic delivery, over the 5e6-neuron / in-degree-1,000
share with 2,000 virtual partitions on 250 nodes of 8 (synthetic, seeded).
The network is built and uploaded before timing; the timed region is K whole
steps replayed from a HIP graph, bracketed by device synchronisation.

Prints one JSON line on stdout (progress goes to stderr):
  value     synaptic events/s (local + remote deliveries over the timed steps)
  roofline  the dominant kernel's algorithmic HBM bytes / its average duration,
            measured with HIP events on the simulation stream
  cpu_baseline  the CPU oracle (single thread) on a bounded sample of the same
            workload structure
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, 8 TB/s


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def code_text(src: str) -> str:
    """Source text without // comments and blank lines: what the compiler
    sees of it (a comment edit does not invalidate measured counters)."""
    lines = []
    for line in src.splitlines():
        code = line.split("//", 1)[0].rstrip()
        if code:
            lines.append(code)
    return "\n".join(lines)


def kernel_source_hash(read=None) -> str:
    h = hashlib.sha256()
    for f in ("snn_kernels.hip", "snn_internal.h"):
        path = os.path.join("paper_2205_07125_amd", "csrc", f)
        if read is None:
            with open(os.path.join(ROOT, path)) as fh:
                text = fh.read()
        else:
            text = read(path)
        h.update(code_text(text).encode())
    return h.hexdigest()[:16]


def _oracle_sample(args):
    """One oracle process: the workload's structure at n neurons with its own
    seed, run for `seconds`; -> (events, steps, seconds)."""
    name, n, seed, seconds = args
    import oracle
    import synth
    wl = synth.get_workload(name).scaled(n)
    wl = wl.replace(seed=wl.seed + seed)
    gen = synth.Generator(wl)
    sim = oracle.Sim(oracle.params_from_workload(wl), gen.edges(), gen.part_map(),
                     synth.initial_u(wl))
    sim.run(20)  # warm
    steps, events, t0 = 0, 0, time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        c, st = sim.run(50)
        steps += 50
        events += int(st[:, oracle.LOCAL_EVENTS].sum() + st[:, oracle.REMOTE_EVENTS].sum())
    return events, steps, time.perf_counter() - t0


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _one_thread():
    # each oracle process computes on one thread; the seeded generator's
    # OpenMP set-up is kept to one as well (read when libgomp loads)
    os.environ["OMP_NUM_THREADS"] = "1"


def cpu_baseline(wl_full, seconds_budget=10.0):
    """The oracle (plain C, FP64 + binary32 trajectories, one thread per
    process) on the same structure at 1/100 of the neurons (same in-degree,
    partitions, rate): one process alone, then one process per available
    core at once, each on its own seeded network; value = the all-core rate.
    The processes are started fresh (spawn), so they inherit no OpenMP or
    GPU runtime state of this process."""
    import multiprocessing as mp
    n = max(wl_full.n_neurons // 100, 1000)
    name = wl_full.name
    ctx = mp.get_context("spawn")
    log(f"cpu baseline (oracle): one process on {n:,} neurons for {seconds_budget:.0f} s")
    with ctx.Pool(1, initializer=_one_thread) as pool:
        ev1, st1, dt1 = pool.apply(_oracle_sample, ((name, n, 0, seconds_budget),))
    cores = min(len(os.sched_getaffinity(0)), 16)
    log(f"cpu baseline: {ev1 / dt1:.3g} events/s on one process; now {cores} processes")
    with ctx.Pool(cores, initializer=_one_thread) as pool:
        res = pool.map(_oracle_sample, [(name, n, i, seconds_budget) for i in range(cores)])
    ev = sum(r[0] for r in res)
    steps = sum(r[1] for r in res)
    dt = max(r[2] for r in res)
    return dict(value=ev / dt, unit="synaptic events/s", cores=cores, kind="oracle",
                cpu_model=cpu_model(), single_thread_value=ev1 / dt1,
                sample=f"{name} structure at {n:,} neurons (1/100), K={wl_full.k_in}: "
                       f"{cores} processes of one thread each, {steps} steps and {ev:,} events "
                       f"in {dt:.1f} s; one process alone {ev1 / dt1:.3g} events/s "
                       f"({1e3 * dt1 / st1:.2f} ms/step)")


def calibrate_copy(nbytes: int, reps: int = 5):
    """A plain device copy of nbytes (read nbytes, write nbytes), repeated:
    the reference that scales rocprofv3's FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    n = nbytes // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"calibrate_copy_bytes": n * 4, "reps": reps}), flush=True)


def pmc_summary(fetch_dir, write_dir, cal_fetch_dir, cal_write_dir, cal_bytes, workload, out):
    """Per-kernel HBM traffic per launch from FETCH_SIZE / WRITE_SIZE runs
    (KiB per dispatch), each scaled by copy_bytes / counter of the copy."""
    import csv
    import statistics

    def per_kernel(d, counter):
        import glob
        files = sorted(glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True))
        if not files:
            raise FileNotFoundError(f"no *counter_collection.csv under {d}")
        rows = list(csv.DictReader(open(files[0])))
        vals = {}
        for r in rows:
            if r["Counter_Name"] != counter:
                continue
            # "void snn::k_update<true>(snn::KParams)" -> "k_update"
            name = r["Kernel_Name"].split("(")[0].split("::")[-1].split("<")[0]
            vals.setdefault(name, []).append(float(r["Counter_Value"]))
        # drop the first third (warm-up steps), median of the rest
        return {k: statistics.median(v[len(v) // 3:]) for k, v in vals.items()}

    def copy_kib(d, counter):
        v = per_kernel(d, counter)
        k = max(v, key=lambda n: v[n])          # the copy is the largest dispatch
        return v[k]
    f_scale = cal_bytes / (copy_kib(cal_fetch_dir, "FETCH_SIZE") * 1024.0)
    w_scale = cal_bytes / (copy_kib(cal_write_dir, "WRITE_SIZE") * 1024.0)
    fetch, write = per_kernel(fetch_dir, "FETCH_SIZE"), per_kernel(write_dir, "WRITE_SIZE")
    res = {}
    for k in fetch:
        if not k.startswith("k_"):
            continue
        fb, wb = fetch[k] * 1024.0 * f_scale, write.get(k, 0.0) * 1024.0 * w_scale
        res[k[2:]] = {"fetch_kib": fetch[k], "write_kib": write.get(k, 0.0),
                      "fetch_scale": f_scale, "write_scale": w_scale,
                      "bytes_per_launch": fb + wb, "kernel_hash": kernel_source_hash()}
    allres = {}
    if os.path.exists(out):
        with open(out) as fh:
            allres = json.load(fh)
    allres[workload] = res
    with open(out, "w") as fh:
        json.dump(allres, fh, indent=1, sort_keys=True)
    print(json.dumps(allres[workload]), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="paper_share")
    ap.add_argument("--mode", choices=["two_level", "flat"], default="two_level")
    ap.add_argument("--graph", type=int, choices=[0, 1, 2], default=2,
                    help="0 eager launches, 1 16-step HIP graphs, 2 one HIP graph of all "
                         "timed steps (default)")
    ap.add_argument("--per-partition", action="store_true",
                    help="also time the same steps with the update launched once per "
                         "partition (materialised partitions)")
    ap.add_argument("--autotune", action="store_true",
                    help="pick the launch shapes by timing (autotune.tune) before the timed "
                         "region")
    ap.add_argument("--tuning", default="", metavar="U,S,M",
                    help="launch shapes to use (snn_tuning): update_blocks, recv_split, "
                         "recv_merged; overridden by --autotune")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--phase-steps", type=int, default=100)
    ap.add_argument("--tile-neurons", type=int, default=0,
                    help="neurons per tile (snn_params.tile_neurons; 0: the library's default)")
    ap.add_argument("--neurons", type=int, default=0,
                    help="run the workload's structure at this many neurons (quick checks)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES (counter calibration)")
    ap.add_argument("--pmc-summary", nargs=5, metavar=("FETCH_DIR", "WRITE_DIR", "CAL_FETCH_DIR",
                                                       "CAL_WRITE_DIR", "CAL_BYTES"),
                    help="write profiles/traffic.json from rocprofv3 --pmc output directories")
    args = ap.parse_args()
    if args.calibrate_copy:
        calibrate_copy(args.calibrate_copy)
        return
    if args.pmc_summary:
        fd, wd, cfd, cwd, cb = args.pmc_summary
        pmc_summary(fd, wd, cfd, cwd, int(cb), args.workload,
                    os.path.join(ROOT, "profiles", "traffic.json"))
        return

    if args.gpus != 1:
        print(f"bench.py runs one GPU's share on one GPU; --gpus {args.gpus} is not supported "
              "(no exchange between GPUs is implemented)", file=sys.stderr)
        sys.exit(2)

    import numpy as np

    import synth
    wl0 = synth.get_workload(args.workload)
    cpu = None
    if not args.no_cpu_baseline:
        # first, before this process starts OpenMP threads or touches the GPU
        cpu = cpu_baseline(wl0.scaled(args.neurons) if args.neurons else wl0)
        log(f"cpu baseline: {cpu['value']:.3g} events/s on {cpu['cores']} processes")

    import torch
    from paper_2205_07125_amd import SNN_ROUTE_FLAT, SNN_ROUTE_TWO_LEVEL, HostNetwork, Simulation
    from paper_2205_07125_amd.sim import Simulation as _Sim  # noqa: F401

    mode = SNN_ROUTE_TWO_LEVEL if args.mode == "two_level" else SNN_ROUTE_FLAT
    wl = synth.get_workload(args.workload)
    if args.neurons:
        wl = wl.scaled(args.neurons)
    log(f"workload {wl.name}: N={wl.n_neurons:,} K={wl.k_in} P={wl.n_partitions} "
        f"G={wl.gpus_per_node} weights={wl.weight_type}")
    t0 = time.time()
    host = HostNetwork(wl, verbose=True)
    log(f"host setup {time.time() - t0:.1f}s, {host.host_bytes() / 1e9:.1f} GB")
    # steps the log must hold back to the timed region: warm-up, the run that
    # captures the whole-run graph, the timed steps, the per-kernel timing
    # and the per-partition comparison
    reps = 2 if args.graph == 2 else 1
    total_steps = (args.warmup + reps * args.steps + args.phase_steps
                   + (args.warmup + reps * args.steps if args.per_partition else 0))
    t1 = time.time()
    sim = Simulation(wl, host=host, log_steps=total_steps,
                     log_cap=int(wl.n_neurons * max(wl.rate_on_hz, 50.0) * wl.dt_ms * 1e-3 * 4
                                 * total_steps) + (1 << 20), tile_neurons=args.tile_neurons)
    nnz = host.nnz
    sim_tile = sim.tile_neurons
    del host
    sim.host = None
    log(f"device upload {time.time() - t1:.1f}s")

    use_graph = args.graph
    tuned = None
    if args.tuning:
        u, r, m = (int(x) for x in args.tuning.split(","))
        sim.set_tuning(update_blocks=u, recv_split=r, recv_merged=m)
        log(f"tuning: {sim.tuning()}")
    if args.autotune:
        from paper_2205_07125_amd import autotune
        tuned = autotune.tune(sim, mode, log=log)
        log(f"autotune: {tuned['tuning']} ({'cached' if tuned['cached'] else 'timed'})")
    def timed(run):
        """Warm-up, then (for a whole-run graph) one run that captures the
        graph of args.steps steps, then the timed replay of those steps:
        -> (first timed step, HIP-event ms, wall s)."""
        run(args.warmup, 1 if use_graph else 0)
        if use_graph == 2:
            run(args.steps, 2)
        sim.sync()
        torch.cuda.synchronize()
        t_first = sim.t
        s = sim.stream
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        w0 = time.perf_counter()
        e0.record(s)
        run(args.steps, use_graph)
        e1.record(s)
        s.synchronize()
        torch.cuda.synchronize()
        wall_s = time.perf_counter() - w0
        sim.sync()
        return t_first, e0.elapsed_time(e1), wall_s

    t_first, ms, wall = timed(lambda n, g: sim.run(n, mode, g))
    cnt = sim.read_counters(t_first, args.steps).astype(np.float64)
    sec = ms / 1e3
    spikes = cnt[:, 0].sum()
    events = cnt[:, 1].sum() + cnt[:, 2].sum()
    msgs = cnt[:, 3].sum() + cnt[:, 4].sum()
    flat = cnt[:, 5].sum()
    entries = cnt[:, 6].sum() if mode == SNN_ROUTE_TWO_LEVEL else flat
    log(f"timed {args.steps} steps: {ms:.2f} ms (wall {wall * 1e3:.2f} ms), "
        f"{spikes / args.steps:.0f} spikes/step, {events / args.steps:,.0f} events/step")

    # per-kernel durations: eager steps, every kernel bracketed by HIP events
    # on the simulation stream (the stream all kernels are launched on)
    kt = sim.kernel_times(args.phase_steps, mode)
    # connections of the last step (the paper's per-GPU count, Sec. V, Fig. 4):
    # destination partitions reached (what flat exchange opens) against
    # destination nodes reached (what two-level exchange opens), and the
    # largest message count on one of them
    links = None
    if mode == SNN_ROUTE_TWO_LEVEL:
        per_part = sim.route_sizes(1)
        per_node = sim.route_sizes(2)
        links = {"partitions_reached": int((per_part > 0).sum()),
                 "nodes_reached": int((per_node > 0).sum()),
                 "max_entries_per_partition": int(per_part.max()),
                 "max_msgs_per_node": int(per_node.max()),
                 "of": "the last step of the per-kernel timing"}
    pc = sim.read_counters(sim.t - args.phase_steps, args.phase_steps).astype(np.float64)
    log("kernels (ms): " + "  ".join(f"{k} {v:.4f}" for k, v in kt.items() if v > 0))
    N = wl.n_neurons
    bw = 2 if wl.weight_type == "bf16" else 4
    per = pc.mean(axis=0)
    spk, e_loc, e_rem, m2 = per[0], per[1], per[2], per[3] + per[4]
    pairs = per[5] if mode == SNN_ROUTE_FLAT else per[6]   # (source, destination partition)
    # algorithmic HBM bytes per launch, per kernel (what the method must move):
    #   update      18 B per neuron: input slot read + clear 8, u read + write 8,
    #               refractory count read + write 2 (+ the routing's bytes when
    #               the update kernel routes two-level itself)
    #   route       2 B per destination-list entry read, 8 B per message written
    #               (flat: 2 B read + 4 B per entry written)
    #   expand      8 B per message read, 4 B per receive entry written
    #   recv_stage  4 B per receive entry read + 4 B segment index, and (4 + b_w) B
    #               per remote synapse (target/delay + weight)
    #   deliver     (4 + b_w) B per own-partition synapse
    alg = {
        "update": 18.0 * N,
        "route_two_level": 2.0 * pairs + 8.0 * m2,
        "expand": 8.0 * m2 + 4.0 * pairs,
        "route_flat": 6.0 * pairs,
        "recv_stage": 8.0 * pairs + (4 + bw) * e_rem,
        "deliver": (4 + bw) * e_loc,
    }
    # two-level routing done inside the update kernel (no routing launch): its
    # bytes belong to the update launch
    fused = mode == SNN_ROUTE_TWO_LEVEL and kt.get("route_two_level", 0.0) == 0.0
    if fused:
        alg["update"] += alg["route_two_level"]
    # mask expansion, staging and the whole delivery share the receive-side
    # launch of a two-level step: their bytes belong there (the staged
    # events it writes and reads back are the implementation's, not the
    # method's, and are not counted)
    fused_x = mode == SNN_ROUTE_TWO_LEVEL and kt.get("expand", 0.0) == 0.0
    # the receive side as two launches: k_recv_local (expansion, staging, own-
    # partition delivery), then k_deliver_remote, which reads the staged remote
    # synapses back (8 B each, the implementation's queue) and bins them
    split_x = fused_x and kt.get("deliver", 0.0) > 0.0
    if fused_x:
        alg["recv_stage"] += alg["expand"] + alg["deliver"]
        if split_x:
            alg["deliver"] = 8.0 * e_rem
    kernels = {k: {"ms": kt[k], "alg_bytes": alg[k],
                   "gbs": alg[k] / (kt[k] * 1e-3) / 1e9 if kt[k] > 0 else None}
               for k in kt if kt[k] > 0}
    if fused:
        kernels["update"]["includes"] = "two-level routing of the tile's fired neurons"
    if fused_x and split_x:
        kernels["recv_stage"]["includes"] = ("mask expansion of the node's messages and staging; "
                                             "delivery of the own-partition synapses")
        kernels["deliver"]["includes"] = "the staged remote synapses (queue read back)"
    elif fused_x:
        kernels["recv_stage"]["includes"] = ("mask expansion of the node's messages; delivery of "
                                             "the own-partition and the staged remote synapses")
    dom = max(kernels, key=lambda k: kernels[k]["ms"])
    b, t_ms = kernels[dom]["alg_bytes"], kernels[dom]["ms"]
    achieved = b / (t_ms * 1e-3) / 1e9
    traffic = None
    tf = os.path.join(ROOT, "profiles", "traffic.json")
    if os.path.exists(tf):
        with open(tf) as fh:
            tj = json.load(fh).get(wl.name, {})
        h = kernel_source_hash()
        # counters are keyed by kernel symbol; the combined receive-side
        # launch and the remote-only deliver have their own
        symbol = ({"recv_stage": "recv_local", "deliver": "deliver_remote"} if split_x
                  else {"recv_stage": "recv_deliver"} if fused_x else {})
        for k, v in kernels.items():
            ent = tj.get(symbol.get(k, k))
            v["traffic_bytes"] = ent["bytes_per_launch"] if ent and ent.get("kernel_hash") == h else None
        traffic = kernels[dom].get("traffic_bytes")
    # whole step: the sum of the launches' algorithmic bytes defined above
    step_bytes = sum(v["alg_bytes"] for v in kernels.values())
    out = {
        "metric": "synaptic events/s + routed spike msgs/s per GPU; % of HBM peak BW",
        "value": events / sec,
        "unit": "synaptic events/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if wl.weight_type == "fp32" else "bf16 weights, f32 accumulate",
        "data": "synthetic",
        "config": {"workload": wl.name, "n_neurons": N, "in_degree": wl.k_in,
                   "partitions": wl.n_partitions, "gpus_per_node": wl.gpus_per_node,
                   # uneven partitions draw each one's cross fraction from a range
                   "remote_frac": ([wl.cross_lo, wl.cross_hi] if wl.cross_hi > 0
                                   else wl.remote_frac), "rate_hz": wl.rate_on_hz if wl.forced else None,
                   "route": args.mode, "graph": use_graph, "synapses": int(nnz),
                   "tile_neurons": sim_tile},
        "routed_msgs_per_s": (msgs if mode == SNN_ROUTE_TWO_LEVEL else flat) / sec,
        "recv_entries_per_s": entries / sec,
        "spikes_per_step": spikes / args.steps,
        "events_per_step": events / args.steps,
        "msgs_per_step": {"two_level_l1": cnt[:, 3].sum() / args.steps,
                          "two_level_l2": cnt[:, 4].sum() / args.steps,
                          "flat": flat / args.steps},
        "hbm_frac_step": step_bytes / (sec / args.steps) / 1e9 / HBM_PEAK_GBS,
        "kernels": kernels,
        "links": links,
        "roofline": {"kernel": dom, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "algorithmic_bytes_per_launch": b, "avg_launch_ms": t_ms,
                     "timing": "HIP events on the launch stream, %d eager steps" % args.phase_steps},
        "graph": {0: "eager launches", 1: "16-step HIP graphs",
                  2: "one HIP graph of all %d timed steps" % args.steps}[use_graph],
    }
    if args.per_partition:
        # the same steps with the update launched once per partition
        tp, ms_p, _ = timed(lambda n, g: sim.run_partitioned(n, mode, g))
        cp = sim.read_counters(tp, args.steps).astype(np.float64)
        ev_p = cp[:, 1].sum() + cp[:, 2].sum()
        out["layouts"] = {
            "one_launch": {"ms_per_step": ms / args.steps, "events_per_s": events / sec,
                           "update_launches_per_step": 1},
            "per_partition": {"ms_per_step": ms_p / args.steps,
                              "events_per_s": ev_p / (ms_p / 1e3),
                              "update_launches_per_step": int(
                                  (np.diff(synth.partition_starts(wl)) > 0).sum()
                                  if synth.partition_starts(wl) is not None else 1)}}
        log(f"per-partition update launches: {ms_p / args.steps * 1e3:.1f} us/step "
            f"against {ms / args.steps * 1e3:.1f} us/step in one launch")
    if tuned is not None:
        out["tuning"] = {"choice": tuned["tuning"], "cached": tuned["cached"],
                         "candidates": len(tuned.get("timings", []))}
    elif args.tuning:
        out["tuning"] = {"choice": sim.tuning(), "cached": False, "candidates": 0}
    sim.close()
    del sim
    torch.cuda.empty_cache()
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
