"""Parity at full size, in the launch configuration the benchmark times
(two-level routing, HIP-graph replay): the 5e6-neuron / in-degree-1,000 share
in FP32 and with BF16 weights, the heavy-traffic shape (1e6 neurons,
in-degree 10,000, 200 destination partitions per source) over steps of its
first burst, and the 64 uneven partitions of the batched shape (5.8e6
neurons, all partitions materialised).

The oracle cannot hold 5e9 synapses, so it checks what it can compute one by
one at any size: with the forced raster a spike is a pure function of (seed,
neuron, step), so the oracle recomputes the complete raster of every step,
and the exact trajectory (u, refractory count, pending ring input) of sampled
neurons from the generator's incoming synapses of those neurons alone.  The
routing buffers of the last step are checked through properties that hold at
any size: expanded lists equal flat lists as multisets, one message per
distinct destination node, masks valid, events equal out-degree sums."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

ROUTE_TWO_LEVEL, ROUTE_BOTH = 0, 2


# workload -> steps run (all of heavy's are burst steps: 1e4 spikes and 1e8
# events each)
FULL = {"paper_share": 40, "paper_share_bf16": 40, "heavy": 12, "batched": 40}


@pytest.mark.timeout(1500)
@pytest.mark.parametrize("name", list(FULL))
def test_full_size_sampled(name):
    from paper_2205_07125_amd import HostNetwork, Simulation
    wl = synth.get_workload(name)
    T = FULL[name]
    assert wl.forced
    print(f"[gpu] full size {wl.name}: building N={wl.n_neurons:,} K={wl.k_in}", flush=True)
    host = HostNetwork(wl, verbose=True)
    row_ptr = host.row_ptr.copy()
    vp_ptr, vp_part = host.vp_ptr.copy(), host.vp_part.copy()
    part = host.part.copy()
    sim = Simulation(wl, host=host, log_steps=T)
    sim.host = None
    del host
    sim.run(T - 1, ROUTE_TWO_LEVEL, use_graph=True)
    sim.full_step(ROUTE_BOTH)
    sim.sync()
    print("[gpu] device steps done", flush=True)
    params = oracle.params_from_workload(wl)

    # 1. the complete raster of every step
    ids, counts = sim.read_spikes(0, T)
    offs = np.concatenate([[0], np.cumsum(counts.astype(np.int64))])
    for t in range(T):
        want = oracle.forced_raster(params, t)
        assert np.array_equal(ids[offs[t]:offs[t + 1]], want.astype(np.int32)), f"raster step {t}"
    print(f"[gpu] raster of {T} steps matches ({len(ids):,} spikes)", flush=True)

    # 2. counters: spikes, and events = sum of out-degrees of the fired sources
    cnt = sim.read_counters(0, T).astype(np.int64)
    assert np.array_equal(cnt[:, 0], counts.astype(np.int64))
    outdeg = np.diff(row_ptr)
    for t in range(T):
        f = ids[offs[t]:offs[t + 1]]
        assert cnt[t, 1] + cnt[t, 2] == outdeg[f].sum()

    # 3. sampled neurons: exact trajectory from their own incoming synapses
    st = sim.state()
    u0 = synth.initial_u(wl)
    gen = synth.Generator(wl)
    D = wl.max_delay + 1
    rng = np.random.default_rng(0)
    sample = np.unique(np.concatenate([[0, 1, wl.n_neurons - 1],
                                       rng.integers(0, wl.n_neurons, 300)]))
    spiking = 0
    for j in sample:
        e = gen.edges(int(j), int(j) + 1)
        u, ref, ns, pend = oracle.forced_neuron(params, int(j), u0[j], e["src"], e["delay"],
                                                e["w"], T)
        spiking += ns > 0
        assert u == st["u"][j], f"u of neuron {j}"
        assert ref == st["ref"][j], f"ref of neuron {j}"
        for d in range(1, wl.max_delay + 1):
            assert pend[d - 1] == st["ring"][(T - 1 + d) % D][j], f"ring of neuron {j}, +{d}"
    print(f"[gpu] {len(sample)} sampled neurons exact ({spiking} of them fired)", flush=True)

    # 4. routes of the last step (properties that hold at any size)
    flat = sim.read_routes(0, sources_only=True)
    xrecv = sim.read_routes(1, sources_only=True)
    buckets = sim.read_routes(2)
    for p in range(wl.n_partitions):
        assert np.array_equal(np.sort(flat[p]), np.sort(xrecv[p])), f"partition {p}"
    fired = ids[offs[T - 1]:offs[T]]
    G = wl.gpus_per_node
    want_msgs = 0
    want_entries = 0
    for s in fired:
        v = vp_part[vp_ptr[s]:vp_ptr[s + 1]].astype(np.int64)
        want_msgs += len(np.unique(v // G))
        want_entries += len(v)
    assert sum(len(b) for b in buckets) == want_msgs == cnt[T - 1, 3] + cnt[T - 1, 4]
    assert sum(len(x) for x in xrecv) == want_entries == cnt[T - 1, 6] == cnt[T - 1, 5]
    for n, b in enumerate(buckets):
        src = (b[:, 0] & np.uint64(0xFFFFFFFF)).astype(np.int64)
        mask = b[:, 1]
        gn = min(G, wl.n_partitions - G * n)             # partitions of node n
        assert np.all(mask > 0)
        if gn < 64:
            assert np.all(mask < np.uint64(1 << gn))
        own = part[src] // G == n                        # level 1: the source's own node
        own_bit = np.left_shift(np.uint64(1), (part[src] - G * n).clip(0).astype(np.uint64))
        assert not np.any(own & ((mask & own_bit) != 0)), "own partition in a mask"
        assert len(np.unique(src)) == len(src)          # one message per source and node
    print(f"[gpu] {name}: routing invariants hold at full size", flush=True)
