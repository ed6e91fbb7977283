"""The allocation-free entry point snn_create_static (workspace in the
library's static device scratch) against snn_create with a caller-provided
workspace: the same network driven through both handles gives the same fired
ids, counters, routing buffers and state, bit for bit.  Two calls in a row,
the second with a smaller network, so the second runs on scratch the first
left behind."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

ROUTE_BOTH = 2


def _steps(sim, n):
    """Both step paths: one kernel per row, and the launches of snn_run."""
    for t in range(n):
        if t % 3 == 2:
            sim.full_step(ROUTE_BOTH)
        else:
            sim.step_route(ROUTE_BOTH)
            sim.deliver()


def _same(a, b, wl, n):
    ia, ca = a.read_spikes(0, n)
    ib, cb = b.read_spikes(0, n)
    assert ca.sum() > 0
    assert np.array_equal(ca, cb) and np.array_equal(ia, ib), "fired ids differ"
    assert np.array_equal(a.read_counters(0, n), b.read_counters(0, n)), "counters differ"
    for which in (0, 1):
        ra, rb = a.read_routes(which), b.read_routes(which)
        for p in range(wl.n_partitions):
            assert np.array_equal(np.sort(ra[p]), np.sort(rb[p])), f"list {which}/{p} differs"
    ba, bb = a.read_routes(2), b.read_routes(2)
    for k in range(wl.n_nodes):
        assert sorted(map(tuple, ba[k].tolist())) == sorted(map(tuple, bb[k].tolist()))
    sa, sb = a.state(), b.state()
    for k in ("u", "ref", "ring"):
        assert np.array_equal(sa[k].view(np.uint8), sb[k].view(np.uint8)), f"{k} differs"


@pytest.mark.parametrize("neurons,steps", [(4096, 120), (2048, 80)])
def test_static_handle_matches_workspace_handle(neurons, steps):
    """Run in this order: the 2,048-neuron case replaces the 4,096-neuron
    handle's state in the device's scratch."""
    from paper_2205_07125_amd import Simulation, _abi
    wl = synth.get_workload("tiny_active")
    if neurons != wl.n_neurons:
        wl = wl.scaled(neurons)
    print(f"[gpu] static handle, {wl.name}: {neurons} neurons, {steps} steps", flush=True)
    ref = Simulation(wl, log_steps=steps)
    sta = Simulation(wl, log_steps=steps, static=True)
    assert sta.ws_bytes <= _abi.SNN_STATIC_SCRATCH_BYTES
    _steps(ref, steps)
    _steps(sta, steps)
    _same(ref, sta, wl, steps)
    # graph replay would instantiate (allocate): refused for a static handle
    with pytest.raises(_abi.SNNError) as ei:
        sta.run(4, ROUTE_BOTH, use_graph=True)
    assert ei.value.status == _abi.SNN_ERR_UNSUPPORTED
    # eager whole steps through snn_run agree as well
    ref.run(16, ROUTE_BOTH, use_graph=False)
    sta.run(16, ROUTE_BOTH, use_graph=False)
    ia, ca = ref.read_spikes(steps, 16)
    ib, cb = sta.read_spikes(steps, 16)
    assert np.array_equal(ca, cb) and np.array_equal(ia, ib)
    sa, sb = ref.state(), sta.state()
    for k in ("u", "ref", "ring"):
        assert np.array_equal(sa[k].view(np.uint8), sb[k].view(np.uint8)), f"{k} differs"
    ref.close()
    sta.close()
