"""The oracle's any-size forced-raster functions (raster of a step from the
random draws alone; one neuron's trajectory from its incoming synapses)
agree with the oracle's whole-network simulation.  CPU only."""
import numpy as np
import pytest

import oracle
import synth


@pytest.mark.parametrize("bf16", [False, True])
def test_forced_neuron_matches_network_sim(bf16):
    wl = synth.get_workload("paper_share").scaled(3000, k_in=80, rate_on_hz=400.0,
                                                  rate_off_hz=400.0)
    if bf16:
        wl = wl.replace(weight_type="bf16")
    gen = synth.Generator(wl)
    e = gen.edges()
    u0 = synth.initial_u(wl)
    params = oracle.params_from_workload(wl)
    sim = oracle.Sim(params, e, gen.part_map(), u0)
    T = 57
    for t in range(T):
        sim.step()
        want = oracle.forced_raster(params, t)
        assert np.array_equal(sim.fired(), want)
    st = sim.state()
    D = wl.max_delay + 1
    K = wl.k_in
    for j in list(range(0, wl.n_neurons, 97)) + [wl.n_neurons - 1]:
        sl = slice(j * K, (j + 1) * K)      # canonical list: target-major
        assert np.all(e["tgt"][sl] == j)
        u, ref, ns, pend = oracle.forced_neuron(params, j, u0[j], e["src"][sl], e["delay"][sl],
                                                e["w"][sl], T)
        assert u == st["u"][j] and ref == st["ref"][j]
        for d in range(1, wl.max_delay + 1):
            assert pend[d - 1] == st["ring"][(T - 1 + d) % D][j], (j, d)


def test_forced_raster_partial_range_and_schedule():
    wl = synth.get_workload("heavy").scaled(5000, k_in=10, period_steps=20, on_steps=5)
    params = oracle.params_from_workload(wl)
    full = oracle.forced_raster(params, 3)
    part = np.concatenate([oracle.forced_raster(params, 3, 0, 1234),
                           oracle.forced_raster(params, 3, 1234, 5000)])
    assert np.array_equal(full, part) and len(full) > 0
    assert len(oracle.forced_raster(params, 7)) == 0      # off phase, rate 0


def test_burst_schedule_and_rate_from_the_workload_definition():
    """The heavy workload's bursts (rate_on for the first on_steps of every
    period_steps, silence otherwise), pinned by what that definition implies
    rather than by the oracle's formula: a step has spikes exactly when
    t mod period < on_steps, in the network simulation and in the any-size
    raster alike, and the spikes of the on steps are Binomial(N * steps, p)
    with p = rate_on * dt, within 4 sigma."""
    wl = synth.get_workload("heavy").scaled(6000, k_in=10, period_steps=20, on_steps=5)
    assert wl.rate_off_hz == 0.0
    N, T = wl.n_neurons, 60
    p = wl.rate_on_hz * wl.dt_ms * 1e-3
    gen = synth.Generator(wl)
    params = oracle.params_from_workload(wl)
    sim = oracle.Sim(params, gen.edges(), gen.part_map(), synth.initial_u(wl))
    counts = []
    for t in range(T):
        sim.step()
        counts.append(len(sim.fired()))
        assert len(oracle.forced_raster(params, t)) == counts[-1]
    on = [t for t in range(T) if t % 20 < 5]
    # an on step without spikes has probability (1 - p)^N, about e^-60
    assert [t for t in range(T) if counts[t] > 0] == on
    n = N * len(on)
    total = sum(counts[t] for t in on)
    assert abs(total - n * p) < 4 * np.sqrt(n * p * (1 - p)), (total, n * p)
