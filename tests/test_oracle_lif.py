"""Pins of the oracle's neuron update against closed forms and numpy float32
arithmetic (an independent IEEE binary32 implementation).  CPU only."""
import math

import numpy as np

import oracle
from oracle_util import make_sim

ALPHA32 = np.float32(0.995012462139129638671875)  # fl32(exp(-dt / tau_m))


def test_free_decay():
    """No drive, no synapses: u_t = u_0 alpha^t (FP64) and the binary32
    trajectory equals repeated float32 multiplication."""
    u0 = np.array([14.9, 7.25, 0.001, 3.0, 0.0, 12.5], np.float32)
    sim = make_sim(len(u0), u0=u0)
    u32 = u0.copy()
    for t in range(1, 301):
        assert sim.step() == 0
        u32 = (u32 * ALPHA32).astype(np.float32)
        u32 = (u32 + np.float32(0.0)).astype(np.float32)
        st = sim.state()
        assert np.array_equal(st["u"].view(np.uint32), u32.view(np.uint32)), t
        exact = u0.astype(np.float64) * float(ALPHA32) ** t
        assert np.allclose(st["u64"], exact, rtol=1e-12, atol=1e-300)


def _constant_drive_spike_times(I, alpha, theta, n_ref, n_steps):
    """Spike steps of u <- alpha u + I with reset to 0 and n_ref clamped
    steps, from the closed form u_c = I (1 - alpha^c) / (1 - alpha)."""
    c = math.ceil(math.log(1.0 - theta * (1.0 - alpha) / I) / math.log(alpha))
    # guard against the closed form landing within rounding of the threshold
    assert abs(I * (1 - alpha ** c) / (1 - alpha) - theta) > 1e-9
    times, t = [], c - 1
    while t < n_steps:
        times.append(t)
        t += n_ref + c
    return times


def test_constant_drive_first_crossing_and_refractory():
    """Huge Poisson rate empties the inversion table, so k = 15 on every step:
    a constant input I = fl32(15 w_ext).  Spike times follow the closed form,
    inter-spike interval = crossing time + 20 refractory steps."""
    w_ext = 0.1
    n_steps = 1500
    sim = make_sim(3, nu_ext_hz=1e7, w_ext_mv=w_ext)   # lambda = 1000
    I32 = np.float32(np.float32(15) * np.float32(w_ext))
    times64 = _constant_drive_spike_times(float(I32), float(ALPHA32), 15.0, 20, n_steps)
    # numpy float32 iteration of the same update (one rounding per operation)
    u, ref, times32, traj32 = np.float32(0), 0, [], []
    for t in range(n_steps):
        if ref > 0:
            ref -= 1
        else:
            u = np.float32(np.float32(u * ALPHA32) + np.float32(np.float32(0) + I32))
            if u >= np.float32(15):
                times32.append(t)
                u, ref = np.float32(0), 20
        traj32.append(u)
    got32, got64 = [], []
    for t in range(n_steps):
        n = sim.step()
        assert sim.state()["u"][0] == traj32[t], t
        f, f64 = sim.fired(), sim.fired64()
        if n:
            assert list(f) == [0, 1, 2]
            got32.append(t)
        if len(f64):
            got64.append(t)
    assert got64 == times64
    assert got32 == times32
    assert len(times64) >= 5
    # refractory: during the n_ref steps after a spike u stays at reset
    sim2 = make_sim(1, nu_ext_hz=1e7, w_ext_mv=w_ext)
    first = times64[0]
    for t in range(first + 1):
        sim2.step()
    for k in range(20):
        st = sim2.state()
        assert st["u"][0] == 0.0 and st["ref"][0] == 20 - k
        sim2.step()
    st = sim2.state()
    assert st["ref"][0] == 0 and st["u"][0] == 0.0   # 20th clamped step done
    sim2.step()
    assert sim2.state()["u"][0] == I32               # integrates again


def test_delay_arrival_and_refractory_discard():
    """Neuron 0 starts above threshold and fires at step 0; its synapse to
    neuron 1 (delay d) arrives exactly at step d.  A second synapse to neuron 0
    itself is not allowed (no autapses), so use neuron 2 which is refractory
    when the input arrives: its input is discarded."""
    d = 7
    edges = [(0, 1, d, 0, 0.5), (0, 2, 3, 0, 0.5)]
    u0 = np.array([20.0, 0.0, 16.0], np.float32)     # 0 and 2 fire at step 0
    sim = make_sim(3, edges=edges, u0=u0)
    u1 = np.float32(0.0)
    for t in range(40):
        sim.step()
        st = sim.state()
        if t == 0:
            assert list(sim.fired()) == [0, 2]
        # neuron 1: nothing before step d, exactly 0.5 at step d, then pure
        # decay (the consumed ring slot was cleared, so nothing arrives again
        # when the ring wraps around after 11 steps)
        u1 = np.float32(u1 * ALPHA32)
        if t == d:
            u1 = np.float32(u1 + np.float32(0.5))
        assert st["u"][1] == u1, t
        # neuron 2 is refractory for steps 1..20: the arrival at step 3 is lost
        assert st["u"][2] == 0.0


def test_threshold_is_inclusive():
    """A neuron whose membrane lands exactly on the threshold fires (the
    threshold test is u >= theta): 30 simultaneous 0.5 mV inputs from rest
    give exactly 15.0 mV."""
    edges = [(s, 30, 2, 0, 0.5) for s in range(30)]
    u0 = np.zeros(31, np.float32)
    u0[:30] = 20.0
    sim = make_sim(31, edges=edges, u0=u0)
    sim.step()
    sim.step()
    assert sim.step() == 1 and list(sim.fired()) == [30]
    assert list(sim.fired64()) == [30]


def test_compaction_is_flatnonzero():
    """One step from a random state without drive or synapses: the fired list
    is numpy's flatnonzero of the float32 threshold test, ascending."""
    rng = np.random.default_rng(2)
    u0 = rng.uniform(10, 20, 4099).astype(np.float32)
    sim = make_sim(len(u0), u0=u0)
    sim.step()
    u1 = (u0 * ALPHA32).astype(np.float32)
    want = np.flatnonzero(u1 >= np.float32(15.0))
    assert np.array_equal(sim.fired(), want.astype(np.uint32))
    st = sim.state()
    assert np.all(st["u"][want] == 0.0) and np.all(st["ref"][want] == 20)
    rest = np.setdiff1d(np.arange(len(u0)), want)
    assert np.all(st["u"][rest] < 15.0)


def test_fp64_trajectory_accuracy_tiny():
    """On the tiny net the binary32 and FP64 trajectories stay within 1e-4 mV
    before any raster divergence."""
    import synth
    wl = synth.get_workload("tiny_active")
    sim = oracle.sim_for_workload(wl)
    sim.run(300)
    acc = sim.accuracy()
    assert acc["max_dv"] < 1e-4


def test_forced_raster_rate():
    """Forced raster: spikes are Bernoulli(rate dt) draws, independent of the
    membrane; the on/off schedule follows the period."""
    n, steps = 2000, 60
    sim = make_sim(n, forced=1, rate_on_hz=500.0, rate_off_hz=0.0, period_steps=20,
                   on_steps=10)
    counts = []
    for t in range(steps):
        counts.append(sim.step())
    counts = np.array(counts)
    off = np.array([(t % 20) >= 10 for t in range(steps)])
    assert np.all(counts[off] == 0)
    p = 500.0 * 1e-4
    mean = counts[~off].mean()
    assert abs(mean - n * p) < 4 * math.sqrt(n * p * (1 - p) / (~off).sum())
