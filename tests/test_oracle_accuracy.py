"""Pins of the oracle's accuracy report (orc_accuracy): the largest
|u32 - u64| before the first step whose rasters differ, that step, the count
of steps whose rasters agree, the smallest threshold margin of the FP64
trajectory and its largest |u| (before resets).  CPU only.

The reference is an independent re-implementation of the two trajectories
with numpy: float32 arithmetic (IEEE binary32, one rounding per operation)
and float64, on a hand-made network whose divergence step is constructed:
neuron B decays from a chosen u0 for m steps, then one synapse from neuron
A adds w = 15 - fl32(u32 * alpha) exactly, so the binary32 trajectory lands
on the threshold 15.0 (and fires) while the FP64 trajectory, which decayed
without rounding to a slightly smaller value, stays below it."""
import numpy as np

from oracle_util import make_sim

ALPHA32 = np.float32(0.995012462139129638671875)
THETA = np.float32(15.0)
N_REF = 20
D = 11


def _reference(n, edges, u0, n_steps):
    """Both trajectories of a network without drive, step by step as the
    neuron model is stated (input of slot t mod D, then u = u alpha + I,
    refractory clamp, threshold u >= theta, reset to 0)."""
    u32 = u0.astype(np.float32).copy()
    u64 = u0.astype(np.float64).copy()
    ref32 = np.zeros(n, np.int64)
    ref64 = np.zeros(n, np.int64)
    ring32 = np.zeros((D, n), np.float32)
    ring64 = np.zeros((D, n), np.float64)
    max_dv, first_div, agree, margin, max_u = 0.0, -1, 0, np.inf, 0.0
    for t in range(n_steps):
        s = t % D
        syn32, syn64 = ring32[s].copy(), ring64[s].copy()
        ring32[s] = 0
        ring64[s] = 0
        i32 = ref32 == 0
        ref32[~i32] -= 1
        u32[i32] = (u32[i32] * ALPHA32).astype(np.float32) + syn32[i32]   # float32 add
        f32 = np.flatnonzero(i32 & (u32 >= THETA))
        u32[f32] = 0
        ref32[f32] = N_REF
        i64 = ref64 == 0
        ref64[~i64] -= 1
        u64[i64] = u64[i64] * float(ALPHA32) + syn64[i64]
        if i64.any():
            margin = min(margin, float(np.min(np.abs(u64[i64] - 15.0))))
            max_u = max(max_u, float(np.max(np.abs(u64[i64]))))
        f64 = np.flatnonzero(i64 & (u64 >= 15.0))
        u64[f64] = 0
        ref64[f64] = N_REF
        same = np.array_equal(f32, f64)
        agree += same
        if first_div < 0:
            if same:
                max_dv = max(max_dv, float(np.max(np.abs(u32.astype(np.float64) - u64))))
            else:
                first_div = t
        for (a, b, d, w) in edges:
            if a in f32:
                ring32[(t + d) % D, b] = np.float32(ring32[(t + d) % D, b] + np.float32(w))
            if a in f64:
                ring64[(t + d) % D, b] += float(np.float32(w))
    return dict(max_dv=max_dv, first_divergence=first_div, agree_steps=agree,
                min_margin=margin, max_abs_u=max_u)


def _constructed_case(m=7):
    """Neuron 0 (A) fires at step 0; neuron 1 (B) decays from u0 and receives
    at step m (delay m) the weight that puts its binary32 membrane exactly on
    15.0; neurons 2.. decay from non-dyadic values (they contribute |u32 - u64|
    before the divergence) and one gets 0.1 mV at step 3."""
    rng = np.random.default_rng(5)
    for _ in range(200):
        b0 = np.float32(rng.uniform(9.0, 13.0))
        a32, a64 = b0, float(b0)
        for _ in range(m + 1):       # steps 0 .. m - 1 decay, then step m's product
            a32 = np.float32(a32 * ALPHA32)
            a64 = a64 * float(ALPHA32)
        w = np.float32(THETA - a32)   # exact (Sterbenz): a32 in [7.5, 30]
        if np.float32(a32 + w) == THETA and a64 + float(w) < 15.0:
            break
    else:
        raise AssertionError("no u0 found whose FP64 trajectory stays below threshold")
    u0 = np.concatenate([[np.float32(20.0), b0],
                         rng.uniform(0.5, 14.0, 30).astype(np.float32)]).astype(np.float32)
    edges = [(0, 1, m, 0, float(w)), (0, 5, 3, 0, 0.1)]
    return u0, edges


def test_accuracy_report_matches_reference():
    m = 7
    u0, edges = _constructed_case(m)
    n, steps = len(u0), 40
    sim = make_sim(n, edges=[(a, b, d, vp, w) for (a, b, d, vp, w) in edges], u0=u0)
    sim.run(steps)
    got = sim.accuracy()
    want = _reference(n, [(a, b, d, w) for (a, b, d, _, w) in edges], u0, steps)
    assert want["first_divergence"] == m          # the constructed divergence
    assert want["agree_steps"] == steps - 1       # B is refractory in one trajectory only
    assert 0.0 < want["max_dv"] < 1e-5
    assert 0.0 < want["min_margin"] < 1e-5        # B's FP64 membrane just below 15
    assert got["first_divergence"] == want["first_divergence"]
    assert got["agree_steps"] == want["agree_steps"]
    assert got["max_dv"] == want["max_dv"]
    assert got["min_margin"] == want["min_margin"]
    assert got["max_abs_u"] == want["max_abs_u"] == 20.0 * float(ALPHA32)


def test_accuracy_without_divergence():
    """The same network without B's synapse: no divergence (-1), every step
    agrees, and max |u32 - u64| is taken over the whole run."""
    u0, edges = _constructed_case()
    edges = [e for e in edges if e[1] != 1]
    n, steps = len(u0), 60
    sim = make_sim(n, edges=edges, u0=u0)
    sim.run(steps)
    got = sim.accuracy()
    want = _reference(n, [(a, b, d, w) for (a, b, d, _, w) in edges], u0, steps)
    assert want["first_divergence"] == -1 and want["agree_steps"] == steps
    for k in ("max_dv", "first_divergence", "agree_steps", "min_margin", "max_abs_u"):
        assert got[k] == want[k], k
