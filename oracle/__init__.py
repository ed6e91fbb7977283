"""Plain CPU reference of the simulation step (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path never does.  The
native part is ``liboracle.so`` built from ``oracle.c`` by ``oracle/build.py``;
``oracle.c`` states what each step computes and which passage it follows.

Parity pins (each checked in ``tests/test_oracle_*.py`` against something
other than the oracle itself):
  * Philox-4x32-10: AMD's rocRAND host engine on random counters and keys.
  * Poisson table: scipy's Poisson CDF; sample mean and P(k=0) statistically.
  * BF16 rounding: torch's float32 -> bfloat16 conversion.
  * Neuron update: closed forms (free decay, constant drive, first crossing,
    refractory length) and numpy float32 arithmetic.
  * Compaction: numpy flatnonzero on the threshold test.
  * Routing: invariants (messages = distinct destination nodes from numpy
    unique, expanded lists = flat lists as multisets, entries = mask
    popcounts, own-partition bit never set) and the fan-in example of
    Sec. IV-B (Fig. 2) stored under tests/golden/.
  * Delivery: dense FP64 product W_d^T 1_F with numpy.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("SNN_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")

SPIKES, LOCAL_EVENTS, REMOTE_EVENTS, MSG_L1, MSG_L2, FLAT_MSGS, RECV_ENTRIES = range(7)
NSTAT = 7
STAT_NAMES = ["spikes", "local_events", "remote_events", "msg_l1", "msg_l2", "flat_msgs",
              "recv_entries"]


class Params(ctypes.Structure):
    _fields_ = [
        ("n_neurons", ctypes.c_uint32),
        ("n_partitions", ctypes.c_uint32),
        ("gpus_per_node", ctypes.c_uint32),
        ("max_delay", ctypes.c_uint32),
        ("dt_ms", ctypes.c_double),
        ("tau_m_ms", ctypes.c_double),
        ("theta_mv", ctypes.c_double),
        ("u_reset_mv", ctypes.c_double),
        ("t_ref_ms", ctypes.c_double),
        ("nu_ext_hz", ctypes.c_double),
        ("w_ext_mv", ctypes.c_double),
        ("seed", ctypes.c_uint64),
        ("forced", ctypes.c_uint32),
        ("period_steps", ctypes.c_uint32),
        ("on_steps", ctypes.c_uint32),
        ("rate_on_hz", ctypes.c_double),
        ("rate_off_hz", ctypes.c_double),
        ("bf16_weights", ctypes.c_uint32),
    ]


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run oracle/build.py")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        L.orc_create.restype = P
        L.orc_create.argtypes = [ctypes.POINTER(Params), ctypes.c_uint64, P, P, P, P, P, P, P]
        L.orc_destroy.argtypes = [P]
        L.orc_step.restype = ctypes.c_uint32
        L.orc_step.argtypes = [P]
        L.orc_run.argtypes = [P, ctypes.c_uint32, P, P]
        L.orc_time.restype = ctypes.c_uint64
        L.orc_time.argtypes = [P]
        L.orc_fired.restype = ctypes.c_uint32
        L.orc_fired.argtypes = [P, P]
        L.orc_fired64.restype = ctypes.c_uint32
        L.orc_fired64.argtypes = [P, P]
        L.orc_counters.argtypes = [P, P]
        L.orc_recv.restype = ctypes.c_uint64
        L.orc_recv.argtypes = [P, ctypes.c_int, P, P]
        L.orc_buckets.restype = ctypes.c_uint64
        L.orc_buckets.argtypes = [P, P, P]
        L.orc_state.argtypes = [P] * 7
        L.orc_accuracy.argtypes = [P, P]
        L.orc_alpha.restype = ctypes.c_float
        L.orc_alpha.argtypes = [ctypes.POINTER(Params)]
        L.orc_poisson_table.argtypes = [ctypes.c_double, P]
        L.orc_poisson_k.restype = ctypes.c_uint32
        L.orc_poisson_k.argtypes = [P, ctypes.c_uint32]
        L.orc_n_ref.restype = ctypes.c_uint32
        L.orc_n_ref.argtypes = [ctypes.POINTER(Params)]
        L.orc_raster_threshold.restype = ctypes.c_uint32
        L.orc_raster_threshold.argtypes = [ctypes.c_double, ctypes.c_double]
        L.orc_philox4x32_10.argtypes = [P, P, P]
        L.orc_forced_raster.restype = ctypes.c_uint32
        L.orc_forced_raster.argtypes = [ctypes.POINTER(Params), ctypes.c_uint64, ctypes.c_uint32,
                                        ctypes.c_uint32, P]
        L.orc_forced_neuron.restype = ctypes.c_int
        L.orc_forced_neuron.argtypes = [ctypes.POINTER(Params), ctypes.c_uint32, ctypes.c_float,
                                        ctypes.c_uint32, P, P, P, ctypes.c_uint32, P, P, P, P]
        L.orc_bf16_round.restype = ctypes.c_float
        L.orc_bf16_round.argtypes = [ctypes.c_float]
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def params_from_workload(wl, **over) -> Params:
    kw = dict(n_neurons=wl.n_neurons, n_partitions=wl.n_partitions,
              gpus_per_node=wl.gpus_per_node, max_delay=wl.max_delay, dt_ms=wl.dt_ms,
              tau_m_ms=wl.tau_m_ms, theta_mv=wl.theta_rel_mv, u_reset_mv=wl.u_reset_mv,
              t_ref_ms=wl.t_ref_ms, nu_ext_hz=wl.nu_ext_hz, w_ext_mv=wl.w_ext_mv, seed=wl.seed,
              forced=wl.forced, period_steps=max(wl.period_steps, 1), on_steps=wl.on_steps,
              rate_on_hz=wl.rate_on_hz, rate_off_hz=wl.rate_off_hz,
              bf16_weights=1 if wl.weight_type == "bf16" else 0)
    kw.update(over)
    return Params(**kw)


def philox4x32_10(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, np.uint32)
    lib().orc_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def poisson_table(lam: float) -> np.ndarray:
    out = np.zeros(15, np.uint32)
    lib().orc_poisson_table(lam, _p(out))
    return out


def poisson_k(thr: np.ndarray, r: int) -> int:
    t = np.ascontiguousarray(thr, dtype=np.uint32)
    return int(lib().orc_poisson_k(_p(t), r))


def bf16_round(x: float) -> float:
    return float(lib().orc_bf16_round(float(x)))


def forced_raster(params: Params, t: int, lo: int = 0, hi: int | None = None) -> np.ndarray:
    """Fired ids of step t under a forced raster, computed from the random
    draws alone (any network size)."""
    hi = params.n_neurons if hi is None else hi
    out = np.zeros(max(hi - lo, 1), np.uint32)
    n = lib().orc_forced_raster(ctypes.byref(params), t, lo, hi, _p(out))
    return out[:n].copy()


def forced_neuron(params: Params, j: int, u0: float, in_src, in_delay, in_w, n_steps: int):
    """Neuron j alone under a forced raster from its incoming synapses:
    -> (u, ref, spike count, pending input of the next max_delay steps)."""
    src = np.ascontiguousarray(in_src, np.uint32)
    dly = np.ascontiguousarray(in_delay, np.uint8)
    w = np.ascontiguousarray(in_w, np.float32)
    u = ctypes.c_float()
    ref = ctypes.c_uint8()
    ns = ctypes.c_uint32()
    pend = np.zeros(params.max_delay, np.float32)
    rc = lib().orc_forced_neuron(ctypes.byref(params), j, float(u0), len(src), _p(src), _p(dly),
                                 _p(w), n_steps, ctypes.byref(u), ctypes.byref(ref), _p(pend),
                                 ctypes.byref(ns))
    if rc != 0:
        raise ValueError("forced_neuron needs a forced-raster parameter set")
    return np.float32(u.value), int(ref.value), int(ns.value), pend


def alpha(params: Params) -> np.float32:
    return np.float32(lib().orc_alpha(ctypes.byref(params)))


def n_ref(params: Params) -> int:
    return int(lib().orc_n_ref(ctypes.byref(params)))


def raster_threshold(rate_hz: float, dt_ms: float) -> int:
    return int(lib().orc_raster_threshold(rate_hz, dt_ms))


class Sim:
    """Stepwise reference simulation over an explicit synapse list."""

    def __init__(self, params: Params, edges: dict, part: np.ndarray, u0: np.ndarray):
        self.params = params
        self.N = params.n_neurons
        self.P = params.n_partitions
        self.G = params.gpus_per_node
        self.n_nodes = (self.P + self.G - 1) // self.G
        self.D = params.max_delay + 1
        e = {k: np.ascontiguousarray(v) for k, v in edges.items()}
        assert e["src"].dtype == np.uint32 and e["tgt"].dtype == np.uint32
        assert e["delay"].dtype == np.uint8 and e["vp"].dtype == np.uint16
        assert e["w"].dtype == np.float32
        part = np.ascontiguousarray(part, dtype=np.int32)
        u0 = np.ascontiguousarray(u0, dtype=np.float32)
        m = len(e["src"])
        h = lib().orc_create(ctypes.byref(params), m, _p(e["src"]), _p(e["tgt"]), _p(e["delay"]),
                             _p(e["vp"]), _p(e["w"]), _p(part), _p(u0))
        if not h:
            raise ValueError("oracle rejected the network")
        self.h = ctypes.c_void_p(h)

    def close(self):
        if self.h:
            lib().orc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def t(self) -> int:
        return int(lib().orc_time(self.h))

    def step(self) -> int:
        return int(lib().orc_step(self.h))

    def run(self, n: int):
        counts = np.zeros(n, np.uint32)
        stats = np.zeros((n, NSTAT), np.uint64)
        lib().orc_run(self.h, n, _p(counts), _p(stats))
        return counts, stats

    def fired(self) -> np.ndarray:
        out = np.zeros(self.N, np.uint32)
        n = lib().orc_fired(self.h, _p(out))
        return out[:n].copy()

    def fired64(self) -> np.ndarray:
        out = np.zeros(self.N, np.uint32)
        n = lib().orc_fired64(self.h, _p(out))
        return out[:n].copy()

    def counters(self) -> np.ndarray:
        out = np.zeros(NSTAT, np.uint64)
        lib().orc_counters(self.h, _p(out))
        return out

    def recv(self, which: int):
        """which 0: flat lists, 1: expanded two-level lists -> list of arrays."""
        sizes = np.zeros(self.P, np.uint64)
        total = lib().orc_recv(self.h, which, _p(sizes), None)
        ent = np.zeros(max(int(total), 1), np.uint32)
        lib().orc_recv(self.h, which, _p(sizes), _p(ent))
        offs = np.concatenate([[0], np.cumsum(sizes.astype(np.int64))])
        return [ent[offs[p]:offs[p + 1]].copy() for p in range(self.P)]

    def buckets(self):
        """Per node, the messages of the last step as an (n, 2) uint64 array of
        (source id, mask of the node's destination partitions)."""
        sizes = np.zeros(self.n_nodes, np.uint64)
        total = lib().orc_buckets(self.h, _p(sizes), None)
        msgs = np.zeros((max(int(total), 1), 2), np.uint64)
        lib().orc_buckets(self.h, _p(sizes), _p(msgs))
        offs = np.concatenate([[0], np.cumsum(sizes.astype(np.int64))])
        return [msgs[offs[n]:offs[n + 1]].copy() for n in range(self.n_nodes)]

    def state(self) -> dict:
        N, D = self.N, self.D
        out = dict(u=np.zeros(N, np.float32), ref=np.zeros(N, np.uint8),
                   ring=np.zeros((D, N), np.float32), u64=np.zeros(N, np.float64),
                   ref64=np.zeros(N, np.uint8), ring64=np.zeros((D, N), np.float64))
        lib().orc_state(self.h, _p(out["u"]), _p(out["ref"]), _p(out["ring"]), _p(out["u64"]),
                        _p(out["ref64"]), _p(out["ring64"]))
        return out

    def membrane64(self) -> np.ndarray:
        """u of the FP64 trajectory (copy)."""
        out = np.zeros(self.N, np.float64)
        lib().orc_state(self.h, None, None, None, _p(out), None, None)
        return out

    def accuracy(self) -> dict:
        out = np.zeros(5, np.float64)
        lib().orc_accuracy(self.h, _p(out))
        return dict(max_dv=out[0], first_divergence=int(out[1]), agree_steps=int(out[2]),
                    min_margin=out[3], max_abs_u=out[4])


def sim_for_workload(wl, part_map=None, **over) -> "Sim":
    """Build the reference simulation of a (small) workload from the seeded
    generator (with an explicit neuron -> partition map if given)."""
    import synth
    gen = synth.Generator(wl, part_map=part_map)
    edges = gen.edges()
    part = gen.part_map()
    u0 = synth.initial_u(wl)
    return Sim(params_from_workload(wl, **over), edges, part, u0)
