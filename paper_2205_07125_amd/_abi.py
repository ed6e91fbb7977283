"""ctypes mirror of include/snn.h and include/snn_setup.h (argument
marshalling only; every step of the simulation runs in libsnn's kernels)."""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("SNN_LIB") or os.path.join(_PKG, "libsnn.so")

SNN_OK = 0
SNN_ERR_INVALID_ARG = -1
SNN_ERR_BAD_STATE = -2
SNN_ERR_CAPACITY = -3
SNN_ERR_HIP = -4
SNN_ERR_UNSUPPORTED = -5

SNN_STATIC_SCRATCH_BYTES = 32 << 20   # snn_create_static's device scratch

SNN_ROUTE_TWO_LEVEL = 0
SNN_ROUTE_FLAT = 1
SNN_ROUTE_BOTH = 2

SNN_W_FP32 = 0
SNN_W_BF16 = 1
SNN_FORCED_RASTER = 1

# receive-list entries: source id in the low ENTRY_SRC_BITS bits, pair index above
ENTRY_SRC_BITS = 27

STAT_NAMES = ["spikes", "local_events", "remote_events", "msg_l1", "msg_l2", "flat_msgs",
              "recv_entries"]
SNN_NSTAT = len(STAT_NAMES)
KERNEL_NAMES = ["update", "route_two_level", "expand", "route_flat", "recv_stage", "deliver"]
SNN_NKERNEL = len(KERNEL_NAMES)

EXPORTED = [
    "snn_ring_stride", "snn_workspace_size", "snn_create", "snn_create_static", "snn_step", "snn_route", "snn_step_route",
    "snn_deliver", "snn_run", "snn_run_partitioned", "snn_set_tuning", "snn_get_tuning",
    "snn_kernel_times", "snn_flush", "snn_sync", "snn_time",
    "snn_bin_geometry",
    "snn_ring_events",
    "snn_read_spikes", "snn_read_routes",
    "snn_read_counters", "snn_destroy", "snn_last_error",
    "snn_setup_create", "snn_setup_sizes", "snn_setup_fill_rows", "snn_setup_fill_routes",
    "snn_setup_input_bound", "snn_setup_destroy", "snn_setup_model_params",
]

u32, u64, i32, f32, f64 = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int32, ctypes.c_float, ctypes.c_double
vp = ctypes.c_void_p


class snn_params(ctypes.Structure):
    _fields_ = [
        ("n_neurons", u32), ("n_partitions", u32), ("gpus_per_node", u32), ("max_delay", u32),
        ("alpha", f32), ("theta", f32), ("u_reset", f32), ("w_ext", f32),
        ("n_ref", u32), ("poisson_thr", u32 * 15),
        ("seed", u64), ("weight_type", u32), ("flags", u32),
        ("raster_thr_on", u32), ("raster_thr_off", u32), ("raster_period", u32), ("raster_on", u32),
        ("bucket_total", u64), ("recv_total", u64),
        ("log_steps", u32), ("input_bound", f32), ("log_cap", u64),
        ("bin_cap", u64), ("stage_cap", u64), ("tile_neurons", u32),
    ]


class snn_network_dev(ctypes.Structure):
    _fields_ = [(n, vp) for n in (
        "row_ptr", "n_local", "delay_off", "tgt_delay", "weight", "vp_ptr", "vp_part", "vp_rec",
        "part_of_neuron", "bucket_off", "recv_off", "u", "ref", "ring")]


class snn_tuning(ctypes.Structure):
    _fields_ = [("update_blocks", u32), ("recv_split", u32), ("recv_merged", u32)]


class snn_setup_spec(ctypes.Structure):
    _fields_ = [
        ("seed", u64), ("n_neurons", u32), ("k_in", u32), ("max_delay", u32),
        ("n_partitions", u32), ("topology", u32), ("vp_set_size", u32),
        ("remote_frac", f64), ("w_exc", f64), ("w_inh", f64), ("w_jitter", f64),
        ("gpus_per_node", u32), ("weight_type", u32), ("n_threads", u32), ("verbose", u32),
        ("n_clusters", u32), ("p_in", f64),
    ]


class snn_model(ctypes.Structure):
    _fields_ = [(n, f64) for n in ("dt_ms", "tau_m_ms", "theta_mv", "u_reset_mv", "t_ref_ms",
                                   "nu_ext_hz", "w_ext_mv", "rate_on_hz", "rate_off_hz")]


class SNNError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"snn status {status}: {msg}")
        self.status = status


_lib = None


def lib() -> ctypes.CDLL:
    """The HIP library.  There is no fallback: without it nothing runs."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python paper_2205_07125_amd/build.py` (or __graft_entry__.build())")
        # One HIP runtime per process: torch (which owns the device memory and
        # streams) ships its own libamdhip64 and asks for it under another
        # name, so it is loaded first; the library's libamdhip64.so.7 then
        # resolves to the same copy.  Loaded the other way round, the process
        # would hold two runtimes and the second finds no device.
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        I = ctypes.c_int
        sig = {
            "snn_ring_stride": (u64, [u32]),
            "snn_workspace_size": (I, [ctypes.POINTER(snn_params), ctypes.POINTER(ctypes.c_size_t)]),
            "snn_create": (I, [ctypes.POINTER(snn_params), ctypes.POINTER(snn_network_dev), vp,
                               ctypes.c_size_t, vp, ctypes.POINTER(vp)]),
            "snn_create_static": (I, [ctypes.POINTER(snn_params), ctypes.POINTER(snn_network_dev),
                                      vp, ctypes.POINTER(vp)]),
            "snn_step": (I, [vp]),
            "snn_route": (I, [vp, I]),
            "snn_step_route": (I, [vp, I]),
            "snn_deliver": (I, [vp]),
            "snn_run": (I, [vp, u32, I, I]),
            "snn_run_partitioned": (I, [vp, u32, I, I, vp]),
            "snn_set_tuning": (I, [vp, ctypes.POINTER(snn_tuning)]),
            "snn_get_tuning": (I, [vp, ctypes.POINTER(snn_tuning)]),
            "snn_kernel_times": (I, [vp, u32, I, vp]),
            "snn_flush": (I, [vp]),
            "snn_sync": (I, [vp]),
            "snn_ring_events": (I, [vp, ctypes.POINTER(u64)]),
            "snn_time": (u64, [vp]),
            "snn_bin_geometry": (I, [ctypes.POINTER(snn_params)] + [ctypes.POINTER(u32)] * 3),
            "snn_read_spikes": (I, [vp, u64, u32, vp, u64, vp, ctypes.POINTER(u64)]),
            "snn_read_routes": (I, [vp, I, vp, vp, u64, ctypes.POINTER(u64)]),
            "snn_read_counters": (I, [vp, u64, u32, vp]),
            "snn_destroy": (I, [vp]),
            "snn_last_error": (ctypes.c_char_p, []),
            "snn_setup_create": (I, [ctypes.POINTER(snn_setup_spec), vp, vp, vp,
                                     ctypes.POINTER(vp)]),
            "snn_setup_sizes": (I, [vp] + [ctypes.POINTER(u64)] * 4),
            "snn_setup_fill_rows": (I, [vp] * 6),
            "snn_setup_fill_routes": (I, [vp] * 9),
            "snn_setup_input_bound": (I, [vp, ctypes.POINTER(f32)]),
            "snn_setup_destroy": (None, [vp]),
            "snn_setup_model_params": (I, [ctypes.POINTER(snn_model), ctypes.POINTER(snn_params)]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(status: int):
    if status != SNN_OK:
        raise SNNError(status, lib().snn_last_error().decode(errors="replace"))
    return status


# Same names as the C ABI; each one marshals its arguments and checks the status.
def snn_ring_stride(n: int) -> int:
    return int(lib().snn_ring_stride(n))


def snn_workspace_size(params: snn_params) -> int:
    out = ctypes.c_size_t(0)
    check(lib().snn_workspace_size(ctypes.byref(params), ctypes.byref(out)))
    return out.value


def snn_create(params: snn_params, net: snn_network_dev, workspace: int, ws_bytes: int,
               stream: int) -> int:
    h = vp()
    check(lib().snn_create(ctypes.byref(params), ctypes.byref(net), workspace, ws_bytes, stream,
                           ctypes.byref(h)))
    return h.value


def snn_create_static(params: snn_params, net: snn_network_dev, stream: int) -> int:
    h = vp()
    check(lib().snn_create_static(ctypes.byref(params), ctypes.byref(net), stream,
                                  ctypes.byref(h)))
    return h.value


def snn_step(h):
    check(lib().snn_step(h))


def snn_route(h, mode: int):
    check(lib().snn_route(h, mode))


def snn_step_route(h, mode: int):
    check(lib().snn_step_route(h, mode))


def snn_deliver(h):
    check(lib().snn_deliver(h))


def snn_run(h, n_steps: int, mode: int, use_graph):
    """use_graph: False / 0 eager, True / 1 16-step graphs, 2 one graph of all steps."""
    check(lib().snn_run(h, n_steps, mode, int(use_graph)))


def snn_run_partitioned(h, n_steps: int, mode: int, use_graph, part_start):
    import numpy as np
    starts = np.ascontiguousarray(part_start, np.uint32)
    check(lib().snn_run_partitioned(h, n_steps, mode, int(use_graph),
                                    starts.ctypes.data_as(ctypes.c_void_p)))


def snn_set_tuning(h, update_blocks: int = 0, recv_split: int = 0, recv_merged: int = 1):
    """Defaults are the library's own: one update block per tile, as many
    receive blocks per node as the receive launch holds, the receive side as
    one launch."""
    t = snn_tuning(update_blocks=update_blocks, recv_split=recv_split, recv_merged=recv_merged)
    check(lib().snn_set_tuning(h, ctypes.byref(t)))


def snn_get_tuning(h) -> dict:
    t = snn_tuning()
    check(lib().snn_get_tuning(h, ctypes.byref(t)))
    return {"update_blocks": t.update_blocks, "recv_split": t.recv_split,
            "recv_merged": t.recv_merged}


def snn_kernel_times(h, n_steps: int, mode: int):
    """-> list of SNN_NKERNEL average kernel durations (ms)."""
    out = (f32 * SNN_NKERNEL)()
    check(lib().snn_kernel_times(h, n_steps, mode, out))
    return [float(x) for x in out]


def snn_flush(h):
    check(lib().snn_flush(h))


def snn_sync(h):
    check(lib().snn_sync(h))


def snn_ring_events(h) -> int:
    n = u64()
    check(lib().snn_ring_events(h, ctypes.byref(n)))
    return n.value


def snn_setup_model_params(params: snn_params, **model) -> snn_params:
    """Fills params' model constants (alpha, theta, u_reset, w_ext, n_ref,
    poisson_thr, raster thresholds) from the physical ones (snn_model's
    fields as keywords); returns params."""
    m = snn_model(**model)
    check(lib().snn_setup_model_params(ctypes.byref(m), ctypes.byref(params)))
    return params


def snn_bin_geometry(n_neurons: int, tile_neurons: int = 0):
    """-> (tile_neurons, deliver_blocks, stage_blocks) of the binned delivery
    for n_neurons neurons and a requested tile size (0: the default)."""
    p = snn_params(n_neurons=n_neurons, tile_neurons=tile_neurons)
    a, b, c = u32(), u32(), u32()
    check(lib().snn_bin_geometry(ctypes.byref(p), ctypes.byref(a), ctypes.byref(b),
                                 ctypes.byref(c)))
    return a.value, b.value, c.value


def snn_time(h) -> int:
    return int(lib().snn_time(h))


def snn_destroy(h):
    check(lib().snn_destroy(h))


def snn_last_error() -> str:
    return lib().snn_last_error().decode(errors="replace")
