"""Seeded synthetic inputs shared by the CPU oracle and the GPU path.

This package only generates inputs (the synapse list, the partition map and the
initial membrane state) and names the workloads; it holds none of the method's
arithmetic.  The native part is ``libsynth.so`` built from ``synth.c`` by
``synth/build.py``.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from .workloads import (  # noqa: F401  (re-exported)
    TOPO_BATCHED,
    TOPO_CLUSTERED,
    TOPO_LOOPBACK,
    TOPO_LOOPBACK_SETS,
    TOPO_MATERIALIZED,
    WORKLOADS,
    Workload,
    get_workload,
)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsynth.so")


class _Spec(ctypes.Structure):
    _fields_ = [
        ("seed", ctypes.c_uint64),
        ("n_neurons", ctypes.c_uint32),
        ("k_in", ctypes.c_uint32),
        ("max_delay", ctypes.c_uint32),
        ("n_partitions", ctypes.c_uint32),
        ("topology", ctypes.c_uint32),
        ("vp_set_size", ctypes.c_uint32),
        ("remote_frac", ctypes.c_double),
        ("w_exc", ctypes.c_double),
        ("w_inh", ctypes.c_double),
        ("w_jitter", ctypes.c_double),
        ("n_clusters", ctypes.c_uint32),
        ("p_in", ctypes.c_double),
    ]


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run synth/build.py (or __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        L.syn_create.restype = P
        L.syn_create.argtypes = [ctypes.POINTER(_Spec), P, P]
        L.syn_destroy.argtypes = [P]
        L.syn_edges.argtypes = [P, ctypes.c_uint32, ctypes.c_uint32, P, P, P, P, P]
        L.syn_part_map.argtypes = [P, P]
        L.syn_set_part_map.restype = ctypes.c_int
        L.syn_set_part_map.argtypes = [P, P]
        L.syn_cluster_of.restype = ctypes.c_uint32
        L.syn_cluster_of.argtypes = [P, ctypes.c_uint32]
        L.syn_initial_u.argtypes = [ctypes.c_uint64, ctypes.c_double, ctypes.c_uint32, P]
        L.syn_lognormal_sizes.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_double,
                                          ctypes.c_double, ctypes.c_uint32, ctypes.c_uint32, P]
        L.syn_uniform_doubles.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                          ctypes.c_double, ctypes.c_double, P]
        L.syn_vp_set.restype = ctypes.c_int
        L.syn_vp_set.argtypes = [P, ctypes.c_uint32, P]
        L.syn_hash.restype = ctypes.c_uint64
        L.syn_hash.argtypes = [ctypes.c_uint64] * 4
        _lib = L
    return _lib


def _ptr(a: np.ndarray | None):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def partition_starts(wl: Workload) -> np.ndarray | None:
    """Ascending neuron offsets (P+1) of the materialised partitions, or None
    for the loopback topologies (every neuron in partition 0)."""
    if wl.topology in (TOPO_LOOPBACK, TOPO_LOOPBACK_SETS):
        return None
    return np.concatenate([[0], np.cumsum(partition_sizes(wl))]).astype(np.uint32)


def partition_sizes(wl: Workload) -> np.ndarray:
    if wl.topology in (TOPO_MATERIALIZED, TOPO_CLUSTERED):
        P = wl.n_partitions
        base, rem = divmod(wl.n_neurons, P)
        return np.array([base + (1 if p < rem else 0) for p in range(P)], dtype=np.uint32)
    if wl.topology == TOPO_BATCHED:
        return batched_sizes(wl.seed, wl.n_partitions, wl.size_median, wl.size_sigma_ln,
                             wl.size_lo, wl.size_hi, wl.size_scale)
    raise ValueError("loopback topologies have a single materialised partition")


def batched_sizes(seed, n_part, median, sigma_ln, lo, hi, scale=1.0) -> np.ndarray:
    out = np.zeros(n_part, dtype=np.uint32)
    lib().syn_lognormal_sizes(seed, n_part, median, sigma_ln, lo, hi, _ptr(out))
    if scale != 1.0:
        out = np.maximum(np.round(out.astype(np.float64) * scale), 2).astype(np.uint32)
    return out


def cross_fracs(wl: Workload) -> np.ndarray | None:
    if wl.topology != TOPO_BATCHED:
        return None
    out = np.zeros(wl.n_partitions, dtype=np.float64)
    lib().syn_uniform_doubles(wl.seed, 1, wl.n_partitions, wl.cross_lo, wl.cross_hi, _ptr(out))
    return out


class Generator:
    """Handle over the native generator for one workload.  part_map: an
    explicit neuron -> partition map (int32[n_neurons]) in place of the
    workload's contiguous partitions (materialised and clustered topologies),
    e.g. the neuron-GPU mapping a partitioning produced."""

    def __init__(self, wl: Workload, part_map: np.ndarray | None = None):
        self.wl = wl
        spec = _Spec(wl.seed, wl.n_neurons, wl.k_in, wl.max_delay, wl.n_partitions, wl.topology,
                     wl.vp_set_size, wl.remote_frac, wl.w_exc, wl.w_inh, wl.w_jitter,
                     wl.n_clusters, wl.p_in)
        self._starts = partition_starts(wl)
        self._fracs = cross_fracs(wl)
        h = lib().syn_create(ctypes.byref(spec), _ptr(self._starts), _ptr(self._fracs))
        if not h:
            raise ValueError(f"generator rejected workload {wl.name}")
        self.handle = ctypes.c_void_p(h)
        if part_map is not None:
            pm = np.ascontiguousarray(part_map, np.int32)
            if len(pm) != wl.n_neurons or lib().syn_set_part_map(self.handle, _ptr(pm)) != 0:
                raise ValueError("partition map rejected: one entry per neuron in "
                                 "[0, n_partitions), materialised or clustered topology")

    def close(self):
        if self.handle:
            lib().syn_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def edges(self, tgt_lo: int = 0, tgt_hi: int | None = None) -> dict:
        """Canonical synapse list (target-major, then k) as numpy arrays."""
        if tgt_hi is None:
            tgt_hi = self.wl.n_neurons
        m = (tgt_hi - tgt_lo) * self.wl.k_in
        out = dict(src=np.empty(m, np.uint32), tgt=np.empty(m, np.uint32),
                   delay=np.empty(m, np.uint8), vp=np.empty(m, np.uint16),
                   w=np.empty(m, np.float32))
        lib().syn_edges(self.handle, tgt_lo, tgt_hi, _ptr(out["src"]), _ptr(out["tgt"]),
                        _ptr(out["delay"]), _ptr(out["vp"]), _ptr(out["w"]))
        return out

    def part_map(self) -> np.ndarray:
        out = np.empty(self.wl.n_neurons, np.int32)
        lib().syn_part_map(self.handle, _ptr(out))
        return out

    def clusters(self) -> np.ndarray:
        """Cluster of every neuron (clustered topology)."""
        f = lib().syn_cluster_of
        return np.array([f(self.handle, i) for i in range(self.wl.n_neurons)], np.uint32)

    def vp_set(self, src: int) -> np.ndarray | None:
        out = np.empty(max(self.wl.vp_set_size, 1), np.uint16)
        ok = lib().syn_vp_set(self.handle, src, _ptr(out))
        return out if ok else None


def initial_u(wl: Workload) -> np.ndarray:
    out = np.empty(wl.n_neurons, np.float32)
    lib().syn_initial_u(wl.seed, wl.theta_rel_mv, wl.n_neurons, _ptr(out))
    return out
