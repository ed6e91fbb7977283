"""Per-link traffic of a routed step, read from the device routing buffers:
who sends how many receive entries (flat view) or messages (two-level view)
to whom.  The paper's latency model waits for the GPU pair with the largest
traffic (Sec. V) and counts connections per GPU (Sec. VI, Fig. 4); this is
that bookkeeping for the step in the buffers.  Host-side analysis of what the
kernels produced; nothing here is on the simulation path."""
from __future__ import annotations

import numpy as np


def link_traffic(sim, part: np.ndarray, two_level: bool = True) -> dict:
    """part: partition of every neuron (HostNetwork.part).  Uses the expanded
    receive lists and the node buckets of a two-level step (two_level), else
    the flat lists; -> dict with
      partition_matrix [P][P]    entries per (source partition, destination partition)
      node_matrix [P][n_nodes]   messages per (source partition, destination node)
                                 (two-level only)
      level1 / level2            messages to the source's own node / to other nodes
      max_partition_link, max_node_link
      connections_flat [P], connections_two_level [P]
                                 destinations each source partition sends to."""
    wl = sim.wl
    P, G, nn = wl.n_partitions, wl.gpus_per_node, wl.n_nodes
    part = np.asarray(part, np.int64)
    lists = sim.read_routes(1 if two_level else 0, sources_only=True)
    pm = np.zeros((P, P), np.int64)
    for p, src in enumerate(lists):
        if len(src):
            pm[:, p] = np.bincount(part[src.astype(np.int64)], minlength=P)
    out = {"partition_matrix": pm, "max_partition_link": int(pm.max()) if pm.size else 0,
           "connections_flat": (pm > 0).sum(axis=1)}
    if two_level:
        buckets = sim.read_routes(2, sources_only=True)
        nm = np.zeros((P, nn), np.int64)
        for n, src in enumerate(buckets):
            if len(src):
                nm[:, n] = np.bincount(part[src.astype(np.int64)], minlength=P)
        own = np.arange(P) // G
        level1 = int(nm[np.arange(P), own].sum())
        out.update(node_matrix=nm, level1=level1, level2=int(nm.sum()) - level1,
                   max_node_link=int(nm.max()) if nm.size else 0,
                   connections_two_level=(nm > 0).sum(axis=1))
    return out
