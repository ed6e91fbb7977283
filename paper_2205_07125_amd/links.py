"""Per-link traffic of a routed step, read from the device routing buffers:
who sends how many receive entries (flat view) or messages (two-level view)
to whom.  The paper's latency model waits for the GPU pair with the largest
traffic (Sec. V) and counts connections per GPU (Sec. V, Fig. 4); this is
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


def bridge_load(node_matrix: np.ndarray, gpus_per_node: int, policy: str = "balanced") -> dict:
    """Receive-side bridges of two-level routing: which GPU of node n takes
    the level-2 messages of source partition p, and then expands their masks
    for the node (Sec. IV-B).  node_matrix[p, n] counts messages from p to n
    (link_traffic's node_matrix).  Messages to the source's own node are
    level 1 and need no bridge.
      policy="fixed":    the node's first GPU bridges everything.
      policy="rotate":   GPU p mod G of the node, so that the sources take
                         turns whatever their traffic.
      policy="balanced": per node, the sources by decreasing message count,
                         each onto the member with the fewest level-2
                         messages so far (largest job first, least loaded
                         machine; ties to the lower GPU).  No member then
                         takes more than the node's mean plus one source's
                         messages.
    Returns dict:
      bridge [P][n_nodes]   receiving GPU (partition id), -1 where p sends
                            nothing or n is p's own node
      load [P]              level-2 messages each partition receives as a bridge
      peak                  load.max()
      connections [P]       distinct bridges each source partition sends to
    The bridge choice does not change what is delivered, only where the
    level-2 messages land."""
    nm = np.asarray(node_matrix, np.int64)
    P, n_nodes = nm.shape
    G = int(gpus_per_node)
    if policy not in ("fixed", "rotate", "balanced"):
        raise ValueError("policy must be 'fixed', 'rotate' or 'balanced'")
    own = np.arange(P) // G
    bridge = np.full((P, n_nodes), -1, np.int64)
    load = np.zeros(P, np.int64)
    for n in range(n_nodes):
        members = np.arange(n * G, min((n + 1) * G, P))
        srcs = np.nonzero((nm[:, n] > 0) & (own != n))[0]
        if not len(srcs) or not len(members):
            continue
        if policy == "fixed":
            bridge[srcs, n] = members[0]
        elif policy == "rotate":
            bridge[srcs, n] = members[srcs % len(members)]
        else:
            acc = np.zeros(len(members), np.int64)
            for p in srcs[np.argsort(-nm[srcs, n], kind="stable")]:
                k = int(np.argmin(acc))
                bridge[p, n] = members[k]
                acc[k] += nm[p, n]
        np.add.at(load, bridge[srcs, n], nm[srcs, n])
    conn = (bridge >= 0).sum(axis=1)
    return dict(bridge=bridge, load=load, peak=int(load.max()) if P else 0, connections=conn)
