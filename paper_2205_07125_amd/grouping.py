"""Grouping of GPUs for two-level routing (Algorithm 2, Sec. IV-B), on the host.

Inputs are the GPU connection-probability matrix PG[N, N] and the data
volume of each GPU WG[N] (the summed weight of its neurons).  The output is a
routing table TB: for traffic from GPU i to GPU j, the next hop.  GPUs of one
group exchange directly (level 1).  Traffic to another group goes to a bridge
GPU, which forwards it to the destination (level 2).  There is one bridge per
(group, destination group).  The objectives are few connections per GPU, and
little inter-group traffic, the sum of PG[i, j] * WG[i] * WG[j] over pairs in
different groups (Sec. IV-B).

The paper outlines the algorithm without every rule; this module reads it so:
  * Groups have near-equal sizes, at most cap = ceil(N / n_groups).  A group
    grows greedily from a seed GPU.  The GPU added each time is the
    unassigned one with the largest summed connection probability, in either
    direction, to the members so far.  Growth stops at cap members, or once
    the group's volume reaches the mean group volume sum(WG) / n_groups.
    GPUs left over join the group with room that they are most connected to.
  * In the first iteration, seeds are taken by decreasing total connection
    probability.  Later iterations take them in a seeded random order.  The
    grouping kept is the one with the least inter-group traffic.
  * Bridges are spread over the members of a group, as the paper asks for
    balanced traffic (Sec. III, Sec. IV-B): one member bridging every group
    would carry all of the group's level-2 traffic.  The destination groups
    are taken by decreasing traffic from g.  Each goes to the member with the
    least level-2 traffic so far.  select_bridges(balance="roles") balances
    the number of roles instead.

With every pair connected, a GPU in a group of s has s - 1 level-1
connections.  On average it bridges (n_groups - 1) / s groups, each fanning
out to s GPUs.  That is a mean of about s + N / s - 2 connections, which is least at s near
sqrt(N): 88 for N = 2000, the mean the paper reports for its 2,000 GPUs
(Sec. V, Fig. 4).

Plain numpy; nothing here runs on the GPU.  The device path groups
partitions by node: partition p is on node p div G.  relabel() renumbers
partitions so that each group of size G holds contiguous ids."""
from __future__ import annotations

import numpy as np


def inter_group_traffic(PG: np.ndarray, WG: np.ndarray, group_of: np.ndarray) -> float:
    """Sum of PG[i, j] * WG[i] * WG[j] over pairs i, j in different groups."""
    T = np.asarray(PG, np.float64) * np.outer(WG, WG)
    diff = group_of[:, None] != group_of[None, :]
    return float(T[diff].sum())


def greedy_groups(PG: np.ndarray, WG: np.ndarray, n_groups: int,
                  order: np.ndarray | None = None) -> np.ndarray:
    """One greedy pass.  Seeds are tried in `order`, by default by decreasing
    total connection probability.  Returns group_of[N] in [0, n_groups)."""
    PG = np.asarray(PG, np.float64)
    WG = np.asarray(WG, np.float64)
    N = len(WG)
    if not 1 <= n_groups <= N:
        raise ValueError("need 1 <= n_groups <= number of GPUs")
    cap = -(-N // n_groups)
    target = WG.sum() / n_groups
    sym = PG + PG.T
    if order is None:
        order = np.argsort(-sym.sum(axis=1), kind="stable")
    group_of = np.full(N, -1, np.int64)
    size = np.zeros(n_groups, np.int64)
    n_free = N
    g = 0
    for s in order:
        if g == n_groups:
            break
        if group_of[s] >= 0:
            continue
        group_of[s] = g
        size[g] = 1
        n_free -= 1
        vol = WG[s]
        affinity = sym[s].copy()
        # grow, but leave one unassigned GPU to seed each group still to open
        while size[g] < cap and vol < target and n_free > n_groups - g - 1:
            cand = np.where(group_of < 0, affinity, -np.inf)
            j = int(np.argmax(cand))
            group_of[j] = g
            size[g] += 1
            n_free -= 1
            vol += WG[j]
            affinity += sym[j]
        g += 1
    # Leftover GPUs: most connected group with room.  Every group is open by
    # now: each growth step left a GPU for every group still to open.
    for i in np.where(group_of < 0)[0]:
        strength = np.bincount(group_of[group_of >= 0], weights=sym[i, group_of >= 0],
                               minlength=n_groups)
        strength[size >= cap] = -np.inf
        k = int(np.argmax(strength))
        group_of[i] = k
        size[k] += 1
    return group_of


def group_gpus(PG: np.ndarray, WG: np.ndarray, n_groups: int, iters: int = 8,
               seed: int = 0) -> np.ndarray:
    """The loop of Algorithm 2: `iters` greedy passes, keeping the grouping
    with the least inter-group traffic.  Returns group_of[N]."""
    N = len(WG)
    rng = np.random.default_rng(seed)
    best, best_cost = None, np.inf
    for t in range(max(iters, 1)):
        go = greedy_groups(PG, WG, n_groups, None if t == 0 else rng.permutation(N))
        cost = inter_group_traffic(PG, WG, go)
        if cost < best_cost:
            best, best_cost = go, cost
    return best


def select_bridges(PG: np.ndarray, WG: np.ndarray, group_of: np.ndarray,
                   balance: str = "traffic") -> np.ndarray:
    """Returns bridge[g, h], the member of group g that forwards g's traffic
    to group h.  The entry is -1 on the diagonal.  Destination groups are
    taken by decreasing traffic from g.
      balance="traffic": each goes to the member with the least level-2
                         traffic so far, ties to the member with the most
                         traffic to h, as in scheduling the largest job
                         first onto the least loaded machine.  No bridge
                         then carries more than its fair share of g's
                         level-2 traffic plus the largest single flow.
      balance="roles":   each goes to the member with the fewest roles so
                         far, ties to the member with the most traffic to h.
                         Connection counts come out even, but one bridge may
                         carry much more traffic than another."""
    if balance not in ("roles", "traffic"):
        raise ValueError("balance must be 'roles' or 'traffic'")
    n_groups = int(group_of.max()) + 1
    if np.any(np.bincount(group_of, minlength=n_groups) == 0):
        raise ValueError("every group id below the largest must have members")
    T = np.asarray(PG, np.float64) * np.outer(WG, WG)
    to_group = np.zeros((len(WG), n_groups))
    for h in range(n_groups):
        to_group[:, h] = T[:, group_of == h].sum(axis=1)
    bridge = np.full((n_groups, n_groups), -1, np.int64)
    for g in range(n_groups):
        members = np.where(group_of == g)[0]
        roles = np.zeros(len(members), np.int64)
        load = np.zeros(len(members))
        flow = to_group[members].sum(axis=0)          # g's traffic to each group
        others = [h for h in range(n_groups) if h != g]
        others.sort(key=lambda h: (-flow[h], h))
        for h in others:
            free = roles == roles.min() if balance == "roles" else load == load.min()
            k = int(np.argmax(np.where(free, to_group[members, h], -np.inf)))
            bridge[g, h] = members[k]
            roles[k] += 1
            load[k] += flow[h]
    return bridge


def routing_table(group_of: np.ndarray, bridge: np.ndarray) -> np.ndarray:
    """TB[i, j]: next hop of traffic from GPU i to GPU j.  It is j itself
    inside a group, or where i is its group's bridge towards j's group.
    Otherwise it is that bridge.  TB[i, i] = i."""
    N = len(group_of)
    ids = np.arange(N)
    b = bridge[group_of[:, None], group_of[None, :]]
    direct = (group_of[:, None] == group_of[None, :]) | (b == ids[:, None])
    return np.where(direct, ids[None, :], b)


def hop_matrix(dest: np.ndarray, TB: np.ndarray) -> np.ndarray:
    """Connections under TB.  H[a, b] is true when some traffic i -> j,
    with dest[i, j] set and i != j, takes the hop a -> b.  That hop is
    either i -> TB[i, j], or TB[i, j] -> j when the bridge forwards."""
    N = dest.shape[0]
    i, j = np.nonzero(dest & ~np.eye(N, dtype=bool))
    nh = TB[i, j]
    H = np.zeros((N, N), bool)
    H[i, nh] = True
    fwd = nh != j
    H[nh[fwd], j[fwd]] = True
    np.fill_diagonal(H, False)
    return H


def connections(PG: np.ndarray, TB: np.ndarray | None = None) -> np.ndarray:
    """Connections departing from each GPU.  Without TB (flat peer-to-peer
    exchange) these are its destinations with PG > 0.  With TB they are the
    distinct hops that it sends on, forwarding included."""
    dest = np.asarray(PG) > 0
    N = dest.shape[0]
    if TB is None:
        return (dest & ~np.eye(N, dtype=bool)).sum(axis=1)
    return hop_matrix(dest, TB).sum(axis=1)


def link_load(T: np.ndarray, TB: np.ndarray) -> np.ndarray:
    """Traffic on each connection when the traffic matrix T[i, j] follows TB.
    T[i, j] goes over i -> TB[i, j], and then over TB[i, j] -> j when a
    bridge forwards it.  The result L[a, b] has a zero diagonal.  Messages
    are not merged at the bridge here; the device path sends one message per
    (spike, node), which merges them, and counts that per step."""
    T = np.asarray(T, np.float64)
    N = T.shape[0]
    L = np.zeros((N, N))
    i, j = np.nonzero(T * ~np.eye(N, dtype=bool))
    nh = TB[i, j]
    np.add.at(L, (i, nh), T[i, j])
    fwd = nh != j
    np.add.at(L, (nh[fwd], j[fwd]), T[i, j][fwd])
    return L


def relabel(group_of: np.ndarray) -> np.ndarray:
    """Returns new_id[N]: GPUs renumbered so that each group's members are
    contiguous.  Groups are taken in order, and members by old id within a
    group.  With groups of equal size G, group k holds ids [k G, (k+1) G),
    which is the node layout that the device path assumes."""
    order = np.lexsort((np.arange(len(group_of)), group_of))
    new_id = np.empty(len(group_of), np.int64)
    new_id[order] = np.arange(len(group_of))
    return new_id


def dense_group_size(n: int) -> int:
    """Group size s that minimises s + ceil(n / s) - 2, the approximate
    connections per GPU when every pair of GPUs exchanges traffic."""
    s = np.arange(1, n + 1)
    return int(s[np.argmin(s + -(-n // s) - 2)])


def synthetic_pg(n_gpus: int, n_regions: int, p_in: float, p_out: float, seed: int,
                 wg_sigma: float = 0.3) -> tuple[np.ndarray, np.ndarray]:
    """Seeded GPU connection probabilities with regional structure.  GPUs
    get random regions.  A pair within one region is connected with
    probability p_in, any other pair with probability p_out, and a connected
    pair gets a uniform strength in (0, 1).  Volumes are lognormal around 1.
    Returns (PG, WG)."""
    rng = np.random.default_rng(seed)
    region = rng.integers(0, n_regions, n_gpus)
    same = region[:, None] == region[None, :]
    U = rng.random((n_gpus, n_gpus))
    PG = np.where(same, U < p_in, U < p_out) * rng.random((n_gpus, n_gpus))
    np.fill_diagonal(PG, 0.0)
    WG = np.exp(rng.normal(0.0, wg_sigma, n_gpus))
    return PG, WG


def partition_graph(part: np.ndarray, vp_ptr: np.ndarray, vp_part: np.ndarray,
                    n_partitions: int) -> tuple[np.ndarray, np.ndarray]:
    """PG and WG for the partitions of a built network.  The inputs are the
    network's partition of each neuron, and each source's list of distinct
    destination partitions (vp_ptr / vp_part).  PG[p, q] is the fraction of
    partition p's neurons with a synapse in partition q.  WG[p] is the number
    of (source, destination partition) pairs sourced in p, the messages that
    flat exchange would send if every neuron of p fired once."""
    part = np.asarray(part, np.int64)
    P = int(n_partitions)
    n_dest = np.diff(np.asarray(vp_ptr, np.int64))
    pairs = int(vp_ptr[-1])
    src_part = np.repeat(part, n_dest)
    dst = np.asarray(vp_part[:pairs], np.int64)
    counts = np.bincount(src_part * P + dst, minlength=P * P).reshape(P, P).astype(np.float64)
    size = np.bincount(part, minlength=P).astype(np.float64)
    PG = counts / np.maximum(size, 1.0)[:, None]
    WG = counts.sum(axis=1)
    return PG, WG


def routing_report(PG: np.ndarray, WG: np.ndarray, n_groups: int, iters: int = 8,
                   seed: int = 0, balance: str = "traffic") -> dict:
    """Algorithm 2 end to end, and what the paper measures of it (Sec. V,
    Figs. 3(b) and 4).  Groups, bridges and TB come first.  Then, per GPU,
    the connections under flat and two-level routing, and the traffic T =
    PG * WG * WG leaving it towards other groups (level 2) under both."""
    PG = np.asarray(PG, np.float64)
    WG = np.asarray(WG, np.float64)
    go = group_gpus(PG, WG, n_groups, iters, seed)
    br = select_bridges(PG, WG, go, balance)
    TB = routing_table(go, br)
    T = PG * np.outer(WG, WG)
    np.fill_diagonal(T, 0.0)
    cross = go[:, None] != go[None, :]
    L = link_load(T, TB)
    c_flat, c_two = connections(PG), connections(PG, TB)
    level2_flat = (T * cross).sum(axis=1)
    level2_two = (L * cross).sum(axis=1)
    return dict(group_of=go, bridge=br, TB=TB,
                inter_group_traffic=inter_group_traffic(PG, WG, go),
                connections_flat=c_flat, connections_two_level=c_two,
                mean_connections_flat=float(c_flat.mean()),
                mean_connections_two_level=float(c_two.mean()),
                level2_flat=level2_flat, level2_two_level=level2_two,
                peak_level2_flat=float(level2_flat.max()),
                peak_level2_two_level=float(level2_two.max()))


def _main(argv=None) -> None:
    """Connections per GPU, flat against two-level, on a seeded random PG in
    which a GPU reaches a given mean number of others.  This is the count of
    Sec. V, Fig. 4."""
    import argparse
    import json
    ap = argparse.ArgumentParser(prog="python -m paper_2205_07125_amd.grouping")
    ap.add_argument("--gpus", type=int, default=2000)
    ap.add_argument("--reach", type=float, default=1552.0,
                    help="mean number of GPUs each GPU sends to")
    ap.add_argument("--group-size", type=int, default=0,
                    help="GPUs per group (default: dense_group_size)")
    ap.add_argument("--iters", type=int, default=1)
    ap.add_argument("--balance", choices=["traffic", "roles"], default="traffic")
    ap.add_argument("--seed", type=int, default=2205)
    a = ap.parse_args(argv)
    n = a.gpus
    rng = np.random.default_rng(a.seed)
    PG = (rng.random((n, n)) < a.reach / max(n - 1, 1)) * rng.random((n, n))
    np.fill_diagonal(PG, 0.0)
    WG = np.exp(rng.normal(0.0, 0.3, n))
    s = a.group_size or dense_group_size(n)
    r = routing_report(PG, WG, -(-n // s), a.iters, a.seed, a.balance)
    print(json.dumps({
        "gpus": n, "group_size": s, "groups": -(-n // s),
        "mean_connections_flat": round(r["mean_connections_flat"], 2),
        "mean_connections_two_level": round(r["mean_connections_two_level"], 2),
        "max_connections_two_level": int(r["connections_two_level"].max()),
        "peak_level2_flat": round(r["peak_level2_flat"], 1),
        "peak_level2_two_level": round(r["peak_level2_two_level"], 1)}))


if __name__ == "__main__":
    _main()
