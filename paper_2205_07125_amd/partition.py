"""Neuron -> GPU partitioning (Algorithm 1, Sec. IV-A), on the host.

Inputs are the neuron connection probabilities P[M, M] and the neuron
weights W[M].  W is the data volume that a neuron sends.  P may be a dense
array or a scipy sparse matrix; the brain's is very sparse.  The output is
the neuron -> GPU map PM[M].  The objective is the traffic cut by the map,
the sum of P[i, j] * W[i] * W[j] over neurons on different GPUs, with every
GPU's total weight near the mean sum(W) / N.

The paper gives the loop of Algorithm 1 but not its rules.  This module
reads it so:
  * Each pass starts every GPU from one seed neuron.  The first pass takes
    them farthest-first: the heaviest neuron, then each time the neuron the
    most hops away from the seeds so far, and among those the one least
    connected to them.  Neurons with no path to a seed are the farthest, so
    each connected component gets a seed before any gets a second.  Later
    passes draw N distinct neurons with a seeded generator.
  * Then the GPUs take turns, in order.  A GPU whose weight is still below
    the mean takes the unassigned neuron with the largest summed connection
    probability, in either direction, to its members.  That is x_{i,t}, the
    neuron that pass t places on GPU i.  A GPU stops once its weight reaches
    the mean.  The turns end when no unassigned neuron is left, or no GPU is
    below the mean.  Any neuron still unassigned then goes to the lightest
    GPU, heaviest neuron first.
  * After T passes the map kept is the one with the least cut traffic.
Every GPU then ends below mean + max(W): it takes a neuron only while below
the mean.  Turns end with neurons left over only when every GPU has reached
the mean, so all weight is placed already and the leftovers weigh nothing.

gpu_graph() turns a map into the inputs of Algorithm 2, PG[N, N] and
WG[N].  Plain numpy / scipy; nothing here runs on the GPU."""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def _sym_csr(P) -> sp.csr_matrix:
    """P + P^T as CSR, with the diagonal dropped."""
    A = sp.csr_matrix(P, dtype=np.float64)
    A = (A + A.T).tocsr()
    A.setdiag(0.0)
    A.eliminate_zeros()
    return A


def cut_traffic(P, W: np.ndarray, pm: np.ndarray) -> float:
    """Sum of P[i, j] * W[i] * W[j] over pairs i, j on different GPUs."""
    C = sp.coo_matrix(P)
    W = np.asarray(W, np.float64)
    diff = pm[C.row] != pm[C.col]
    return float((C.data[diff] * W[C.row[diff]] * W[C.col[diff]]).sum())


def gpu_traffic(P, W: np.ndarray, pm: np.ndarray, n_gpus: int) -> np.ndarray:
    """Traffic each GPU sends to other GPUs: for GPU g, the sum of
    P[i, j] * W[i] * W[j] over i on g and j elsewhere."""
    C = sp.coo_matrix(P)
    W = np.asarray(W, np.float64)
    diff = pm[C.row] != pm[C.col]
    t = C.data[diff] * W[C.row[diff]] * W[C.col[diff]]
    return np.bincount(pm[C.row[diff]], weights=t, minlength=n_gpus)


def greedy_pass(P, W: np.ndarray, n_gpus: int, seeds: np.ndarray,
                A: sp.csr_matrix | None = None) -> np.ndarray:
    """One pass of Algorithm 1's loop from the given seed neurons (one per
    GPU, distinct).  Returns PM[M] in [0, n_gpus).

    Each GPU keeps its frontier sparse: the summed probability to its members
    of only the free neurons adjacent to them, in a max-heap (stale entries
    are skipped when popped).  A GPU whose frontier is empty takes the
    lowest-id free neuron, which is what a dense argmax over all-zero sums
    would pick, so the maps equal those of the dense form while memory stays
    O(synapses + M) instead of O(n_gpus * M)."""
    import heapq
    W = np.asarray(W, np.float64)
    M = len(W)
    if not 1 <= n_gpus <= M:
        raise ValueError("need 1 <= number of GPUs <= number of neurons")
    seeds = np.asarray(seeds, np.int64)
    if len(seeds) != n_gpus or len(np.unique(seeds)) != n_gpus:
        raise ValueError("need one distinct seed neuron per GPU")
    A = _sym_csr(P) if A is None else A
    target = W.sum() / n_gpus
    pm = np.full(M, -1, np.int64)
    load = np.zeros(n_gpus)
    aff = [dict() for _ in range(n_gpus)]   # free neuron -> summed probability to members
    heaps = [[] for _ in range(n_gpus)]     # (-sum, neuron), possibly stale
    free = np.ones(M, bool)
    lowest_free = 0

    def place(i, j):
        pm[j] = i
        free[j] = False
        load[i] += W[j]
        lo, hi = A.indptr[j], A.indptr[j + 1]
        ai, hp = aff[i], heaps[i]
        for k, a in zip(A.indices[lo:hi].tolist(), A.data[lo:hi].tolist()):
            if free[k]:
                v = ai.get(k, 0.0) + a
                ai[k] = v
                heapq.heappush(hp, (-v, k))

    def best(i):
        nonlocal lowest_free
        ai, hp = aff[i], heaps[i]
        while hp:
            v, k = hp[0]
            if free[k] and ai.get(k) == -v:
                return k
            heapq.heappop(hp)
        while not free[lowest_free]:
            lowest_free += 1
        return lowest_free

    for i, j in enumerate(seeds):
        place(i, int(j))
    n_free = M - n_gpus
    while n_free:
        moved = False
        for i in range(n_gpus):
            if not n_free:
                break
            if load[i] >= target:
                continue
            place(i, best(i))
            n_free -= 1
            moved = True
        if not moved:
            break
    for j in np.where(free)[0][np.argsort(-W[free], kind="stable")]:
        place(int(np.argmin(load)), int(j))
    return pm


def spread_seeds(A: sp.csr_matrix, W: np.ndarray, n_gpus: int) -> np.ndarray:
    """Farthest-first seeds: the heaviest neuron (lowest id on ties), then
    repeatedly the unseeded neuron with the most hops to its nearest seed;
    ties go to the least summed connection probability to the seeds so far,
    then to the heaviest, then to the lowest id.  A neuron without a path to
    any seed is infinitely far, so every connected component gets a seed
    before any gets a second, whether its clusters are dense or sparse; inside
    a component the summed probability separates clusters that hops cannot
    (every pair one hop apart, but weakly linked)."""
    from scipy.sparse.csgraph import shortest_path
    W = np.asarray(W, np.float64)
    M = len(W)
    seeds = [int(np.argmax(W))]
    dist = np.full(M, np.inf)
    tot = np.zeros(M)
    for _ in range(n_gpus - 1):
        j = seeds[-1]
        dist = np.minimum(dist, shortest_path(A, unweighted=True, indices=j))
        lo, hi = A.indptr[j], A.indptr[j + 1]
        tot[A.indices[lo:hi]] += A.data[lo:hi]
        d = dist.copy()
        d[seeds] = -1.0
        seeds.append(int(np.lexsort((np.arange(M), -W, tot, -d))[0]))
    return np.array(seeds, np.int64)


def partition_neurons(P, W: np.ndarray, n_gpus: int, iters: int = 4,
                      seed: int = 0) -> np.ndarray:
    """Algorithm 1: `iters` greedy passes, the first from spread_seeds and
    the others from seeded random seed neurons, keeping the map with the
    least cut traffic.  Returns PM[M]."""
    W = np.asarray(W, np.float64)
    A = _sym_csr(P)
    rng = np.random.default_rng(seed)
    best, best_cost = None, np.inf
    for t in range(max(iters, 1)):
        seeds = (spread_seeds(A, W, n_gpus) if t == 0
                 else rng.choice(len(W), n_gpus, replace=False))
        pm = greedy_pass(P, W, n_gpus, seeds, A)
        cost = cut_traffic(P, W, pm)
        if cost < best_cost:
            best, best_cost = pm, cost
    return best


def gpu_graph(P, W: np.ndarray, pm: np.ndarray, n_gpus: int) -> tuple[np.ndarray, np.ndarray]:
    """Inputs of Algorithm 2 from a neuron map.  WG[g] is the total weight of
    the neurons on GPU g.  PG[g, h] is the W-weighted mean of P over the pairs
    from g to h: sum of P[i, j] * W[i] * W[j], i on g and j on h, divided by
    WG[g] * WG[h].  PG[g, h] * WG[g] * WG[h] is then exactly the neuron
    traffic from g to h, so Algorithm 2's objective is the part of Algorithm
    1's cut that crosses groups."""
    C = sp.coo_matrix(P)
    W = np.asarray(W, np.float64)
    WG = np.bincount(pm, weights=W, minlength=n_gpus)
    t = C.data * W[C.row] * W[C.col]
    T = np.bincount(pm[C.row] * n_gpus + pm[C.col], weights=t,
                    minlength=n_gpus * n_gpus).reshape(n_gpus, n_gpus)
    np.fill_diagonal(T, 0.0)
    denom = np.outer(WG, WG)
    PG = np.divide(T, denom, out=np.zeros_like(T), where=denom > 0)
    return PG, WG


def synthetic_neurons(M: int, n_clusters: int, k_in: float, k_out: float, seed: int,
                      rate_sigma: float = 0.5) -> tuple[sp.csr_matrix, np.ndarray]:
    """Seeded clustered connectivity: neurons get random clusters of uneven
    size.  Each neuron draws about k_in targets in its own cluster and k_out
    elsewhere, each with a uniform probability in (0, 1].  W is the
    out-degree times a lognormal rate.  Returns (P as CSR, W)."""
    rng = np.random.default_rng(seed)
    cl = np.sort(rng.integers(0, n_clusters, M))
    rows, cols = [], []
    members = [np.where(cl == c)[0] for c in range(n_clusters)]
    for i in range(M):
        own = members[cl[i]]
        ni = min(rng.poisson(k_in), len(own))
        rows.append(np.full(ni, i))
        cols.append(rng.choice(own, ni, replace=False))
        no = rng.poisson(k_out)
        rows.append(np.full(no, i))
        cols.append(rng.integers(0, M, no))
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    keep = r != c
    P = sp.csr_matrix((1.0 - rng.random(int(keep.sum())), (r[keep], c[keep])), shape=(M, M))
    P.sum_duplicates()
    P.data = np.minimum(P.data, 1.0)
    deg = np.diff(P.indptr).astype(np.float64)
    W = np.maximum(deg, 1.0) * np.exp(rng.normal(0.0, rate_sigma, M))
    perm = rng.permutation(M)                 # hide the clusters from the neuron order
    P = P[perm][:, perm].tocsr()
    return P, W[perm]


def plan(P, W: np.ndarray, n_gpus: int, n_groups: int, iters: int = 4, seed: int = 0,
         balance: str = "traffic") -> dict:
    """The paper's setup end to end (Sec. IV).  Algorithm 1 maps neurons to
    GPUs.  gpu_graph() derives the GPU graph.  Algorithm 2 groups the GPUs,
    picks the bridges and builds the routing table.  Returns
    grouping.routing_report's dict plus PM (neuron -> GPU), PG, WG, the cut
    traffic of the map, and the per-GPU traffic that leaves its GPU."""
    from . import grouping
    pm = partition_neurons(P, W, n_gpus, iters, seed)
    PG, WG = gpu_graph(P, W, pm, n_gpus)
    rep = grouping.routing_report(PG, WG, n_groups, iters, seed, balance)
    rep.update(PM=pm, PG=PG, WG=WG, cut_traffic=cut_traffic(P, W, pm),
               gpu_traffic=gpu_traffic(P, W, pm, n_gpus))
    return rep


def connectivity(src: np.ndarray, tgt: np.ndarray, n_neurons: int,
                 rate: np.ndarray | float = 1.0) -> tuple[sp.csr_matrix, np.ndarray]:
    """Algorithm 1's inputs from a synapse list: P[i, j] = number of synapses
    i -> j (a connection weight; only its pattern and relative size matter to
    the greedy rule and the cut), W[i] = out-degree of i times its firing rate
    (the data volume neuron i sends)."""
    src = np.asarray(src, np.int64)
    tgt = np.asarray(tgt, np.int64)
    P = sp.csr_matrix((np.ones(len(src)), (src, tgt)), shape=(n_neurons, n_neurons))
    P.sum_duplicates()
    W = np.bincount(src, minlength=n_neurons).astype(np.float64) * rate
    return P, W


def device_map(P, W: np.ndarray, n_gpus: int, gpus_per_node: int, kind: str = "alg1",
               iters: int = 4, seed: int = 0) -> tuple[np.ndarray, dict]:
    """A neuron -> partition map for the device path, whose node n holds
    partitions [n G, (n+1) G).  The neurons are mapped to GPUs by Algorithm 1
    (kind="alg1"), by contiguous id ranges ("contiguous") or by a seeded
    random balanced assignment ("random"); the GPUs are then grouped by
    Algorithm 2 into groups of G and renumbered so that each group is one
    node (grouping.relabel).  Returns (map, info) with info holding the
    GPU-level map before renumbering, PG, WG, the groups and the cut
    traffic."""
    from . import grouping
    W = np.asarray(W, np.float64)
    M = len(W)
    G = int(gpus_per_node)
    if n_gpus % G:
        raise ValueError("the GPU count must be a multiple of the group size")
    if kind == "alg1":
        pm = partition_neurons(P, W, n_gpus, iters, seed)
    elif kind == "contiguous":
        pm = (np.arange(M) * n_gpus) // M
    elif kind == "random":
        pm = np.random.default_rng(seed).permutation(np.arange(M) % n_gpus)
    else:
        raise ValueError("kind must be 'alg1', 'contiguous' or 'random'")
    PG, WG = gpu_graph(P, W, pm, n_gpus)
    group_of = grouping.group_gpus(PG, WG, n_gpus // G, iters, seed)
    if np.any(np.bincount(group_of, minlength=n_gpus // G) != G):
        raise ValueError("Algorithm 2 did not return groups of equal size")
    new_id = grouping.relabel(group_of)
    info = dict(gpu_map=pm, PG=PG, WG=WG, group_of=group_of, new_id=new_id,
                cut_traffic=cut_traffic(P, W, pm), gpu_traffic=gpu_traffic(P, W, pm, n_gpus))
    return new_id[pm].astype(np.int32), info


def device_layout(pm: np.ndarray, group_of: np.ndarray, gpus_per_node: int) -> dict:
    """The renumbering that puts a plan on the device path's layout.  The
    device takes each partition as a contiguous range of neuron ids, and
    node n as partitions [n G, (n+1) G).  Groups must all have G members.
    Returns
      partition_id [N]    new id of each GPU: groups in order, members by old id
      neuron_id [M]       new id of each neuron: by new partition, then by old id
      starts [N + 1]      first new neuron id of each new partition
    so that neuron_id[i] lies in [starts[q], starts[q + 1]) with
    q = partition_id[pm[i]], and q div G is the group of pm[i]."""
    from . import grouping
    pm = np.asarray(pm, np.int64)
    group_of = np.asarray(group_of, np.int64)
    G = int(gpus_per_node)
    sizes = np.bincount(group_of)
    if G < 1 or np.any(sizes != G):
        raise ValueError("every group must hold exactly gpus_per_node GPUs")
    part_id = grouping.relabel(group_of)
    new_part = part_id[pm]
    order = np.lexsort((np.arange(len(pm)), new_part))
    neuron_id = np.empty(len(pm), np.int64)
    neuron_id[order] = np.arange(len(pm))
    starts = np.zeros(len(group_of) + 1, np.int64)
    starts[1:] = np.cumsum(np.bincount(new_part, minlength=len(group_of)))
    return dict(partition_id=part_id, neuron_id=neuron_id, starts=starts)
