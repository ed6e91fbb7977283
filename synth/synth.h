/*
 * synth.h — seeded synthetic network generator.
 *
 * This module produces the INPUTS of a simulation step: the synapse list of a
 * spiking network (source, delay, destination partition, weight per synapse),
 * the neuron->partition map and the initial membrane state.  It holds none of
 * the method's arithmetic (no membrane update, no routing, no delivery).  Both
 * the CPU oracle and the GPU path's host setup call it, so the two sides see
 * the identical network without sharing any other code.
 *
 * The paper (Sec. V) runs a non-public model built from a scanned human brain;
 * these seeded random networks stand in for it at the per-GPU shapes the paper
 * implies (10 billion neurons over 2,000 GPUs, about 1,000 synapses per neuron
 * from the synapse count quoted in Sec. I).
 *
 * Every random draw is a pure function of (seed, stream, a, b) through the
 * SplitMix64 output mixer (Steele, Lea, Flood, "Fast splittable pseudorandom
 * number generators", OOPSLA 2014), so results do not depend on thread count.
 *
 * Synapse (tgt, k), k in [0, k_in), is the k-th incoming synapse of target tgt
 * ("fixed in-degree").  Its fields:
 *   src   source neuron, uniform over the allowed set, never tgt (no autapses;
 *         repeated pairs are allowed)
 *   delay integer steps, uniform in [1, max_delay]
 *   vp    destination partition the spike must reach: for a target on this
 *         GPU's own partitions vp = part_of(tgt); in the loopback topologies a
 *         remote synapse is tagged with a virtual partition vp != 0
 *   w     weight in mV by source type: inhibitory iff src % 5 == 4 (80/20
 *         interleaved), optionally jittered per synapse
 */
#ifndef SYNTH_H
#define SYNTH_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

enum {
  /* all partitions live on this GPU; vp = part_of(tgt); sources uniform */
  SYN_TOPO_MATERIALIZED = 0,
  /* one GPU's share: all neurons in partition 0; each synapse is remote with
     probability remote_frac and then tagged vp uniform in [1, P-1] */
  SYN_TOPO_LOOPBACK = 1,
  /* as LOOPBACK, but each source owns a fixed set of vp_set_size distinct
     virtual partitions and a remote synapse draws its vp from that set */
  SYN_TOPO_LOOPBACK_SETS = 2,
  /* partitions of uneven size, all on this GPU; a target in partition q draws
     a source outside q with probability cross_frac[q] (size-weighted, i.e.
     uniform over neurons outside q), else uniform inside q; vp = q */
  SYN_TOPO_BATCHED = 3,
  /* all partitions on this GPU, neurons in n_clusters clusters (each neuron's
     cluster drawn uniformly, so clusters are scattered over the ids); a target
     draws its source inside its own cluster with probability p_in, else
     uniform over all neurons; vp = part_of(tgt).  Connectivity with locality
     for a partitioning to find (Algorithm 1) */
  SYN_TOPO_CLUSTERED = 4
};

typedef struct {
  uint64_t seed;
  uint32_t n_neurons;
  uint32_t k_in;          /* incoming synapses per target */
  uint32_t max_delay;     /* delays uniform in [1, max_delay] */
  uint32_t n_partitions;
  uint32_t topology;      /* SYN_TOPO_* */
  uint32_t vp_set_size;   /* SYN_TOPO_LOOPBACK_SETS only */
  double remote_frac;     /* SYN_TOPO_LOOPBACK[_SETS] only */
  double w_exc, w_inh;    /* mV */
  double w_jitter;        /* 0: none; else w *= 1 + w_jitter * (U[0,1) - 1/2) */
  uint32_t n_clusters;    /* SYN_TOPO_CLUSTERED only */
  double p_in;            /* SYN_TOPO_CLUSTERED only */
} syn_spec;

typedef struct syn_gen syn_gen;

/* part_start: n_partitions+1 ascending neuron offsets (MATERIALIZED, BATCHED,
   CLUSTERED); ignored (may be NULL) for the loopback topologies, where every
   neuron is in partition 0.  cross_frac: n_partitions probabilities (BATCHED
   only).  Returns NULL on invalid input. */
syn_gen* syn_create(const syn_spec* spec, const uint32_t* part_start,
                    const double* cross_frac);
/* An explicit neuron -> partition map (n_neurons entries in [0, n_partitions))
   replacing the contiguous ranges of part_start: part_of() and the vp of
   every synapse follow it (MATERIALIZED and CLUSTERED only).  Returns 0, or
   -1 if the topology takes no map or an entry is out of range. */
int syn_set_part_map(syn_gen* g, const int32_t* part);
/* Cluster of a neuron (CLUSTERED; 0 otherwise). */
uint32_t syn_cluster_of(const syn_gen* g, uint32_t neuron);
void syn_destroy(syn_gen* g);

/* One synapse, pure function of (spec, tgt, k). */
void syn_edge(const syn_gen* g, uint32_t tgt, uint32_t k, uint32_t* src,
              uint32_t* delay, uint32_t* vp, float* w);

/* All synapses of targets [tgt_lo, tgt_hi) in canonical order (tgt-major,
   then k); each output array holds (tgt_hi - tgt_lo) * k_in entries.  Any
   output pointer may be NULL.  Multithreaded, deterministic. */
void syn_edges(const syn_gen* g, uint32_t tgt_lo, uint32_t tgt_hi,
               uint32_t* src, uint32_t* tgt, uint8_t* delay, uint16_t* vp,
               float* w);

uint32_t syn_part_of(const syn_gen* g, uint32_t neuron);
void syn_part_map(const syn_gen* g, int32_t* part);  /* n_neurons entries */

/* Initial membrane state, relative to rest: uniform on [0, theta). */
void syn_initial_u(uint64_t seed, double theta, uint32_t n, float* u);

/* Partition sizes lognormal(median, sigma_ln) clipped to [lo, hi]. */
void syn_lognormal_sizes(uint64_t seed, uint32_t n_part, double median,
                         double sigma_ln, uint32_t lo, uint32_t hi,
                         uint32_t* sizes);
/* n values uniform on [lo, hi). */
void syn_uniform_doubles(uint64_t seed, uint32_t stream, uint32_t n, double lo,
                         double hi, double* out);

/* The per-source vp set of SYN_TOPO_LOOPBACK_SETS (vp_set_size entries,
   ascending); returns 0 if the topology has no sets. */
int syn_vp_set(const syn_gen* g, uint32_t src, uint16_t* out);

/* The raw mixer, exposed for tests of the generator itself. */
uint64_t syn_hash(uint64_t seed, uint64_t stream, uint64_t a, uint64_t b);

#ifdef __cplusplus
}
#endif
#endif
