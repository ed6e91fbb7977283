/*
 * snn_setup.h — host-side setup of the arrays that snn_create consumes.
 *
 * Partition assignment and the routing table are setup steps of the paper's
 * design, run before the simulation (Algorithm 1 produces the neuron-GPU
 * mapping PM, Sec. IV-A; Algorithm 2 the routing table TB, Sec. IV-B).  Here
 * PM is given: by the seeded network description (contiguous partitions, or
 * every neuron in partition 0 for one GPU's share with virtual remote
 * partitions), or explicitly as a neuron -> partition map (for instance
 * Algorithm 1's, with partitions numbered so that Algorithm 2's groups are
 * consecutive nodes of gpus_per_node).  TB becomes each source's ascending
 * list of destination partitions, grouped into nodes of gpus_per_node.
 *
 * The setup regenerates the synapse list twice from the counter-based
 * generator (once to count out-degrees, once to place synapses), so host
 * memory holds only the output arrays plus one 16-bit partition tag per
 * synapse while rows are sorted.  Multithreaded with OpenMP; the output does
 * not depend on the thread count.
 *
 * Usage:
 *   snn_setup_create(...)               count out-degrees -> nnz
 *   snn_setup_fill_rows(...)            row_ptr, n_local, tgt_delay, weight
 *   snn_setup_sizes(...)                pairs, bucket_total, recv_total
 *   snn_setup_input_bound(...)          snn_params.input_bound
 *   snn_setup_fill_routes(...)          vp_ptr, vp_part, vp_rec, part_of_neuron,
 *                                       bucket_off, recv_off
 *   snn_setup_destroy(...)
 * All output pointers are caller-owned HOST arrays of the sizes stated.
 */
#ifndef SNN_SETUP_H
#define SNN_SETUP_H

#include <stdint.h>

#include "snn.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct snn_setup* snn_setup_handle;

/* Network description; the same fields the seeded generator takes. */
typedef struct {
  uint64_t seed;
  uint32_t n_neurons;
  uint32_t k_in;            /* incoming synapses per target */
  uint32_t max_delay;       /* delays in [1, max_delay], <= 15 */
  uint32_t n_partitions;
  uint32_t topology;        /* 0 materialised, 1 loopback, 2 loopback with per-source
                               partition sets, 3 uneven partitions, 4 clustered */
  uint32_t vp_set_size;
  double remote_frac;
  double w_exc, w_inh;      /* mV */
  double w_jitter;
  uint32_t gpus_per_node;   /* 1..64 */
  uint32_t weight_type;     /* SNN_W_FP32 or SNN_W_BF16 (round to nearest even) */
  uint32_t n_threads;       /* 0: OpenMP default */
  uint32_t verbose;         /* nonzero: progress lines on stderr during long passes */
  uint32_t n_clusters;      /* topology 4: clusters of neurons */
  double p_in;              /* topology 4: probability that an input comes from the
                               target's own cluster */
} snn_setup_spec;

/* part_start: n_partitions+1 ascending neuron offsets for topologies 0, 3 and
   4 (NULL otherwise); cross_frac: n_partitions probabilities for topology 3;
   part_map: NULL, or n_neurons partitions in [0, n_partitions) replacing the
   contiguous ranges (topologies 0 and 4; SNN_ERR_INVALID_ARG otherwise).
   Counts out-degrees (first pass over the synapses). */
snn_status snn_setup_create(const snn_setup_spec* spec, const uint32_t* part_start,
                            const double* cross_frac, const int32_t* part_map,
                            snn_setup_handle* out);

/* nnz = total synapses (known after create); pairs, bucket_total and
   recv_total are known after snn_setup_fill_rows (0 before). */
snn_status snn_setup_sizes(snn_setup_handle h, uint64_t* nnz, uint64_t* pairs,
                           uint64_t* bucket_total, uint64_t* recv_total);

/* Second pass: places every synapse in its source row and sorts each row into
   [own-partition synapses | destination partitions ascending], each part by
   (delay, target, weight).  row_ptr[N+1], n_local[N], delay_off[N][max_delay+1]
   (start of each delay's run in the own-partition part; the last entry is
   n_local, which must stay below 65536), tgt_delay[nnz], weight[nnz] (float or
   uint16 per weight_type). */
snn_status snn_setup_fill_rows(snn_setup_handle h, int64_t* row_ptr, uint32_t* n_local,
                               uint16_t* delay_off, uint32_t* tgt_delay, void* weight);

/* Largest synaptic input a neuron can receive in one step: the maximum over
   neurons of the sum of |w| (as stored, i.e. after BF16 rounding) over the
   neuron's incoming synapses; the value for snn_params.input_bound, rounded
   up to a float.  Known after snn_setup_fill_rows (SNN_ERR_BAD_STATE before). */
snn_status snn_setup_input_bound(snn_setup_handle h, float* bound);

/* Destination-partition lists, receive records and capacity bounds, from the
   rows that snn_setup_fill_rows wrote (tgt_delay and weight are its output):
   vp_ptr[N+1], vp_part[pairs], vp_rec[2 * pairs] (see snn_network_dev),
   part_of_neuron[N], bucket_off[n_nodes+1] (bucket of node n: number of
   sources with a destination partition in n), recv_off[P+1] (list of
   partition p: number of sources with destination p).  These bounds are exact
   maxima per step, so routing can never overflow.  SNN_ERR_UNSUPPORTED if a
   source has 2^24 or more synapses into one partition. */
snn_status snn_setup_fill_routes(snn_setup_handle h, const uint32_t* tgt_delay,
                                 const void* weight, int64_t* vp_ptr, uint16_t* vp_part,
                                 uint64_t* vp_rec, int32_t* part_of_neuron,
                                 uint64_t* bucket_off, uint64_t* recv_off);

void snn_setup_destroy(snn_setup_handle h);

/* Physical constants of the neuron model and its drive (the paper names only
   the model class, LIF, in Table I; the values are the workload's). */
typedef struct {
  double dt_ms;         /* step length */
  double tau_m_ms;      /* membrane time constant */
  double theta_mv;      /* threshold relative to rest */
  double u_reset_mv;    /* reset relative to rest */
  double t_ref_ms;      /* refractory period */
  double nu_ext_hz;     /* rate of the external Poisson drive per neuron */
  double w_ext_mv;      /* jump per external event */
  double rate_on_hz;    /* forced raster: rate in the on phase */
  double rate_off_hz;   /* forced raster: rate in the off phase */
} snn_model;

/* Fills the constants of snn_params that the update takes ready-made, from
   the physical ones: alpha = fl32(exp(-dt/tau_m)); theta, u_reset, w_ext as
   binary32; n_ref = dt-steps of t_ref rounded to nearest (ties to even);
   poisson_thr[j] = min(floor(2^32 CDF(j)), 2^32 - 1) for the Poisson law of
   mean nu_ext dt, j = 0..14, the CDF summed in double from exp(-lambda) by
   the recurrence pmf(j) = pmf(j-1) lambda / j; raster_thr_on/off =
   floor(2^32 rate dt) clamped to [0, 2^32 - 1].  Leaves every other field
   unchanged.  SNN_ERR_INVALID_ARG for NULL pointers, dt or tau_m not
   positive, a negative rate, t_ref or lambda, or n_ref above 255.  Host
   only; no device work. */
snn_status snn_setup_model_params(const snn_model* m, snn_params* p);

#ifdef __cplusplus
}
#endif
#endif /* SNN_SETUP_H */
