/*
 * oracle.h — plain CPU reference of one GPU's share of a spiking-network
 * simulation step with two-level spike routing.  TEST INFRASTRUCTURE ONLY:
 * only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load it; the product path never calls it.
 *
 * What one step computes (per neuron update, fired-ID compaction, routing in
 * both forms, mask expansion, synaptic delivery) is the plain definition
 * written out, in FP64, with an extra trajectory that rounds every operation
 * to binary32 so that a binary32 device implementation can be checked
 * bit-exactly.  See oracle.c for the definitions and the passages they follow.
 */
#ifndef SNN_ORACLE_H
#define SNN_ORACLE_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  uint32_t n_neurons;
  uint32_t n_partitions;
  uint32_t gpus_per_node;   /* group (node) size, <= 64; mask bit b <-> partition G*n+b */
  uint32_t max_delay;       /* ring has max_delay + 1 slots */
  double dt_ms, tau_m_ms;
  double theta_mv;          /* threshold relative to rest */
  double u_reset_mv;        /* reset relative to rest */
  double t_ref_ms;
  double nu_ext_hz, w_ext_mv;
  uint64_t seed;
  uint32_t forced;          /* forced raster: spikes are Bernoulli draws */
  uint32_t period_steps, on_steps;
  double rate_on_hz, rate_off_hz;
  uint32_t bf16_weights;    /* binary32 trajectory uses BF16-rounded weights */
} orc_params;

enum {
  ORC_SPIKES = 0,
  ORC_LOCAL_EVENTS = 1,     /* synapses delivered inside the source's partition */
  ORC_REMOTE_EVENTS = 2,    /* synapses delivered through receive lists */
  ORC_MSG_L1 = 3,           /* two-level messages to the source's own node */
  ORC_MSG_L2 = 4,           /* two-level messages to other nodes */
  ORC_FLAT_MSGS = 5,        /* one per (spike, destination partition) */
  ORC_RECV_ENTRIES = 6,     /* expanded receive-list entries */
  ORC_NSTAT = 7
};

typedef struct orc_sim orc_sim;

/* Edge arrays are the canonical synapse list (any order); the oracle copies
   what it needs.  u0: initial state relative to rest (n_neurons). */
orc_sim* orc_create(const orc_params* p, uint64_t n_edges, const uint32_t* src,
                    const uint32_t* tgt, const uint8_t* delay,
                    const uint16_t* vp, const float* w, const int32_t* part,
                    const float* u0);
void orc_destroy(orc_sim* s);

/* One full step; returns the number of fired neurons (binary32 trajectory). */
uint32_t orc_step(orc_sim* s);
/* n steps without reporting per-step routes; per-step spike counts and
   counters are written when the pointers are non-NULL
   (counts[n], stats[n][ORC_NSTAT]). */
void orc_run(orc_sim* s, uint32_t n, uint32_t* counts, uint64_t* stats);

uint64_t orc_time(const orc_sim* s);  /* steps done so far */

/* Results of the last step. */
uint32_t orc_fired(const orc_sim* s, uint32_t* out);      /* ascending */
uint32_t orc_fired64(const orc_sim* s, uint32_t* out);    /* FP64 trajectory */
void orc_counters(const orc_sim* s, uint64_t* out);       /* ORC_NSTAT */
/* which: 0 = flat lists, 1 = expanded two-level lists; sizes[n_partitions],
   entries concatenated by partition (may be NULL to get sizes only). */
uint64_t orc_recv(const orc_sim* s, int which, uint64_t* sizes, uint32_t* entries);
/* per-node messages, two words each (source id, 64-bit mask of the node's
   destination partitions: bit b <-> partition G*n + b), concatenated by
   node; sizes[n_nodes] counts messages; returns the message total. */
uint64_t orc_buckets(const orc_sim* s, uint64_t* sizes, uint64_t* msgs);

/* Current state; any pointer may be NULL. ring: [max_delay+1][n_neurons]. */
void orc_state(const orc_sim* s, float* u, uint8_t* ref, float* ring,
               double* u64, uint8_t* ref64, double* ring64);

/* FP64-vs-binary32 accuracy so far (out[5]): out[0] = max |u32 - u64| over
   all neuron-steps (after each step's update) before the first step whose
   rasters differ, out[1] = that step (-1 if none), out[2] = number of steps
   whose rasters agree, out[3] = min |u64 - theta| over integrating
   neuron-steps, out[4] = max |u64| over integrating neuron-steps (the
   magnitude at which the update rounds). */
void orc_accuracy(const orc_sim* s, double* out);

/* Derived constants, exposed so tests can compare them with the device
   parameters: fl32(exp(-dt/tau)), the Poisson inversion table, the
   refractory length, forced-raster thresholds. */
float orc_alpha(const orc_params* p);
void orc_poisson_table(double lambda, uint32_t* thr15);
uint32_t orc_poisson_k(const uint32_t* thr15, uint32_t r);
uint32_t orc_n_ref(const orc_params* p);
uint32_t orc_raster_threshold(double rate_hz, double dt_ms);

/* Forced raster at any network size (p->forced must be set):
   orc_forced_raster writes the fired ids in [lo, hi) of step t (ascending)
   and returns their count (out may be NULL).  orc_forced_neuron runs neuron
   j alone for n_steps from state (u0, ref 0, empty ring), given its incoming
   synapses (in_src, in_delay, in_w: n_in entries), and returns its final u
   and ref, its spike count, and pending[max_delay]: the input already
   scheduled for steps n_steps .. n_steps + max_delay - 1.  Returns 0, or -1
   for a non-forced parameter set. */
uint32_t orc_forced_raster(const orc_params* p, uint64_t t, uint32_t lo, uint32_t hi,
                           uint32_t* out);
int orc_forced_neuron(const orc_params* p, uint32_t j, float u0, uint32_t n_in,
                      const uint32_t* in_src, const uint8_t* in_delay, const float* in_w,
                      uint32_t n_steps, float* u_out, uint8_t* ref_out, float* pending,
                      uint32_t* n_spikes);

/* Building blocks, exposed for pinning tests. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
float orc_bf16_round(float x);

#ifdef __cplusplus
}
#endif
#endif
