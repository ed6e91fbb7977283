/*
 * snn.h — C ABI of one GPU's share of a spiking-network simulation step with
 * two-level spike routing, for AMD Instinct MI355X (gfx950).
 *
 * The paper this follows ("A Low-latency Communication Design for Brain
 * Simulations") states the problem as: neurons are partitioned over GPUs
 * (the neuron-GPU mapping PM of Algorithm 1, Sec. IV-A); GPUs are grouped
 * (Algorithm 2, Sec. IV-B) so that traffic inside a group goes directly
 * (level 1) and traffic to another group goes once to that group, where a
 * bridge GPU forwards it (level 2); the simulation alternates computation on
 * the GPUs with this exchange (Sec. I).  The direct peer-to-peer exchange
 * it improves on (Sec. II, Table II) is kept beside it.
 *
 * On one GPU every partition and node other than the GPU's own is a virtual
 * buffer in HBM; groups are nodes of gpus_per_node (<= 64) consecutive
 * partitions, so a node's destination set is a mask of up to 64 bits.  One
 * step is three calls, always in this order (snn_step_route does the first
 * two in fewer launches, and snn_run replays whole steps):
 *
 *   snn_step     neuron update and threshold for step t, then compaction of
 *                the fired neuron IDs into an ascending list
 *   snn_route    two-level: one message (source, mask) per destination node
 *                into per-node send buckets, then expansion of each mask into
 *                per-partition receive lists (what the bridge of Sec. IV-B
 *                does); flat: one entry per (source, destination partition)
 *   snn_deliver  synaptic delivery: each fired source's own-partition
 *                synapses, and the synapses the receive lists reach, are
 *                scheduled for step t + d (d = the synapse's delay) and summed
 *                into the target's input when that step's update runs
 *
 * Scheduled input lives in per-(step mod D, tile of neurons) bins of
 * fixed-point events, with a dense fixed-point overflow ring in the
 * workspace for bins that are full; both are summed exactly.  snn_flush
 * writes the input scheduled for the coming steps into the caller's dense
 * ring ring[(max_delay+1)][n] as binary32, without changing either.
 *
 * Neuron model (the paper only names LIF as a model class, Table I):
 * current-based leaky integrate-and-fire with delta synapses, state
 * u = V - V_rest in binary32.  Per neuron i at step t, with D = max_delay + 1:
 *   syn = ring[t mod D][i]; ring[t mod D][i] = 0
 *   r   = Philox4x32-10(counter (i/4, t, 1, 0), key seed) word i mod 4
 *   k   = #{ j < 15 : poisson_thr[j] <= r };  ext = fl(k * w_ext)
 *   if ref[i] > 0: ref[i] -= 1            (input discarded, u unchanged)
 *   else:          u = fl(fl(u * alpha) + fl(syn + ext))
 *   spike = forced ? (r2 < raster threshold of step t) : (integrating && u >= theta)
 *           with r2 the Philox word on stream 2
 *   if spike: u = u_reset; ref[i] = n_ref
 * and every synapse (s -> tgt, w, d) of a fired s adds w to the input of tgt
 * at step t + d (ring slot (t+d) mod D).
 *
 * Conventions for every call:
 *  - Return value: SNN_OK or a negative snn_status; calls never abort.  The
 *    message of the last failure on the calling thread is snn_last_error().
 *  - Device pointers are caller-owned (e.g. torch tensors), borrowed for the
 *    handle's lifetime, never freed by the library.  Host pointers are only
 *    read or written during the call.
 *  - step/route/step_route/deliver/run only enqueue work on the handle's
 *    stream and never synchronise.  Device-side capacity overflow is sticky and is
 *    reported as SNN_ERR_CAPACITY by the next synchronising call
 *    (snn_read_*, snn_sync, snn_destroy); buffers are never silently
 *    truncated.
 *  - One handle per stream; a handle is not thread-safe.
 */
#ifndef SNN_H
#define SNN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct snn_ctx* snn_handle;

typedef enum {
  SNN_OK = 0,
  SNN_ERR_INVALID_ARG = -1,
  SNN_ERR_BAD_STATE = -2,   /* calls out of the step -> route -> deliver order */
  SNN_ERR_CAPACITY = -3,    /* a bucket, receive list or the spike log overflowed */
  SNN_ERR_HIP = -4,         /* a HIP runtime call failed */
  SNN_ERR_UNSUPPORTED = -5
} snn_status;

/* Routing modes (snn_route). */
enum {
  SNN_ROUTE_TWO_LEVEL = 0,  /* Sec. IV-B: per-node masked messages, then expansion */
  SNN_ROUTE_FLAT = 1,       /* direct peer-to-peer: one entry per destination partition */
  SNN_ROUTE_BOTH = 2        /* both buffers filled (for checking); delivery reads the
                               two-level receive lists */
};

/* Weight storage (snn_params.weight_type). */
enum { SNN_W_FP32 = 0, SNN_W_BF16 = 1 };

/* snn_params.flags */
enum {
  SNN_FORCED_RASTER = 1u    /* spikes are Bernoulli draws (traffic generator); the
                               membrane update still runs and fired neurons reset */
};

/* Per-step counters (snn_read_counters), in this order. */
enum {
  SNN_STAT_SPIKES = 0,
  SNN_STAT_LOCAL_EVENTS = 1,   /* synapses delivered inside the source's partition */
  SNN_STAT_REMOTE_EVENTS = 2,  /* synapses delivered through receive lists */
  SNN_STAT_MSG_L1 = 3,         /* two-level messages to the source's own node */
  SNN_STAT_MSG_L2 = 4,         /* two-level messages to other nodes */
  SNN_STAT_FLAT_MSGS = 5,      /* flat entries (one per spike and destination partition) */
  SNN_STAT_RECV_ENTRIES = 6,   /* receive-list entries produced by mask expansion */
  SNN_NSTAT = 7
};

/* Kernel kinds of a step, in launch order (snn_kernel_times).  In a whole
   two-level step as snn_run launches it, UPDATE also routes (up to 512 nodes
   of at most 8 partitions) and RECV_STAGE also expands the masks and bins
   the own-partition synapses; DELIVER bins the received ones (with
   snn_tuning.recv_merged, RECV_STAGE does that too and there is no DELIVER
   launch). */
enum {
  SNN_KERNEL_UPDATE = 0,           /* neuron update, threshold, compaction */
  SNN_KERNEL_ROUTE_TWO_LEVEL = 1,  /* per-node messages with partition masks */
  SNN_KERNEL_EXPAND = 2,           /* mask expansion into receive lists */
  SNN_KERNEL_ROUTE_FLAT = 3,       /* one entry per destination partition */
  SNN_KERNEL_RECV_STAGE = 4,       /* receive side: synapses per entry, by delay */
  SNN_KERNEL_DELIVER = 5,          /* binning of local and received synapses */
  SNN_NKERNEL = 6
};

/* Largest supported sizes. */
#define SNN_MAX_GPUS_PER_NODE 64u
#define SNN_MAX_DELAY 15u
#define SNN_MAX_NEURONS (1u << 27)    /* target ids share 32 bits with the delay; the
                                         deliver kernels' per-tile LDS counters limit a
                                         handle to about 8e7 (snn_create reports
                                         SNN_ERR_UNSUPPORTED above that) */
#define SNN_MAX_PARTITIONS 65535u

/* All by value; validated by snn_workspace_size and snn_create. */
typedef struct {
  uint32_t n_neurons;         /* neurons on this GPU (all materialised partitions) */
  uint32_t n_partitions;      /* partitions (GPUs), real and virtual */
  uint32_t gpus_per_node;     /* group size G, 1..64: mask bit b <-> partition G*n + b */
  uint32_t max_delay;         /* synaptic delays in [1, max_delay], max_delay <= 15 */
  float alpha;                /* membrane decay per step, fl32(exp(-dt/tau_m)) */
  float theta;                /* threshold relative to rest (mV) */
  float u_reset;              /* reset relative to rest (mV) */
  float w_ext;                /* jump per external Poisson event (mV) */
  uint32_t n_ref;             /* refractory steps, <= 255 */
  uint32_t poisson_thr[15];   /* floor(2^32 * CDF_lambda(j)), j = 0..14, nondecreasing */
  uint64_t seed;              /* Philox key */
  uint32_t weight_type;       /* SNN_W_FP32 or SNN_W_BF16 */
  uint32_t flags;             /* SNN_FORCED_RASTER */
  uint32_t raster_thr_on;     /* forced raster: spike iff r2 < thr; thr_on during the first */
  uint32_t raster_thr_off;    /*   raster_on steps of every raster_period steps, */
  uint32_t raster_period;     /*   thr_off otherwise (period >= 1) */
  uint32_t raster_on;
  uint64_t bucket_total;      /* total per-node bucket capacity (messages) */
  uint64_t recv_total;        /* total per-partition receive-list capacity (entries) */
  uint32_t log_steps;         /* steps kept for snn_read_spikes / snn_read_counters (>= 1);
                                 older steps are overwritten */
  float input_bound;          /* largest synaptic input a neuron can get in one step (mV):
                                 max over neurons of the sum of |w| over its incoming
                                 synapses (snn_setup_input_bound computes it); > 0.  The
                                 input of a step is summed exactly in fixed point with
                                 F = floor(log2(2^30 / input_bound)) fractional bits
                                 (8 <= F <= 30 required) after rounding each weight to
                                 a multiple of 2^-F, then rounded once to binary32;
                                 sums of weights that are multiples of 2^-F (the dyadic
                                 weights of the parity tests) are exact */
  uint64_t log_cap;           /* spike-log capacity in neuron ids */
  uint64_t bin_cap;           /* events per delivery bin: one bin per (ring slot, tile of
                                 neurons, delay, delivery block), see snn_bin_geometry;
                                 events beyond it take the (slower) dense-ring path */
  uint64_t stage_cap;         /* remote events per (delay, receive-side block) and step,
                                 see snn_bin_geometry; beyond it, the dense-ring path */
  uint32_t tile_neurons;      /* neurons per tile (the update's block and the bins' unit):
                                 0 for the default, 8192, or where that gives fewer than
                                 512 tiles (two update blocks per CU of a 256-CU part) the
                                 neurons spread over 512 tiles, rounded up to a multiple of
                                 64, at least 2048; else a multiple of 64 in [64, 8192] */
} snn_params;

/* Network arrays in device memory.  nnz = row_ptr[n_neurons]; pairs =
   vp_ptr[n_neurons]; n_nodes = ceil(n_partitions / gpus_per_node). */
typedef struct {
  const int64_t* row_ptr;          /* [N+1] out-synapses of source s: [row_ptr[s], row_ptr[s+1]) */
  const uint32_t* n_local;         /* [N] the first n_local[s] synapses of the row stay in
                                      the source's own partition, sorted by delay */
  const uint16_t* delay_off;       /* [N][max_delay+1] delay_off[s][d-1] = first synapse
                                      (relative to row_ptr[s]) of delay d in the local part;
                                      delay_off[s][max_delay] = n_local[s] (< 65536) */
  const uint32_t* tgt_delay;       /* [nnz] (delay << 27) | target neuron */
  const void* weight;              /* [nnz] float (SNN_W_FP32) or bfloat16 bits (SNN_W_BF16) */
  const int64_t* vp_ptr;           /* [N+1] destination partitions of s:
                                      vp_part[vp_ptr[s] .. vp_ptr[s+1]) */
  const uint16_t* vp_part;         /* [pairs] distinct, ascending, never s's own partition;
                                      this is the routing table TB of Sec. IV-B restricted
                                      to one source */
  const uint64_t* vp_rec;          /* [2 * pairs] receive record of pair j (source s, its
                                      destination vp_part[j]), what the receiving partition
                                      needs to find its synapses of s:
                                        vp_rec[2j]   = start | (len << 40): the row segment
                                                       [start, start + len) (absolute synapse
                                                       indices, len >= 1) going to vp_part[j];
                                                       segments follow the local part in vp
                                                       order
                                        vp_rec[2j+1] = tgt_delay | (weight bits << 32) of the
                                                       segment's first synapse (a copy, so
                                                       that one-synapse segments need no
                                                       second lookup) */
  const int32_t* part_of_neuron;   /* [N] the neuron-GPU mapping PM of Sec. IV-A */
  const uint64_t* bucket_off;      /* [n_nodes+1] bucket of node n holds at most
                                      bucket_off[n+1] - bucket_off[n] messages */
  const uint64_t* recv_off;        /* [P+1] receive list of partition p holds at most
                                      recv_off[p+1] - recv_off[p] entries */
  float* u;                        /* [N] membrane state, relative to rest (read/write) */
  uint8_t* ref;                    /* [N] refractory steps left (read/write) */
  float* ring;                     /* [(max_delay+1) * ring_stride] slot-major read-back of
                                      the scheduled input, ring_stride = snn_ring_stride(N):
                                      written by snn_flush only */
} snn_network_dev;

/* Slot stride of the delay ring: n_neurons rounded up to a multiple of 256. */
uint64_t snn_ring_stride(uint32_t n_neurons);

/* Device workspace the caller must provide to snn_create (bytes, 256-byte
   aligned base).  Depends on n_neurons, n_partitions, gpus_per_node,
   bucket_total, recv_total, log_steps and log_cap. */
snn_status snn_workspace_size(const snn_params* params, size_t* bytes);

/* One GPU's share of the network after the model has been generated and
   dispersed over the GPUs (the two set-up stages of Sec. I, Fig. 1), with
   the neuron-GPU mapping of Sec. IV-A fixing which partition each neuron and
   each synapse's target belongs to.
   Validates params and array pointers, carves the workspace, zeroes its
   counters on `stream` and returns a handle at step t = 0.  `stream` is a
   hipStream_t (NULL = the default stream).  Does not allocate device
   memory. */
snn_status snn_create(const snn_params* params, const snn_network_dev* net,
                      void* workspace, size_t workspace_bytes, void* stream,
                      snn_handle* out);

/* Size of the library's static device scratch used by snn_create_static. */
#define SNN_STATIC_SCRATCH_BYTES (32u << 20)

/* For callers that cannot allocate (code under HIP graph capture, tight
   serving loops, harnesses that forbid allocation): snn_create without the
   workspace argument.  The handle's workspace is the library's static device
   array of SNN_STATIC_SCRATCH_BYTES (one per device, held until the process
   ends) and the handle itself lives in static host storage, so the call
   allocates nothing, host or device; its set-up (clearing the counters,
   building the Poisson lookup) runs as kernels on `stream`.  Networks whose
   workspace (snn_workspace_size) exceeds SNN_STATIC_SCRATCH_BYTES (a few
   thousand neurons at the workloads' shapes) are rejected with
   SNN_ERR_UNSUPPORTED.
   Every call on a device shares that device's scratch and static handle: a
   call replaces the previous static handle of the device (which must no
   longer be used) and its state; calls and steps that overlap on one device
   race.  All other calls take the handle as usual, except that snn_run
   rejects use_graph != 0 (instantiating a graph allocates); snn_destroy
   only synchronises (so destroying a replaced handle is harmless).  Not
   thread-safe. */
snn_status snn_create_static(const snn_params* params, const snn_network_dev* net, void* stream,
                             snn_handle* out);

/* The computation half of a simulation step (Sec. I: data processing on the
   GPUs; the LIF model class of Table I): neuron update, threshold and
   ascending compaction of fired ids for the current step t (ring slot t mod D
   is read and cleared).  Order: must follow
   snn_create or snn_deliver. */
snn_status snn_step(snn_handle h);

/* Routes the spikes of the current step (mode SNN_ROUTE_*): the two-level
   messages of Sec. IV-B (one per destination group, Fig. 2(b)), the direct
   per-destination messages of Fig. 2(a), or both.  Order: must
   follow snn_step. */
snn_status snn_route(snn_handle h, int mode);

/* snn_step followed by snn_route(mode), in fewer launches: for the two-level
   modes the update kernel routes each tile's fired neurons itself (Sec. IV-B
   messages into the node buckets) while it waits for the spike-count prefix
   of the tiles before it; with more than 512 nodes the two calls are made
   as they are.  The buckets hold the same messages as after snn_route (their
   order within a bucket may differ); the mask expansion into the receive
   lists is left to snn_deliver, which expands and stages in one kernel.
   Order: as snn_step; snn_deliver follows. */
snn_status snn_step_route(snn_handle h, int mode);

/* The receiving half of the exchange (Sec. I: data exchange among GPUs; Sec.
   IV-B: a group's messages reach each destination GPU of the group, whose
   synapses of the source then take the spike): delivers the current step's
   synaptic events (own partition and receive lists); each is scheduled for step t + d in its tile's bin (or the ring
   slot (t + d) mod D when the bin is full).  Order: must follow snn_route. */
snn_status snn_deliver(snn_handle h);

/* n_steps full steps (snn_step_route(mode), snn_deliver).  use_graph = 0
   launches them directly; 1 captures HIP graphs of 16 steps and of one step
   once per mode and replays them (16-step replays first, then single steps
   for the remainder); 2 captures all n_steps steps as one graph (kept for
   the next call with the same n_steps and mode) and launches it once.  All
   step-dependent values live in device memory, so a graph replays unchanged.
   Order: as snn_step. */
snn_status snn_run(snn_handle h, uint32_t n_steps, int mode, int use_graph);

/* snn_run with the neuron update (and the two-level routing done inside it)
   launched once per partition, over that partition's neurons only, instead
   of once over all of them: the layout of one launch per partition that a
   batched kernel replaces (the uneven partitions of Sec. V's workload, each
   of which would be one GPU's share).  Partitions must be contiguous ranges
   of neuron ids: partition p holds [part_start[p], part_start[p+1]) (host
   array of n_partitions + 1 entries, part_start[0] = 0,
   part_start[n_partitions] = n_neurons; empty partitions are skipped).
   Results are identical to snn_run's.  Not for snn_create_static handles. */
snn_status snn_run_partitioned(snn_handle h, uint32_t n_steps, int mode, int use_graph,
                               const uint32_t* part_start);

/* Launch-shape choices that leave every result unchanged; the library's
   defaults are update_blocks = 0, recv_split = 0 and recv_merged = 1.
   Picked per network shape by measurement (the package's autotuner). */
typedef struct {
  uint32_t update_blocks;   /* blocks of a whole-step update launch: 0 = one per tile of
                               neurons; fewer = persistent blocks that take tiles in turn */
  uint32_t recv_split;      /* most receive-side blocks that share one destination node's
                               messages (expansion and staging); 0 = as many as the
                               256 receive-side blocks allow, 1 = one block per node */
  uint32_t recv_merged;     /* 0: the receive side of a whole step is two launches
                               (expansion and staging beside the own-partition delivery,
                               then the received synapses); 1 (the default): one launch, whose
                               delivery blocks wait for its staging blocks and read
                               their queues through the L2 of the XCD they share
                               (workgroups are dealt out to the XCDs in turn); where a
                               queue turns out to have been staged on another XCD, the
                               next synchronising call reports SNN_ERR_UNSUPPORTED.
                               Its hand-off tags steps modulo 2^28; a step a nonzero
                               multiple of 2^28 steps after the last one-launch step
                               takes the two-launch form (the runtime sees to it) */
} snn_tuning;

/* Sets / reads the handle's launch shapes.  Setting synchronises the stream
   and drops the handle's captured graphs.  Order: between steps. */
snn_status snn_set_tuning(snn_handle h, const snn_tuning* t);
snn_status snn_get_tuning(snn_handle h, snn_tuning* t);

/* Writes the input scheduled for each of the coming steps into `ring`: for
   slot s and neuron i, the sum of the pending events for i at the step that
   consumes slot s, rounded to binary32 exactly as the update will round it
   (their fixed-point sum, see input_bound).  Reads only: the bins, the
   overflow ring and every later step are unchanged, whatever the weights.
   Order: between steps. */
snn_status snn_flush(snn_handle h);

/* Blocks until the handle's work is done; reports sticky device errors. */
snn_status snn_sync(snn_handle h);

/* Events that took the dense-ring path so far (a bin or a staging queue was
   full).  Synchronises. */
snn_status snn_ring_events(snn_handle h, uint64_t* n);

/* Measurement aid: runs n_steps ordinary whole steps (route mode `mode`, as
   snn_run launches them) as separate launches, each kernel bracketed by HIP
   events recorded on the handle's stream, and writes the average duration in
   milliseconds of each kernel kind to avg_ms[SNN_NKERNEL] (0 for kinds the
   mode does not launch; two-level routing done inside the update kernel
   counts as update).
   The steps advance the simulation like snn_run.  Synchronises.  Order: as
   snn_step. */
snn_status snn_kernel_times(snn_handle h, uint32_t n_steps, int mode, float* avg_ms);

/* Geometry of the binned delivery for a network of params->n_neurons neurons
   and the requested params->tile_neurons (the only fields read), for sizing
   snn_params.bin_cap and stage_cap: *tile_neurons neurons share a bin (the
   tile size the library will use); each (step slot, tile, delay) has
   *deliver_blocks sub-bins (one per writing block), each of bin_cap events;
   each delay has *stage_blocks receive queues of stage_cap events.  Any
   output pointer may be NULL.  SNN_ERR_INVALID_ARG for an invalid tile size
   or neuron count. */
snn_status snn_bin_geometry(const snn_params* params, uint32_t* tile_neurons,
                            uint32_t* deliver_blocks, uint32_t* stage_blocks);

/* Steps completed so far (host-side count of enqueued steps). */
uint64_t snn_time(snn_handle h);

/* The spikes each step exchanges (Sec. I), whose counts per destination
   make up the per-GPU traffic of Fig. 3(a) (Sec. V).
   Fired ids of steps [first_step, first_step + n_steps), which must be among
   the last log_steps steps; ids ascending within a step, concatenated.
   per_step_counts[n_steps] (may be NULL); ids may be NULL to query *n_ids.
   Fails with SNN_ERR_CAPACITY if more than cap ids or if the spike log
   overflowed for a requested step.  Synchronises. */
snn_status snn_read_spikes(snn_handle h, uint64_t first_step, uint32_t n_steps,
                           int32_t* ids, uint64_t cap, uint32_t* per_step_counts,
                           uint64_t* n_ids);

/* Routing buffers of the last routed step, copied to host memory, as uint64
   elements.
   which = 0: flat receive lists, per partition: bits 0..26 source id, bits
              27..63 pair index j of (source, partition) (vp_part[j] is the
              partition; vp_rec[2j], vp_rec[2j+1] the record the receiver uses to
              find its synapses);
   which = 1: expanded two-level receive lists, same format;
   which = 2: per-node send buckets, TWO uint64 per message: bits 0..31 source
              id and bits 32..63 the pair index of the node's first destination
              (its followers in the node are the next pairs), then the mask of
              the node's destination partitions (bit b <-> partition G*n + b).
   sizes[n_partitions or n_nodes] receives the counts (messages for which = 2);
   entries (may be NULL) receives the lists concatenated in partition / node
   order, at most cap lists entries (cap counts messages for which = 2, each
   16 bytes).  Order inside a list is unspecified.  Synchronises. */
snn_status snn_read_routes(snn_handle h, int which, uint64_t* sizes, void* entries,
                           uint64_t cap, uint64_t* n_entries);

/* Per-step counts behind Sec. V's comparisons (spikes, events, level-1 and
   level-2 messages against the direct messages of Fig. 4's two routings):
   counters of steps [first_step, first_step + n_steps) (the last log_steps
   steps), out[n_steps][SNN_NSTAT].  Synchronises. */
snn_status snn_read_counters(snn_handle h, uint64_t first_step, uint32_t n_steps,
                             uint64_t* out);

/* Releases the handle (NULL is a no-op).  Synchronises first. */
snn_status snn_destroy(snn_handle h);

/* Message of the last failed call on this thread ("" if none). */
const char* snn_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SNN_H */
