/*
 * oracle.c — plain, slow, obviously correct CPU reference.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this file's library.  It shares no code
 * with the GPU path; the only common input is the seeded network generator.
 *
 * What a step computes, in the order written below:
 *
 *  1. Neuron update for every neuron in index order (current-based leaky
 *     integrate-and-fire with delta synapses; the paper only names LIF as a
 *     model class, Table I, so the model is the reading recorded with the
 *     design).  Input arriving at step t is the ring slot t mod D, which is
 *     read and cleared; the external drive is k Poisson events of w_ext with
 *     k drawn by inversion from one Philox-4x32-10 word.  Refractory neurons
 *     count down and ignore input.  Fired neurons are collected in ascending
 *     order (the compaction).
 *  2. Routing of every fired source s (Sec. IV-B).  VP(s) is the set of
 *     destination partitions of s's synapses other than its own partition.
 *     Flat form (the direct peer-to-peer baseline of Sec. II and Table II):
 *     one entry per (s, p), p in VP(s).  Two-level form: partitions are
 *     grouped into nodes of G (a group of GPUs behind one switch, Sec. IV-B);
 *     one message per (s, node n) carrying the mask of destination partitions
 *     of s inside n; traffic to the source's own node is level 1, to other
 *     nodes level 2 (sent once to the node and forwarded there by a bridge).
 *     Expansion: each message's mask bits become entries of the receive list
 *     of partition G*n + b.
 *  3. Delivery: every synapse (s -> tgt, w, d) of every fired s adds w to ring
 *     slot (t + d) mod D at tgt.  The oracle delivers from the synapse list
 *     directly, not through its receive lists, so a routing mistake on the
 *     device shows up as a ring difference.
 *
 * Two trajectories are carried.  The binary32 trajectory rounds every
 * operation to IEEE binary32 (computed in double, then rounded: exact double
 * rounding for +, -, * since 53 >= 2*24 + 2); routes and counters come from
 * it.  The FP64 trajectory uses the same alpha, k and weights in double and
 * is used to report accuracy.
 *
 * Compile without -ffast-math and with -ffp-contract=off.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

enum { STREAM_POISSON = 1, STREAM_RASTER = 2 };

struct orc_sim {
  orc_params p;
  uint32_t N, P, G, D, n_nodes;
  float alpha, theta, u_reset, w_ext;
  uint32_t n_ref;
  uint32_t poisson[15];
  uint32_t thr_on, thr_off;
  /* synapses grouped by source: adj[adj_ptr[s] .. adj_ptr[s+1]) */
  uint64_t* adj_ptr;
  uint32_t* e_tgt;
  uint8_t* e_delay;
  uint16_t* e_vp;
  float* e_w32;       /* weight used by the binary32 trajectory */
  double* e_w64;      /* weight used by the FP64 trajectory */
  int32_t* part;
  /* binary32 trajectory */
  float* u;
  uint8_t* ref;
  float* ring;
  /* FP64 trajectory */
  double* u64;
  uint8_t* ref64;
  double* ring64;
  uint64_t t;
  /* last step */
  uint32_t* fired;
  uint32_t n_fired;
  uint32_t* fired64;
  uint32_t n_fired64;
  uint64_t stats[ORC_NSTAT];
  /* routes of the last step: per-partition / per-node growable lists (a
     node's bucket holds (source, mask) as two words per message) */
  uint32_t** flat;
  uint64_t* flat_n;
  uint64_t* flat_cap;
  uint32_t** xrecv;
  uint64_t* xrecv_n;
  uint64_t* xrecv_cap;
  uint64_t** bucket;
  uint64_t* bucket_n;
  uint64_t* bucket_cap;
  /* scratch */
  uint64_t* seen;    /* per partition: stamp of the source that last marked it */
  uint64_t stamp;
  uint32_t* vps;     /* distinct vps of one source */
  uint64_t* node_mask;
  /* accuracy */
  double max_dv;
  int64_t first_div;
  uint64_t agree_steps;
  double min_margin;
  double max_abs_u;
};

/* ---- Philox-4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers:
   as easy as 1, 2, 3", SC'11).  Ten rounds of the Philox S-box over a
   4 x 32-bit counter with a 2 x 32-bit key bumped by Weyl constants. ---- */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    uint64_t p0 = (uint64_t)M0 * x0;
    uint64_t p1 = (uint64_t)M1 * x2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t y0 = hi1 ^ x1 ^ k0;
    uint32_t y1 = lo1;
    uint32_t y2 = hi0 ^ x3 ^ k1;
    uint32_t y3 = lo0;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    k0 += W0;
    k1 += W1;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* The 32-bit random word of neuron i at step t on a stream: counter
   (i / 4, t, stream, 0), key = seed, word i mod 4. */
static uint32_t draw(uint64_t seed, uint32_t i, uint64_t t, uint32_t stream) {
  uint32_t ctr[4] = {i / 4, (uint32_t)t, stream, 0};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t out[4];
  orc_philox4x32_10(ctr, key, out);
  return out[i % 4];
}

/* Poisson inversion table: thr[j] = floor(2^32 * CDF(j)) for j = 0..14,
   capped at 2^32 - 1; k = number of thr[j] <= r for a uniform 32-bit r. */
void orc_poisson_table(double lambda, uint32_t* thr) {
  double pmf = exp(-lambda), cdf = 0.0;
  for (int j = 0; j < 15; ++j) {
    if (j > 0) pmf = pmf * lambda / j;
    cdf += pmf;
    double v = floor(ldexp(cdf, 32));
    thr[j] = v >= 4294967295.0 ? 4294967295u : (uint32_t)v;
  }
}

uint32_t orc_poisson_k(const uint32_t* thr, uint32_t r) {
  uint32_t k = 0;
  for (int j = 0; j < 15; ++j)
    if (thr[j] <= r) k++;
  return k;
}

float orc_alpha(const orc_params* p) { return (float)exp(-p->dt_ms / p->tau_m_ms); }

uint32_t orc_n_ref(const orc_params* p) {
  return (uint32_t)llround(p->t_ref_ms / p->dt_ms);
}

/* Bernoulli threshold of a forced raster: spike iff r < rate * dt * 2^32. */
uint32_t orc_raster_threshold(double rate_hz, double dt_ms) {
  double v = floor(ldexp(rate_hz * dt_ms * 1e-3, 32));
  if (v <= 0.0) return 0;
  return v >= 4294967295.0 ? 4294967295u : (uint32_t)v;
}

/* Round a binary32 value to the nearest BF16 (8-bit significand), ties to
   even, by comparing the two neighbouring BF16 values in double.  Past the
   largest finite BF16 the upper neighbour is taken as 2^128, so overflow
   rounds to infinity exactly when IEEE round-to-nearest-even would. */
float orc_bf16_round(float x) {
  if (isnan(x) || isinf(x) || x == 0.0f) return x;
  uint32_t b;
  memcpy(&b, &x, 4);
  uint32_t lo_b = b & 0xFFFF0000u;          /* truncation toward zero */
  uint32_t hi_b = lo_b + 0x00010000u;       /* next BF16 away from zero */
  float lo, hi;
  memcpy(&lo, &lo_b, 4);
  memcpy(&hi, &hi_b, 4);
  double hi_d = isinf(hi) ? copysign(ldexp(1.0, 128), (double)x) : (double)hi;
  double dlo = fabs((double)x - (double)lo);
  double dhi = fabs(hi_d - (double)x);
  if (dlo < dhi) return lo;
  if (dhi < dlo) return hi;
  return ((lo_b >> 16) & 1) == 0 ? lo : hi;
}

static float f32(double x) { return (float)x; }

static void* xcalloc(size_t n, size_t sz) {
  void* q = calloc(n ? n : 1, sz);
  if (!q) abort();
  return q;
}

orc_sim* orc_create(const orc_params* p, uint64_t M, const uint32_t* src,
                    const uint32_t* tgt, const uint8_t* delay,
                    const uint16_t* vp, const float* w, const int32_t* part,
                    const float* u0) {
  if (!p || p->n_neurons == 0 || p->gpus_per_node == 0 || p->gpus_per_node > 64 ||
      p->n_partitions == 0 || p->max_delay == 0)
    return NULL;
  orc_sim* s = (orc_sim*)xcalloc(1, sizeof(orc_sim));
  s->p = *p;
  s->N = p->n_neurons;
  s->P = p->n_partitions;
  s->G = p->gpus_per_node;
  s->D = p->max_delay + 1;
  s->n_nodes = (s->P + s->G - 1) / s->G;
  s->alpha = orc_alpha(p);
  s->theta = f32(p->theta_mv);
  s->u_reset = f32(p->u_reset_mv);
  s->w_ext = f32(p->w_ext_mv);
  s->n_ref = orc_n_ref(p);
  orc_poisson_table(p->nu_ext_hz * p->dt_ms * 1e-3, s->poisson);
  s->thr_on = orc_raster_threshold(p->rate_on_hz, p->dt_ms);
  s->thr_off = orc_raster_threshold(p->rate_off_hz, p->dt_ms);

  const uint32_t N = s->N;
  /* group synapses by source (counting sort; order within a source is the
     input order) */
  s->adj_ptr = (uint64_t*)xcalloc(N + 1, sizeof(uint64_t));
  for (uint64_t e = 0; e < M; ++e) {
    if (src[e] >= N || tgt[e] >= N || delay[e] < 1 || delay[e] > p->max_delay ||
        vp[e] >= s->P) {
      free(s->adj_ptr);
      free(s);
      return NULL;
    }
    s->adj_ptr[src[e] + 1]++;
  }
  for (uint32_t i = 0; i < N; ++i) s->adj_ptr[i + 1] += s->adj_ptr[i];
  uint64_t* fill = (uint64_t*)xcalloc(N, sizeof(uint64_t));
  s->e_tgt = (uint32_t*)xcalloc(M, sizeof(uint32_t));
  s->e_delay = (uint8_t*)xcalloc(M, 1);
  s->e_vp = (uint16_t*)xcalloc(M, sizeof(uint16_t));
  s->e_w32 = (float*)xcalloc(M, sizeof(float));
  s->e_w64 = (double*)xcalloc(M, sizeof(double));
  for (uint64_t e = 0; e < M; ++e) {
    uint64_t at = s->adj_ptr[src[e]] + fill[src[e]]++;
    s->e_tgt[at] = tgt[e];
    s->e_delay[at] = delay[e];
    s->e_vp[at] = vp[e];
    s->e_w32[at] = p->bf16_weights ? orc_bf16_round(w[e]) : w[e];
    s->e_w64[at] = (double)w[e];
  }
  free(fill);

  s->part = (int32_t*)xcalloc(N, sizeof(int32_t));
  memcpy(s->part, part, sizeof(int32_t) * N);
  s->u = (float*)xcalloc(N, sizeof(float));
  s->ref = (uint8_t*)xcalloc(N, 1);
  s->ring = (float*)xcalloc((size_t)s->D * N, sizeof(float));
  s->u64 = (double*)xcalloc(N, sizeof(double));
  s->ref64 = (uint8_t*)xcalloc(N, 1);
  s->ring64 = (double*)xcalloc((size_t)s->D * N, sizeof(double));
  for (uint32_t i = 0; i < N; ++i) {
    s->u[i] = u0[i];
    s->u64[i] = (double)u0[i];
  }
  s->fired = (uint32_t*)xcalloc(N, sizeof(uint32_t));
  s->fired64 = (uint32_t*)xcalloc(N, sizeof(uint32_t));

  s->flat = (uint32_t**)xcalloc(s->P, sizeof(uint32_t*));
  s->flat_n = (uint64_t*)xcalloc(s->P, sizeof(uint64_t));
  s->flat_cap = (uint64_t*)xcalloc(s->P, sizeof(uint64_t));
  s->xrecv = (uint32_t**)xcalloc(s->P, sizeof(uint32_t*));
  s->xrecv_n = (uint64_t*)xcalloc(s->P, sizeof(uint64_t));
  s->xrecv_cap = (uint64_t*)xcalloc(s->P, sizeof(uint64_t));
  s->bucket = (uint64_t**)xcalloc(s->n_nodes, sizeof(uint64_t*));
  s->bucket_n = (uint64_t*)xcalloc(s->n_nodes, sizeof(uint64_t));
  s->bucket_cap = (uint64_t*)xcalloc(s->n_nodes, sizeof(uint64_t));
  s->seen = (uint64_t*)xcalloc(s->P, sizeof(uint64_t));
  s->vps = (uint32_t*)xcalloc(s->P, sizeof(uint32_t));
  s->node_mask = (uint64_t*)xcalloc(s->n_nodes, sizeof(uint64_t));
  s->first_div = -1;
  s->min_margin = INFINITY;
  return s;
}

void orc_destroy(orc_sim* s) {
  if (!s) return;
  for (uint32_t p = 0; p < s->P; ++p) { free(s->flat[p]); free(s->xrecv[p]); }
  for (uint32_t n = 0; n < s->n_nodes; ++n) free(s->bucket[n]);
  free(s->flat); free(s->flat_n); free(s->flat_cap);
  free(s->xrecv); free(s->xrecv_n); free(s->xrecv_cap);
  free(s->bucket); free(s->bucket_n); free(s->bucket_cap);
  free(s->seen); free(s->vps); free(s->node_mask);
  free(s->adj_ptr); free(s->e_tgt); free(s->e_delay); free(s->e_vp);
  free(s->e_w32); free(s->e_w64); free(s->part);
  free(s->u); free(s->ref); free(s->ring);
  free(s->u64); free(s->ref64); free(s->ring64);
  free(s->fired); free(s->fired64);
  free(s);
}

static void push32(uint32_t** v, uint64_t* n, uint64_t* cap, uint32_t x) {
  if (*n == *cap) {
    *cap = *cap ? 2 * *cap : 16;
    *v = (uint32_t*)realloc(*v, *cap * sizeof(uint32_t));
    if (!*v) abort();
  }
  (*v)[(*n)++] = x;
}

static void push64(uint64_t** v, uint64_t* n, uint64_t* cap, uint64_t x) {
  if (*n == *cap) {
    *cap = *cap ? 2 * *cap : 16;
    *v = (uint64_t*)realloc(*v, *cap * sizeof(uint64_t));
    if (!*v) abort();
  }
  (*v)[(*n)++] = x;
}

static int cmp_u32(const void* a, const void* b) {
  uint32_t x = *(const uint32_t*)a, y = *(const uint32_t*)b;
  return x < y ? -1 : x > y;
}

/* One neuron's binary32 update with input syn and k drive events; returns
   1 if it fires.  Refractory neurons count down and ignore input; a forced
   raster decides the spike by its own draw. */
static int lif32(float alpha, float theta, float u_reset, float w_ext, uint32_t n_ref,
                 int forced, int forced_spike, uint32_t k, float syn, float* u, uint8_t* ref) {
  float ext = f32((double)k * (double)w_ext);
  int integrating = *ref == 0;
  if (!integrating) {
    *ref -= 1;
  } else {
    float I = f32((double)syn + (double)ext);
    float v = f32((double)*u * (double)alpha);
    *u = f32((double)v + (double)I);
  }
  int spike = forced ? forced_spike : (integrating && *u >= theta);
  if (spike) {
    *u = u_reset;
    *ref = (uint8_t)n_ref;
  }
  return spike;
}

/* Step 1: neuron update of both trajectories. */
static void update_neurons(orc_sim* s) {
  const uint64_t t = s->t;
  const uint32_t slot = (uint32_t)(t % s->D);
  const int forced = s->p.forced != 0;
  const uint32_t thr_raster =
      forced && (t % s->p.period_steps) < s->p.on_steps ? s->thr_on : s->thr_off;
  s->n_fired = 0;
  s->n_fired64 = 0;
  for (uint32_t i = 0; i < s->N; ++i) {
    uint32_t r = draw(s->p.seed, i, t, STREAM_POISSON);
    uint32_t k = orc_poisson_k(s->poisson, r);
    int forced_spike = 0;
    if (forced) forced_spike = draw(s->p.seed, i, t, STREAM_RASTER) < thr_raster;

    /* binary32 trajectory */
    float syn = s->ring[(size_t)slot * s->N + i];
    s->ring[(size_t)slot * s->N + i] = 0.0f;
    if (lif32(s->alpha, s->theta, s->u_reset, s->w_ext, s->n_ref, forced, forced_spike, k, syn,
              &s->u[i], &s->ref[i]))
      s->fired[s->n_fired++] = i;

    /* FP64 trajectory */
    double syn64 = s->ring64[(size_t)slot * s->N + i];
    s->ring64[(size_t)slot * s->N + i] = 0.0;
    double ext64 = (double)k * (double)s->w_ext;
    int integrating64 = s->ref64[i] == 0;
    if (!integrating64) {
      s->ref64[i] -= 1;
    } else {
      s->u64[i] = s->u64[i] * (double)s->alpha + (syn64 + ext64);
      double margin = fabs(s->u64[i] - (double)s->theta);
      if (margin < s->min_margin) s->min_margin = margin;
      if (fabs(s->u64[i]) > s->max_abs_u) s->max_abs_u = fabs(s->u64[i]);
    }
    int spike64 = forced ? forced_spike : (integrating64 && s->u64[i] >= (double)s->theta);
    if (spike64) {
      s->u64[i] = (double)s->u_reset;
      s->ref64[i] = (uint8_t)s->n_ref;
      s->fired64[s->n_fired64++] = i;
    }
  }
  /* accuracy bookkeeping: rasters compared step by step; before the first
     step whose rasters differ, the largest |u32 - u64| over every neuron */
  int agree = s->n_fired == s->n_fired64 &&
              memcmp(s->fired, s->fired64, sizeof(uint32_t) * s->n_fired) == 0;
  if (agree) s->agree_steps++;
  if (s->first_div < 0) {
    if (!agree) {
      s->first_div = (int64_t)t;
    } else {
      for (uint32_t i = 0; i < s->N; ++i) {
        double dv = fabs((double)s->u[i] - s->u64[i]);
        if (dv > s->max_dv) s->max_dv = dv;
      }
    }
  }
}

/* Step 2: routing of the binary32 trajectory's spikes, both forms. */
static void route(orc_sim* s, int keep_lists) {
  for (uint32_t p = 0; p < s->P; ++p) { s->flat_n[p] = 0; s->xrecv_n[p] = 0; }
  for (uint32_t n = 0; n < s->n_nodes; ++n) s->bucket_n[n] = 0;
  for (uint32_t f = 0; f < s->n_fired; ++f) {
    const uint32_t src = s->fired[f];
    const uint32_t own = (uint32_t)s->part[src];
    const uint32_t own_node = own / s->G;
    /* VP(src): distinct destination partitions other than its own */
    uint32_t nv = 0;
    const uint64_t stamp = ++s->stamp;
    for (uint64_t e = s->adj_ptr[src]; e < s->adj_ptr[src + 1]; ++e) {
      uint32_t v = s->e_vp[e];
      if (v == own) continue;
      if (s->seen[v] != stamp) {
        s->seen[v] = stamp;
        s->vps[nv++] = v;
      }
    }
    qsort(s->vps, nv, sizeof(uint32_t), cmp_u32);
    /* flat: one entry per destination partition */
    s->stats[ORC_FLAT_MSGS] += nv;
    for (uint32_t j = 0; j < nv; ++j)
      if (keep_lists) push32(&s->flat[s->vps[j]], &s->flat_n[s->vps[j]], &s->flat_cap[s->vps[j]], src);
    /* two-level: OR the partition bits per destination node (bit b of
       node n's mask is partition G*n + b, G <= 64) */
    for (uint32_t j = 0; j < nv; ++j) {
      uint32_t node = s->vps[j] / s->G;
      s->node_mask[node] |= (uint64_t)1 << (s->vps[j] - s->G * node);
    }
    for (uint32_t j = 0; j < nv; ++j) {
      uint32_t node = s->vps[j] / s->G;
      uint64_t mask = s->node_mask[node];
      if (mask == 0) continue;           /* node already emitted */
      s->node_mask[node] = 0;
      if (node == own_node) s->stats[ORC_MSG_L1]++;
      else s->stats[ORC_MSG_L2]++;
      for (uint32_t b = 0; b < s->G; ++b)
        if ((mask >> b) & 1) s->stats[ORC_RECV_ENTRIES]++;
      if (keep_lists) {
        push64(&s->bucket[node], &s->bucket_n[node], &s->bucket_cap[node], src);
        push64(&s->bucket[node], &s->bucket_n[node], &s->bucket_cap[node], mask);
      }
    }
  }
  /* expansion at each destination node: mask bit b -> partition G*n + b */
  for (uint32_t n = 0; n < s->n_nodes; ++n) {
    for (uint64_t m = 0; m < s->bucket_n[n]; m += 2) {
      uint32_t src = (uint32_t)s->bucket[n][m];
      uint64_t mask = s->bucket[n][m + 1];
      for (uint32_t b = 0; b < s->G; ++b)
        if ((mask >> b) & 1) {
          uint32_t p = s->G * n + b;
          push32(&s->xrecv[p], &s->xrecv_n[p], &s->xrecv_cap[p], src);
        }
    }
  }
}

/* Step 3: delivery of every synapse of every fired source. */
static void deliver(orc_sim* s) {
  const uint64_t t = s->t;
  for (uint32_t f = 0; f < s->n_fired; ++f) {
    const uint32_t src = s->fired[f];
    const uint32_t own = (uint32_t)s->part[src];
    for (uint64_t e = s->adj_ptr[src]; e < s->adj_ptr[src + 1]; ++e) {
      size_t at = (size_t)((t + s->e_delay[e]) % s->D) * s->N + s->e_tgt[e];
      s->ring[at] = f32((double)s->ring[at] + (double)s->e_w32[e]);
      if (s->e_vp[e] == own) s->stats[ORC_LOCAL_EVENTS]++;
      else s->stats[ORC_REMOTE_EVENTS]++;
    }
  }
  for (uint32_t f = 0; f < s->n_fired64; ++f) {
    const uint32_t src = s->fired64[f];
    for (uint64_t e = s->adj_ptr[src]; e < s->adj_ptr[src + 1]; ++e) {
      size_t at = (size_t)((t + s->e_delay[e]) % s->D) * s->N + s->e_tgt[e];
      s->ring64[at] += s->e_w64[e];
    }
  }
}

static uint32_t step_impl(orc_sim* s, int keep_lists) {
  memset(s->stats, 0, sizeof(s->stats));
  update_neurons(s);
  s->stats[ORC_SPIKES] = s->n_fired;
  route(s, keep_lists);
  deliver(s);
  s->t++;
  return s->n_fired;
}

uint32_t orc_step(orc_sim* s) { return step_impl(s, 1); }

void orc_run(orc_sim* s, uint32_t n, uint32_t* counts, uint64_t* stats) {
  for (uint32_t i = 0; i < n; ++i) {
    uint32_t c = step_impl(s, 0);
    if (counts) counts[i] = c;
    if (stats) memcpy(stats + (size_t)i * ORC_NSTAT, s->stats, sizeof(s->stats));
  }
}

uint64_t orc_time(const orc_sim* s) { return s->t; }

uint32_t orc_fired(const orc_sim* s, uint32_t* out) {
  if (out) memcpy(out, s->fired, sizeof(uint32_t) * s->n_fired);
  return s->n_fired;
}

uint32_t orc_fired64(const orc_sim* s, uint32_t* out) {
  if (out) memcpy(out, s->fired64, sizeof(uint32_t) * s->n_fired64);
  return s->n_fired64;
}

void orc_counters(const orc_sim* s, uint64_t* out) {
  memcpy(out, s->stats, sizeof(s->stats));
}

uint64_t orc_recv(const orc_sim* s, int which, uint64_t* sizes, uint32_t* entries) {
  uint32_t** lists = which ? s->xrecv : s->flat;
  const uint64_t* ns = which ? s->xrecv_n : s->flat_n;
  uint64_t total = 0;
  for (uint32_t p = 0; p < s->P; ++p) {
    if (sizes) sizes[p] = ns[p];
    if (entries && ns[p]) memcpy(entries + total, lists[p], sizeof(uint32_t) * ns[p]);
    total += ns[p];
  }
  return total;
}

uint64_t orc_buckets(const orc_sim* s, uint64_t* sizes, uint64_t* msgs) {
  uint64_t total = 0;
  for (uint32_t n = 0; n < s->n_nodes; ++n) {
    const uint64_t nm = s->bucket_n[n] / 2;
    if (sizes) sizes[n] = nm;
    if (msgs && nm) memcpy(msgs + 2 * total, s->bucket[n], sizeof(uint64_t) * 2 * nm);
    total += nm;
  }
  return total;
}

void orc_state(const orc_sim* s, float* u, uint8_t* ref, float* ring,
               double* u64, uint8_t* ref64, double* ring64) {
  const size_t N = s->N, DN = (size_t)s->D * s->N;
  if (u) memcpy(u, s->u, sizeof(float) * N);
  if (ref) memcpy(ref, s->ref, N);
  if (ring) memcpy(ring, s->ring, sizeof(float) * DN);
  if (u64) memcpy(u64, s->u64, sizeof(double) * N);
  if (ref64) memcpy(ref64, s->ref64, N);
  if (ring64) memcpy(ring64, s->ring64, sizeof(double) * DN);
}

void orc_accuracy(const orc_sim* s, double* out) {
  out[0] = s->max_dv;
  out[1] = (double)s->first_div;
  out[2] = (double)s->agree_steps;
  out[3] = s->min_margin;
  out[4] = s->max_abs_u;
}

/* ---- Forced raster at any size, without the synapse list of the whole
   network.  With a forced raster a neuron's spike at step t is a pure
   function of (seed, neuron, t), so the raster of a step and the complete
   trajectory of one neuron (from its own incoming synapses) can be computed
   for a network of any size. ---- */

static uint32_t raster_thr_at(const orc_params* p, uint64_t t) {
  double rate = (t % p->period_steps) < p->on_steps ? p->rate_on_hz : p->rate_off_hz;
  return orc_raster_threshold(rate, p->dt_ms);
}

uint32_t orc_forced_raster(const orc_params* p, uint64_t t, uint32_t lo, uint32_t hi,
                           uint32_t* out) {
  const uint32_t thr = raster_thr_at(p, t);
  uint32_t n = 0;
  for (uint32_t i = lo; i < hi; ++i)
    if (draw(p->seed, i, t, STREAM_RASTER) < thr) {
      if (out) out[n] = i;
      n++;
    }
  return n;
}

int orc_forced_neuron(const orc_params* p, uint32_t j, float u0, uint32_t n_in,
                      const uint32_t* in_src, const uint8_t* in_delay, const float* in_w,
                      uint32_t n_steps, float* u_out, uint8_t* ref_out, float* pending,
                      uint32_t* n_spikes) {
  if (!p->forced || p->max_delay == 0 || p->period_steps == 0) return -1;
  const float alpha = orc_alpha(p), theta = f32(p->theta_mv), u_reset = f32(p->u_reset_mv);
  const float w_ext = f32(p->w_ext_mv);
  const uint32_t n_ref = orc_n_ref(p);
  uint32_t poisson[15];
  orc_poisson_table(p->nu_ext_hz * p->dt_ms * 1e-3, poisson);
  /* input arriving at neuron j at step t: in-synapses whose source fired at
     step t - delay (t - delay >= 0) */
  const uint64_t horizon = (uint64_t)n_steps + p->max_delay;
  float* arrive = (float*)xcalloc(horizon, sizeof(float));
  for (uint32_t m = 0; m < n_in; ++m) {
    const float w = p->bf16_weights ? orc_bf16_round(in_w[m]) : in_w[m];
    for (uint64_t ts = 0; ts < n_steps; ++ts)
      if (draw(p->seed, in_src[m], ts, STREAM_RASTER) < raster_thr_at(p, ts))
        arrive[ts + in_delay[m]] = f32((double)arrive[ts + in_delay[m]] + (double)w);
  }
  float u = u0;
  uint8_t ref = 0;
  uint32_t spikes = 0;
  for (uint64_t t = 0; t < n_steps; ++t) {
    uint32_t k = orc_poisson_k(poisson, draw(p->seed, j, t, STREAM_POISSON));
    int fs = draw(p->seed, j, t, STREAM_RASTER) < raster_thr_at(p, t);
    spikes += (uint32_t)lif32(alpha, theta, u_reset, w_ext, n_ref, 1, fs, k, arrive[t], &u, &ref);
  }
  *u_out = u;
  *ref_out = ref;
  if (n_spikes) *n_spikes = spikes;
  /* pending[d-1]: input already scheduled for step n_steps - 1 + d */
  for (uint32_t d = 1; d <= p->max_delay; ++d) pending[d - 1] = arrive[n_steps - 1 + d];
  free(arrive);
  return 0;
}
