// Host-code sanitizer driver: runs the CPU parts (seeded generator, host setup
// of the network arrays, the oracle) on small networks of every topology, both
// weight types, the error paths of the setup and an oracle run in both raster
// modes, so that an AddressSanitizer / UndefinedBehaviorSanitizer build can
// check them for out-of-bounds accesses, leaks and undefined behaviour.
// Built and run by tests/test_sanitizers.py; prints "sanitize ok" at the end.
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "snn_setup.h"

extern "C" {
#include "oracle.h"
#include "synth.h"
}

// The library's error reporter lives in the HIP runtime; the CPU build only
// needs somewhere for the message to go.
extern "C" snn_status snn_fail_v(snn_status s, const char* fmt, va_list ap) {
  char buf[256];
  std::vsnprintf(buf, sizeof buf, fmt, ap);
  std::fprintf(stderr, "[setup error %d] %s\n", int(s), buf);
  return s;
}

#define CHECK(c)                                                          \
  do {                                                                    \
    if (!(c)) {                                                           \
      std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
      std::exit(1);                                                       \
    }                                                                     \
  } while (0)

namespace {

snn_setup_spec base_spec(uint32_t topo, uint32_t n, uint32_t parts, uint32_t wtype) {
  snn_setup_spec s;
  std::memset(&s, 0, sizeof s);
  s.seed = 1234 + topo;
  s.n_neurons = n;
  s.k_in = 40;
  s.max_delay = 5;
  s.n_partitions = parts;
  s.topology = topo;
  s.vp_set_size = topo == 2 ? 6 : 0;
  s.remote_frac = 0.6;
  s.w_exc = 0.5;
  s.w_inh = -2.5;
  s.w_jitter = 0.2;
  s.gpus_per_node = 4;
  s.weight_type = wtype;
  s.n_threads = 3;
  s.n_clusters = topo == 4 ? 7 : 0;
  s.p_in = topo == 4 ? 0.8 : 0.0;
  return s;
}

// Host setup of one network: every array it writes, at its stated size.
void run_setup(const snn_setup_spec& spec, const uint32_t* part_start, const double* cross,
               const int32_t* part_map) {
  snn_setup_handle h = nullptr;
  CHECK(snn_setup_create(&spec, part_start, cross, part_map, &h) == SNN_OK);
  uint64_t nnz, pairs, buckets, recv;
  CHECK(snn_setup_sizes(h, &nnz, &pairs, &buckets, &recv) == SNN_OK);
  CHECK(nnz == uint64_t(spec.n_neurons) * spec.k_in);
  float bound = 0;
  CHECK(snn_setup_input_bound(h, &bound) == SNN_ERR_BAD_STATE);
  const uint32_t n = spec.n_neurons;
  std::vector<int64_t> row_ptr(n + 1);
  std::vector<uint32_t> n_local(n), tgt_delay(nnz);
  std::vector<uint16_t> delay_off(size_t(n) * (spec.max_delay + 1));
  std::vector<uint8_t> weight(nnz * (spec.weight_type == SNN_W_BF16 ? 2 : 4));
  CHECK(snn_setup_fill_rows(h, row_ptr.data(), n_local.data(), delay_off.data(),
                            tgt_delay.data(), weight.data()) == SNN_OK);
  CHECK(row_ptr[n] == int64_t(nnz));
  CHECK(snn_setup_sizes(h, &nnz, &pairs, &buckets, &recv) == SNN_OK);
  CHECK(snn_setup_input_bound(h, &bound) == SNN_OK && bound > 0);
  const uint32_t nodes = (spec.n_partitions + spec.gpus_per_node - 1) / spec.gpus_per_node;
  std::vector<int64_t> vp_ptr(n + 1);
  std::vector<uint16_t> vp_part(pairs);
  std::vector<uint64_t> vp_rec(2 * pairs), bucket_off(nodes + 1), recv_off(spec.n_partitions + 1);
  std::vector<int32_t> part_of(n);
  CHECK(snn_setup_fill_routes(h, tgt_delay.data(), weight.data(), vp_ptr.data(), vp_part.data(),
                              vp_rec.data(), part_of.data(), bucket_off.data(),
                              recv_off.data()) == SNN_OK);
  CHECK(vp_ptr[n] == int64_t(pairs));
  CHECK(bucket_off[nodes] == buckets && recv_off[spec.n_partitions] == recv);
  snn_setup_destroy(h);
}

void setup_errors() {
  snn_setup_handle h = nullptr;
  snn_setup_spec s = base_spec(0, 1000, 4, SNN_W_FP32);
  const uint32_t ps[5] = {0, 250, 500, 750, 1000};
  CHECK(snn_setup_create(nullptr, ps, nullptr, nullptr, &h) == SNN_ERR_INVALID_ARG);
  s.max_delay = 16;
  CHECK(snn_setup_create(&s, ps, nullptr, nullptr, &h) == SNN_ERR_INVALID_ARG);
  s = base_spec(0, 1000, 4, 7);
  CHECK(snn_setup_create(&s, ps, nullptr, nullptr, &h) == SNN_ERR_INVALID_ARG);
  s = base_spec(0, 1000, 4, SNN_W_FP32);
  std::vector<int32_t> bad(1000, 0);
  bad[17] = 4;  // partition out of range
  CHECK(snn_setup_create(&s, ps, nullptr, bad.data(), &h) == SNN_ERR_INVALID_ARG);
  s = base_spec(1, 1000, 4, SNN_W_FP32);
  std::vector<int32_t> ok(1000, 0);
  CHECK(snn_setup_create(&s, nullptr, nullptr, ok.data(), &h) == SNN_ERR_INVALID_ARG);
}

// The oracle on the materialised network: a few LIF steps and a few forced
// raster steps, with every read-back it offers.
void run_oracle(uint32_t forced, uint32_t bf16) {
  const uint32_t n = 1200, parts = 6, k = 40;
  syn_spec ss;
  std::memset(&ss, 0, sizeof ss);
  ss.seed = 77;
  ss.n_neurons = n;
  ss.k_in = k;
  ss.max_delay = 5;
  ss.n_partitions = parts;
  ss.topology = SYN_TOPO_MATERIALIZED;
  ss.w_exc = 0.5;
  ss.w_inh = -2.5;
  ss.w_jitter = 0.2;
  const uint32_t ps[parts + 1] = {0, 200, 400, 600, 800, 1000, 1200};
  syn_gen* g = syn_create(&ss, ps, nullptr);
  CHECK(g);
  const uint64_t m = uint64_t(n) * k;
  std::vector<uint32_t> src(m), tgt(m);
  std::vector<uint8_t> delay(m);
  std::vector<uint16_t> vp(m);
  std::vector<float> w(m), u0(n);
  std::vector<int32_t> part(n);
  syn_edges(g, 0, n, src.data(), tgt.data(), delay.data(), vp.data(), w.data());
  syn_part_map(g, part.data());
  syn_initial_u(ss.seed, 20.0, n, u0.data());
  syn_destroy(g);

  orc_params p;
  std::memset(&p, 0, sizeof p);
  p.n_neurons = n;
  p.n_partitions = parts;
  p.gpus_per_node = 4;
  p.max_delay = 5;
  p.dt_ms = 0.1;
  p.tau_m_ms = 20.0;
  p.theta_mv = 20.0;
  p.u_reset_mv = 10.0;
  p.t_ref_ms = 2.0;
  p.nu_ext_hz = 20000.0;
  p.w_ext_mv = 0.1;
  p.seed = 5;
  p.forced = forced;
  p.period_steps = 40;
  p.on_steps = 10;
  p.rate_on_hz = 200.0;
  p.rate_off_hz = 5.0;
  p.bf16_weights = bf16;
  orc_sim* s = orc_create(&p, m, src.data(), tgt.data(), delay.data(), vp.data(), w.data(),
                          part.data(), u0.data());
  CHECK(s);
  std::vector<uint32_t> fired(n), counts(30);
  std::vector<uint64_t> stats(30 * ORC_NSTAT), sizes(parts), cnt(ORC_NSTAT);
  uint64_t spikes = 0;
  for (int t = 0; t < 30; ++t) {
    spikes += orc_step(s);
    orc_fired(s, fired.data());
    orc_fired64(s, fired.data());
    orc_counters(s, cnt.data());
    for (int which = 0; which < 2; ++which) {
      const uint64_t tot = orc_recv(s, which, sizes.data(), nullptr);
      std::vector<uint32_t> ent(tot + 1);
      CHECK(orc_recv(s, which, sizes.data(), ent.data()) == tot);
    }
    const uint32_t nodes = (parts + 3) / 4;
    std::vector<uint64_t> bs(nodes);
    const uint64_t msgs = orc_buckets(s, bs.data(), nullptr);
    std::vector<uint64_t> mw(2 * msgs + 2);
    CHECK(orc_buckets(s, bs.data(), mw.data()) == msgs);
  }
  orc_run(s, 30, counts.data(), stats.data());
  CHECK(orc_time(s) == 60);
  std::vector<float> u(n), ring(size_t(6) * n);
  std::vector<uint8_t> ref(n), ref64(n);
  std::vector<double> u64(n), ring64(size_t(6) * n), acc(5);
  orc_state(s, u.data(), ref.data(), ring.data(), u64.data(), ref64.data(), ring64.data());
  orc_accuracy(s, acc.data());
  orc_destroy(s);
  std::printf("oracle forced=%u bf16=%u: %llu spikes in the first 30 steps\n", forced, bf16,
              (unsigned long long)spikes);
}

void model_params() {
  snn_model m = {0.1, 20.0, 20.0, 10.0, 2.0, 8000.0, 0.1, 200.0, 5.0};
  snn_params p;
  std::memset(&p, 0, sizeof p);
  CHECK(snn_setup_model_params(&m, &p) == SNN_OK);
  CHECK(p.n_ref == 20 && p.alpha > 0.99f && p.alpha < 1.0f);
  for (int j = 1; j < 15; ++j) CHECK(p.poisson_thr[j] >= p.poisson_thr[j - 1]);
  m.dt_ms = 0.0;
  CHECK(snn_setup_model_params(&m, &p) == SNN_ERR_INVALID_ARG);
  CHECK(snn_setup_model_params(nullptr, &p) == SNN_ERR_INVALID_ARG);
}

}  // namespace

int main() {
  setup_errors();
  model_params();
  for (uint32_t wt = 0; wt < 2; ++wt) {
    const uint32_t ps[7] = {0, 150, 300, 450, 600, 900, 1200};
    run_setup(base_spec(0, 1200, 6, wt), ps, nullptr, nullptr);
    run_setup(base_spec(1, 1000, 9, wt), nullptr, nullptr, nullptr);
    run_setup(base_spec(2, 1000, 9, wt), nullptr, nullptr, nullptr);
    const double cross[6] = {0.1, 0.5, 0.9, 0.3, 0.0, 1.0};
    run_setup(base_spec(3, 1200, 6, wt), ps, cross, nullptr);
    std::vector<int32_t> map(1200);
    for (uint32_t i = 0; i < 1200; ++i) map[i] = int32_t((i * 7919u) % 6u);
    run_setup(base_spec(4, 1200, 6, wt), ps, nullptr, map.data());
    run_setup(base_spec(0, 1200, 6, wt), ps, nullptr, map.data());
  }
  std::printf("setup ok\n");
  run_oracle(0, 0);
  run_oracle(1, 0);
  run_oracle(0, 1);
  std::printf("sanitize ok\n");
  return 0;
}
