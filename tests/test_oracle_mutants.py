"""The oracle's pins catch plausible mistakes: each mutant below plants one
mistake in a copy of oracle.c (on the CPU), and the pin tests must fail
against it."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PIN_TESTS = ["tests/test_oracle_rng.py", "tests/test_oracle_lif.py",
             "tests/test_oracle_routing.py", "tests/test_oracle_delivery.py",
             "tests/test_oracle_accuracy.py", "tests/test_oracle_forced.py"]

MUTANTS = {
    "philox_word_swap": ("uint32_t y0 = hi1 ^ x1 ^ k0;", "uint32_t y0 = hi1 ^ x3 ^ k0;"),
    "philox_key_bump": ("k1 += W1;", "k1 += W0;"),
    "poisson_strict": ("if (thr[j] <= r) k++;", "if (thr[j] < r) k++;"),
    "drop_drive": ("float I = f32((double)syn + (double)ext);", "float I = f32((double)syn);"),
    "strict_threshold": ("(integrating && *u >= theta)", "(integrating && *u > theta)"),
    "short_refractory": ("*ref = (uint8_t)n_ref;", "*ref = (uint8_t)n_ref - 1;"),
    "fused_update": ("float v = f32((double)*u * (double)alpha);\n"
                     "    *u = f32((double)v + (double)I);",
                     "*u = f32((double)*u * (double)alpha + (double)I);"),
    "mask_bit_shift": ("s->node_mask[node] |= (uint64_t)1 << (s->vps[j] - s->G * node);",
                       "s->node_mask[node] |= 1u << (s->vps[j] - s->G * node + 1);"),
    "own_partition": ("if (v == own) continue;", "if (v == own + 1) continue;"),
    "level_swap": ("if (node == own_node) s->stats[ORC_MSG_L1]++;",
                   "if (node != own_node) s->stats[ORC_MSG_L1]++;"),
    "delay_slot": ("size_t at = (size_t)((t + s->e_delay[e]) % s->D) * s->N + s->e_tgt[e];\n"
                   "      s->ring[at]",
                   "size_t at = (size_t)((t + s->e_delay[e] - 1) % s->D) * s->N + s->e_tgt[e];\n"
                   "      s->ring[at]"),
    "expand_bit_order": ("uint32_t p = s->G * n + b;", "uint32_t p = s->G * n + (s->G - 1 - b);"),
    "bf16_ties_up": ("return ((lo_b >> 16) & 1) == 0 ? lo : hi;", "return hi;"),
    "no_slot_clear": ("s->ring[(size_t)slot * s->N + i] = 0.0f;", ""),
    "fp64_weight": ("s->ring64[at] += s->e_w64[e];",
                    "s->ring64[at] += (double)(float)s->e_w64[e] * 1.0000001;"),
    # the forced raster
    "raster_phase": ("forced && (t % s->p.period_steps) < s->p.on_steps ? s->thr_on : s->thr_off",
                     "forced && (t % s->p.period_steps) <= s->p.on_steps ? s->thr_on : s->thr_off"),
    "raster_phase_any_size": ("double rate = (t % p->period_steps) < p->on_steps ?",
                              "double rate = (t % p->period_steps) <= p->on_steps ?"),
    "raster_rates_swapped": ("? s->thr_on : s->thr_off;", "? s->thr_off : s->thr_on;"),
    "raster_threshold_scale": ("floor(ldexp(rate_hz * dt_ms * 1e-3, 32))",
                               "floor(ldexp(rate_hz * dt_ms * 1e-3, 31))"),
    "raster_stream": ("forced_spike = draw(s->p.seed, i, t, STREAM_RASTER)",
                      "forced_spike = draw(s->p.seed, i, t, STREAM_POISSON)"),
    "forced_neuron_delay": ("arrive[ts + in_delay[m]] = f32((double)arrive[ts + in_delay[m]] + "
                            "(double)w);",
                            "arrive[ts + in_delay[m] - 1] = f32((double)arrive[ts + in_delay[m] - 1] "
                            "+ (double)w);"),
    "forced_neuron_pending": ("pending[d - 1] = arrive[n_steps - 1 + d];",
                              "pending[d - 1] = arrive[n_steps - 2 + d];"),
    # the accuracy report
    "acc_no_max_dv": ("if (dv > s->max_dv) s->max_dv = dv;", "(void)dv;"),
    "acc_no_first_div": ("s->first_div = (int64_t)t;", "(void)t;"),
    "acc_no_margin": ("if (margin < s->min_margin) s->min_margin = margin;", "(void)margin;"),
    "acc_agree_always": ("if (agree) s->agree_steps++;", "s->agree_steps++;"),
    "acc_dv_after_divergence": ("if (s->first_div < 0) {\n    if (!agree) {",
                                "if (1) {\n    if (!agree && s->first_div < 0) {"),
    "acc_max_u_reset": ("if (fabs(s->u64[i]) > s->max_abs_u) s->max_abs_u = fabs(s->u64[i]);",
                        "if (fabs(s->u64[i]) > s->max_abs_u) s->max_abs_u = fabs(s->u64[i]);\n"
                        "      if (s->u64[i] >= (double)s->theta) s->max_abs_u = 0;"),
}


@pytest.mark.slow
@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    src = open(os.path.join(ROOT, "oracle", "oracle.c")).read()
    old, new = MUTANTS[name]
    assert old in src, f"mutation site of {name} not found"
    c = tmp_path / "oracle_mutant.c"
    c.write_text(src.replace(old, new, 1))
    so = tmp_path / "liboracle_mutant.so"
    subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-shared", "-fPIC",
                    "-I", os.path.join(ROOT, "oracle"), "-o", str(so), str(c), "-lm"], check=True)
    env = dict(os.environ, SNN_ORACLE_LIB=str(so))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", *PIN_TESTS],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 1, f"mutant {name} survived:\n{r.stdout[-2000:]}"
