"""Pins of the oracle's random-number and rounding building blocks against
implementations other than its own (CPU only)."""
import math
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
ROCRAND_HDR = "/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"


@pytest.fixture(scope="module")
def rocrand_philox(tmp_path_factory):
    """Builds the rocRAND host-side Philox program (AMD's implementation)."""
    if not os.path.exists(ROCRAND_HDR) or shutil.which("g++") is None:
        pytest.skip("rocRAND headers or g++ not available")
    exe = str(tmp_path_factory.mktemp("philox") / "philox_rocrand")
    subprocess.run(["g++", "-O1", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                    os.path.join(HERE, "pins", "philox_rocrand.cpp"), "-o", exe], check=True)
    return exe


def test_philox_matches_rocrand(rocrand_philox):
    rng = np.random.default_rng(1234)
    cases = []
    for _ in range(300):
        seed = int(rng.integers(0, 2**64, dtype=np.uint64))
        ctr = [int(x) for x in rng.integers(0, 2**32, size=4, dtype=np.uint64)]
        # rocRAND addresses counter words 0,1 through a 64-bit offset counted
        # in 32-bit outputs, so word 1 must stay below 2^30 to be reachable
        ctr[1] >>= 2
        cases.append((seed, *ctr))
    # edge counters and keys
    cases += [(0, 0, 0, 0, 0), (2**64 - 1, 2**32 - 1, 2**30 - 1, 2**32 - 1, 2**32 - 1),
              (11, 0, 999, 1, 0), (11, 1249999, 999, 2, 0)]
    inp = "".join(f"{s} {a} {b} {c} {d}\n" for s, a, b, c, d in cases)
    res = subprocess.run([rocrand_philox], input=inp, capture_output=True, text=True, check=True)
    lines = res.stdout.strip().splitlines()
    assert len(lines) == len(cases)
    for (seed, a, b, c, d), line in zip(cases, lines):
        want = [int(x) for x in line.split()]
        got = oracle.philox4x32_10([a, b, c, d], [seed & 0xFFFFFFFF, seed >> 32])
        assert list(got) == want, (seed, a, b, c, d)


@pytest.mark.parametrize("lam", [0.5, 1e-3, 0.05, 2.0, 7.5])
def test_poisson_table_matches_scipy_cdf(lam):
    from scipy.stats import poisson
    thr = oracle.poisson_table(lam)
    for j in range(15):
        ref = math.ldexp(float(poisson.cdf(j, lam)), 32)
        want = min(math.floor(ref), 2**32 - 1)
        # two FP64 evaluations of the CDF can straddle an integer only when
        # 2^32 * CDF lies within a few ulps of it
        if abs(ref - round(ref)) > 1e-6 * max(ref, 1.0) or ref >= 2**32 - 1:
            assert int(thr[j]) == want, (lam, j)
        else:
            assert abs(int(thr[j]) - want) <= 1
    assert np.all(np.diff(thr.astype(np.int64)) >= 0)


def test_poisson_table_degenerate_rates():
    # zero rate: every threshold is 2^32 - 1, so k = 0 except for r = 2^32 - 1
    assert np.all(oracle.poisson_table(0.0) == 2**32 - 1)
    # huge rate: CDF(14) underflows the table, every threshold is 0, k = 15
    assert np.all(oracle.poisson_table(1000.0) == 0)


def test_poisson_inversion_boundaries():
    """Inverse-transform sampling: k is the smallest j with r < T_j (T_j =
    floor(2^32 CDF(j))), 15 when there is none.  Checked at and around every
    table entry."""
    thr = oracle.poisson_table(0.5)
    def smallest(r):
        for j in range(15):
            if r < int(thr[j]):
                return j
        return 15
    for j in range(15):
        for r in (int(thr[j]) - 1, int(thr[j]), int(thr[j]) + 1):
            if 0 <= r < 2**32:
                assert oracle.poisson_k(thr, r) == smallest(r), (j, r)
    for r in (0, 1, 2**31, 2**32 - 1):
        assert oracle.poisson_k(thr, r) == smallest(r)


def test_poisson_drive_statistics():
    """Inversion of the oracle's Philox words by its table has the Poisson
    law: mean lambda and P(k = 0) = exp(-lambda), within 4 sigma."""
    lam = 0.5
    thr = oracle.poisson_table(lam).astype(np.uint64)
    n = 200_000
    words = np.empty(n, np.uint64)
    for c in range(n // 4):
        words[4 * c:4 * c + 4] = oracle.philox4x32_10([c, 7, 1, 0], [11, 0])
    k = (words[:, None] >= thr[None, :]).sum(axis=1)
    sd_mean = math.sqrt(lam / n)
    assert abs(k.mean() - lam) < 4 * sd_mean
    p0 = math.exp(-lam)
    assert abs((k == 0).mean() - p0) < 4 * math.sqrt(p0 * (1 - p0) / n)
    p1 = lam * math.exp(-lam)
    assert abs((k == 1).mean() - p1) < 4 * math.sqrt(p1 * (1 - p1) / n)


def test_bf16_round_matches_torch():
    import torch
    rng = np.random.default_rng(5)
    xs = np.concatenate([
        rng.standard_normal(4000).astype(np.float32) * 3,
        (rng.standard_normal(500) * 1e30).astype(np.float32),
        np.array([0.5, -2.5, 0.1, -0.1, 1.0 + 2**-8, 1.0 + 3 * 2**-8, 1.0 + 2**-8 + 2**-20,
                  3.3895314e38, 3.4e38, -3.39e38, 1e-40, -1e-41, 1.1754944e-38], np.float32),
    ])
    # exact ties: the bit just below the kept significand set, nothing below it
    ties = (rng.integers(0, 2**16, 500).astype(np.uint32) << 16) | np.uint32(0x8000)
    ties &= np.uint32(0x7F7FFFFF)
    xs = np.concatenate([xs, ties.view(np.float32)])
    xs = xs[np.isfinite(xs)]
    want = torch.from_numpy(xs).to(torch.bfloat16).to(torch.float32).numpy()
    got = np.array([oracle.bf16_round(x) for x in xs], np.float32)
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))


def test_derived_constants():
    import synth
    wl = synth.get_workload("tiny")
    p = oracle.params_from_workload(wl)
    a = oracle.alpha(p)
    # fl32(exp(-0.1 / 20)) = 0.995012462139129638671875 exactly: the binary32
    # neighbours of exp(-0.005) = 0.99501247919268... are this value and one
    # ulp (2^-24) above it, and this one is nearer
    assert float(a) == 0.995012462139129638671875
    assert abs(float(a) - 0.99501247919268232) < 2**-25
    assert oracle.n_ref(p) == 20
    assert oracle.raster_threshold(100.0, 0.1) == math.floor(0.01 * 2**32)
    assert oracle.raster_threshold(0.0, 0.1) == 0
