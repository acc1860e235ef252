"""The library's parameter rule and security bounds (host code, no GPU)
against the oracle's exact-rational statement of Algorithm 1, Theorem 3.3
and Theorem 3.6."""
from __future__ import annotations

import math
import random
from fractions import Fraction

import pytest

from oracle import params as orc
from paper_2402_14607_amd import binding


@pytest.fixture(scope="module")
def lib():
    return binding.load()


def test_paper_point(lib):
    """Sec. 4.2: b = 16, delta = 10.74/16, 2^47 samples (2^51 bits), eps = 2^-30."""
    assert binding.choose_params(16, 1074, 1600, 47.0, -30.0) == (71, 80)
    assert binding.choose_params(16, 1074, 1600, 51.0, -30.0) == (71, 80)


def test_choose_params_matches_oracle(lib):
    rng = random.Random(11)
    for _ in range(500):
        b = rng.choice([1, 2, 4, 8, 16, 32])
        den = rng.choice([10, 16, 100, 1000, 1600, 4096])
        num = rng.randint(den // 2 + 1, den)
        log2_n = rng.randint(4, 62)
        log2_eps = -rng.randint(1, 100)
        delta = Fraction(num, den)
        n_samples = 2 ** log2_n
        try:
            want = orc.choose_params(b, delta, n_samples, Fraction(1, 2 ** -log2_eps))
        except ValueError:
            with pytest.raises(binding.ExtError):
                binding.choose_params(b, num, den, log2_n, log2_eps)
            continue
        assert binding.choose_params(b, num, den, log2_n, log2_eps) == want, (b, num, den, log2_n,
                                                                               log2_eps)


def test_choose_params_rejects(lib):
    for args in [(16, 1, 2, 47.0, -30.0),      # delta = 1/2
                 (16, 3, 2, 47.0, -30.0),      # delta > 1
                 (0, 3, 4, 47.0, -30.0),       # no sample size
                 (16, 3, 4, 47.0, 0.0),        # eps = 1
                 (16, 3, 4, 2.0, -1.0)]:       # N / (eps n_e) below 1
        with pytest.raises(binding.ExtError):
            binding.choose_params(*args)


def test_block_error_matches_oracle(lib):
    rng = random.Random(12)
    for _ in range(300):
        n_e, q = rng.randint(1, 200), rng.randint(1, 20000)
        delta = Fraction(rng.randint(1, 1000), 1000)
        want = orc.block_error_log2(n_e, q, delta)
        got = binding.block_error_log2(n_e, q, float(delta))
        assert got == pytest.approx(want, rel=1e-12, abs=1e-9)
    assert math.isnan(binding.block_error_log2(0, 80, 0.7))


@pytest.mark.parametrize("delta_steps", [0, 1, 3])
def test_stream_error_matches_term_by_term_sum(lib, delta_steps):
    """Closed-form geometric sum (library) against the oracle's term-by-term
    sum, in the converging (n_e from the rule) and the growing (n_e = 4)
    regimes."""
    rng = random.Random(13 + delta_steps)
    for _ in range(60):
        delta = Fraction(rng.randint(520, 1000), 1000)
        n_e = orc.elements_per_block(delta) if rng.random() < 0.7 else 4
        b = rng.choice([8, 16])
        q1 = b * rng.randint(2, 12)
        k = rng.choice([1, 2, 7, 40, 300])
        want = orc.stream_error_log2(n_e, q1, delta_steps, b, delta, k)
        got, closed = binding.stream_error_log2(n_e, q1, delta_steps, b, float(delta), k)
        assert got == pytest.approx(want, abs=1e-9 * max(1.0, abs(want)))
        want_c = orc.stream_error_closed_log2(q1, delta_steps, b)
        if delta_steps == 0:
            assert closed == math.inf and want_c == math.inf
        else:
            assert closed == pytest.approx(want_c, abs=1e-12)


def test_output_bits_matches_oracle(lib):
    rng = random.Random(14)
    for _ in range(200):
        q1, d, b, k = rng.randint(1, 5000), rng.randint(0, 5), rng.choice([1, 8, 16]), rng.randint(0, 5000)
        assert binding.output_bits(q1, d, b, k) == orc.output_bits(q1, d, b, k)
    with pytest.raises(binding.ExtError):
        binding.output_bits(80, 1, 16, 2 ** 40)
