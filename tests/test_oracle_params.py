"""Pins of the oracle's parameter rule, block schedule and error bounds
(CPU only).  Each pin rests on something other than the formula it checks:
numbers the paper prints, exact boundary cases, closed forms checked against
term-by-term sums, and the inequalities the paper proves between them."""
from __future__ import annotations

import math
import random
from fractions import Fraction

import pytest

from oracle import params

PAPER_DELTA = Fraction(1074, 1600)  # 10.74 / 16 (Sec. 4.2)


@pytest.mark.parametrize("n_samples", [2 ** 47, 2 ** 51])
def test_paper_parameter_point(n_samples):
    """Sec. 4.2 prints n = 71 and q = 80 for b = 16, delta = 10.74/16,
    eps = 2^-30 and a raw length of 2^51 bits; the rule gives the same
    whether that length counts samples (2^47 of 16 bits) or is taken as N."""
    assert params.choose_params(16, PAPER_DELTA, n_samples, Fraction(1, 2 ** 30)) == (71, 80)


def test_elements_rule_at_exact_boundaries():
    """24 / (2 delta - 1) is an integer at delta = 3/4 (48) and delta = 1
    (24); just above, the ceiling is unchanged; just below, it steps up."""
    tiny = Fraction(1, 10 ** 9)
    assert params.elements_per_block(Fraction(3, 4)) == 48
    assert params.elements_per_block(Fraction(3, 4) + tiny) == 48
    assert params.elements_per_block(Fraction(3, 4) - tiny) == 49
    assert params.elements_per_block(1) == 24
    assert params.elements_per_block(1 - tiny) == 25
    for bad in (Fraction(1, 2), Fraction(1, 3), Fraction(11, 10)):
        with pytest.raises(ValueError):
            params.elements_per_block(bad)


def test_q_is_the_least_multiple_of_b_reaching_the_target():
    rng = random.Random(5)
    for _ in range(300):
        b = rng.choice([1, 2, 4, 8, 12, 16, 32])
        delta = Fraction(rng.randint(501, 1000), 1000)
        n_samples = rng.randint(2, 2 ** 60)
        eps = Fraction(1, 2 ** rng.randint(1, 80))
        n_e, q = params.choose_params(b, delta, n_samples, eps)
        target = Fraction(n_samples) / (eps * n_e)
        assert q % b == 0 and q > 0
        assert Fraction(2) ** q >= target
        assert q == b or Fraction(2) ** (q - b) < target


def test_rule_makes_each_term_at_most_sqrt3_2_pow_minus_q():
    """Theorem 3.6's middle inequality: with n_e = ceil(24/(2 delta - 1)),
    (delta/4 - 1/8) q n_e - 2q >= q, so each term is at most
    sqrt(3) 2^(-1/4 - q)."""
    for num in range(501, 1001, 7):
        delta = Fraction(num, 1000)
        n_e = params.elements_per_block(delta)
        for q in (8, 16, 80, 256, 2048):
            assert params.block_error_exponent(n_e, q, delta) <= Fraction(-1, 4) - q


def test_bound_says_nothing_at_four_elements():
    """The configured shapes have n_e = 4, below the rule (at least 24):
    there the exponent is -1/4 + q (5/2 - delta) > 0 for every q >= 1."""
    for delta in (Fraction(501, 1000), PAPER_DELTA, Fraction(1)):
        for q in (1, 96, 2048, 16384):
            assert params.block_error_log2(4, q, delta) > 0


def test_output_length_closed_form():
    rng = random.Random(6)
    for _ in range(200):
        q1, d, b, k = rng.randint(1, 500), rng.randint(0, 4), rng.choice([1, 8, 16]), rng.randint(0, 60)
        assert params.output_bits(q1, d, b, k) == k * q1 + k * (k - 1) * d * b // 2


def test_schedule_delta_zero_is_algorithm_one_partition():
    """Delta = 0 makes Algorithm 2 Algorithm 1: equal consecutive blocks of
    q n_e / b samples."""
    blocks = params.schedule(80, 0, 16, 71, 5)
    assert blocks == [(l * 355, 355, 80) for l in range(5)]
    grow = params.schedule(64, 1, 8, 4, 4)
    assert [q for _, _, q in grow] == [64, 72, 80, 88]
    assert [s for s, _, _ in grow] == [0, 32, 68, 108]


def test_stream_error_sum_against_closed_bound():
    """For Delta > 0 the partial sums grow with k and stay below the closed
    geometric bound; for Delta = 0 the sum is k times one term."""
    n_e = params.elements_per_block(PAPER_DELTA)
    prev = -math.inf
    closed = params.stream_error_closed_log2(80, 1, 16)
    sums = [params.stream_error_log2(n_e, 80, 1, 16, PAPER_DELTA, k) for k in (1, 2, 5, 20, 200)]
    assert sums[0] < sums[1]  # later terms shrink below float resolution quickly
    for s in sums:
        assert prev <= s < closed
        prev = s
    one = params.block_error_log2(n_e, 80, PAPER_DELTA)
    for k in (1, 3, 1000):
        assert params.stream_error_log2(n_e, 80, 0, 16, PAPER_DELTA, k) == pytest.approx(
            one + math.log2(k), abs=1e-9)
    assert params.stream_error_closed_log2(80, 0, 16) == math.inf


def test_theorem_3_7_holds_at_the_printed_point():
    """Algorithm 1's N b / (q n_e) blocks, each within Theorem 3.3's bound,
    add up to less than eps = 2^-30 at the printed parameters (either
    reading of N)."""
    for n_samples in (2 ** 47, 2 ** 51):
        n_e, q = params.choose_params(16, PAPER_DELTA, n_samples, Fraction(1, 2 ** 30))
        blocks = n_samples * 16 // (q * n_e)
        total = params.block_error_log2(n_e, q, PAPER_DELTA) + math.log2(blocks)
        assert total <= -30
