"""Parameter rule, block schedules and error bounds of the block-wise
extractors, restated from the paper in exact rational arithmetic.

TEST INFRASTRUCTURE ONLY, like the rest of this package: the tests are its
only callers, and the library's own implementation (host C code) shares
nothing with it.

What it states (Li & Zhou, "Real-Time Seedless Post-Processing for Quantum
Random Number Generators"):

* Algorithm 1, parameters: n_e = ceil(24 / (2 delta - 1)) elements per block
  and q = b * ceil(log2(N / (eps * n_e)) / b) bits per element, for two
  (b, N, delta) forward block sources (N samples of b bits) and a total
  error eps.
* Theorem 3.3: Ext_IP^{n_e,q} errs by at most
  sqrt(3) * 2^(-1/4 - (delta/4 - 1/8) * q * n_e + 2q).
* Algorithm 2: block l holds q_l * n_e / b samples of each source, right after
  block l-1, with q_{l+1} = q_l + Delta * b; Delta = 0 is Algorithm 1's
  partition.
* Theorem 3.6: the first k outputs of Algorithm 2 are within
  sum_{l <= k} sqrt(3) * 2^(-1/4 - (delta/4 - 1/8) q_l n_e + 2 q_l) of uniform;
  with n_e from the rule above each term is at most sqrt(3) * 2^(-1/4 - q_l),
  and for Delta > 0 the sum is below sqrt(3) * 2^(-1/4 - q_1) / (1 - 2^(-Delta b));
  the output length is m_k = k q_1 + k (k - 1) Delta b / 2.
* Theorem 3.7: Algorithm 1's whole output is eps-close to uniform.
"""
from __future__ import annotations

import math
from fractions import Fraction

LOG2_SQRT3 = 0.5 * math.log2(3.0)


def _frac(v) -> Fraction:
    return v if isinstance(v, Fraction) else Fraction(v)


def elements_per_block(delta) -> int:
    """n_e = ceil(24 / (2 delta - 1)) (Algorithm 1); delta in (1/2, 1]."""
    d = _frac(delta)
    if not (Fraction(1, 2) < d <= 1):
        raise ValueError("the min-entropy rate must lie in (1/2, 1]")
    return math.ceil(Fraction(24) / (2 * d - 1))


def choose_params(sample_bits: int, delta, n_samples, eps) -> tuple[int, int]:
    """(n_e, q) of Algorithm 1 for sources of n_samples samples of
    sample_bits bits each and total error eps; q is the least multiple of
    sample_bits whose power of two reaches N / (eps * n_e)."""
    b = int(sample_bits)
    if b <= 0:
        raise ValueError("sample_bits must be positive")
    e = _frac(eps)
    if not (0 < e < 1):
        raise ValueError("eps must lie in (0, 1)")
    n_e = elements_per_block(delta)
    v = _frac(n_samples) / (e * n_e)
    if v <= 1:
        raise ValueError("N / (eps n_e) must exceed 1 for q to be positive")
    k = 1
    while Fraction(2) ** (k * b) < v:
        k += 1
    return n_e, k * b


def block_error_exponent(n_e: int, q: int, delta) -> Fraction:
    """Exponent E of Theorem 3.3's bound sqrt(3) * 2^E, exactly."""
    d = _frac(delta)
    return Fraction(-1, 4) - (d / 4 - Fraction(1, 8)) * q * n_e + 2 * q


def block_error_log2(n_e: int, q: int, delta) -> float:
    """log2 of Theorem 3.3's bound (0 or more: the bound says nothing)."""
    return LOG2_SQRT3 + float(block_error_exponent(n_e, q, delta))


def schedule(q1: int, delta_steps: int, sample_bits: int, n_e: int, k: int):
    """Algorithm 2's first k blocks as (first sample, samples, q_l), samples
    counted per source from 0."""
    out, start, q = [], 0, int(q1)
    for _ in range(int(k)):
        if (q * n_e) % sample_bits:
            raise ValueError("q_l * n_e must be a multiple of the sample size")
        size = q * n_e // sample_bits
        out.append((start, size, q))
        start += size
        q += delta_steps * sample_bits
    return out


def output_bits(q1: int, delta_steps: int, sample_bits: int, k: int) -> int:
    """m_k, the output bits of Algorithm 2's first k blocks, summed block by
    block."""
    return sum(q1 + l * delta_steps * sample_bits for l in range(int(k)))


def stream_error_log2(n_e: int, q1: int, delta_steps: int, sample_bits: int, delta, k: int) -> float:
    """log2 of Theorem 3.6's sum over Algorithm 2's first k blocks (term by
    term; meant for k up to about 10^5)."""
    exps = [block_error_exponent(n_e, q1 + l * delta_steps * sample_bits, delta)
            for l in range(int(k))]
    top = max(exps)
    rest = sum(2.0 ** float(e - top) for e in exps)
    return LOG2_SQRT3 + float(top) + math.log2(rest)


def stream_error_closed_log2(q1: int, delta_steps: int, sample_bits: int) -> float:
    """log2 of Theorem 3.6's closed bound sqrt(3) 2^(-1/4-q1) / (1 - 2^(-Delta b));
    infinite for Delta = 0 (the sum then grows without limit)."""
    if delta_steps == 0:
        return math.inf
    return LOG2_SQRT3 - 0.25 - q1 - math.log2(1.0 - 2.0 ** (-delta_steps * sample_bits))
