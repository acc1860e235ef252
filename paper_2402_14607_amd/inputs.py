"""Seeded synthetic raw data: 8-bit ADC-style samples of two independent
sources, and the workload definitions built from them.

This module only draws random samples; it holds none of the extractor's
arithmetic.  The tests, the smoke check and the benchmark feed the same
arrays to the GPU path and to the CPU oracle.

Distributions (the paper's raw data come from a homodyne QRNG, Sec. 4.2;
none ships with the paper, so these stand in for it):

* i.i.d. discretised Gaussian: round(N(mean, sigma^2)), half-to-even, clipped
  to [0, 255] -- an i.i.d. source is a forward block source (Sec. 3.1); and
  the same with 16-bit samples for the paper's own parameter point.
* AR(1): u_t = phi * u_{t-1} + e_t with e_t ~ N(0, sigma^2) and u_0 drawn from
  the stationary law N(0, sigma^2 / (1 - phi^2)); sample = clip(round(offset +
  u_t)).  Successive samples, hence successive blocks, are correlated.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def gaussian_adc(n_samples: int, seed: int, mean: float = 128.0, sigma: float = 20.0,
                 chunk: int = 1 << 24) -> np.ndarray:
    """n_samples uint8 samples round(N(mean, sigma^2)) clipped to [0, 255]."""
    rng = _rng(seed)
    out = np.empty(n_samples, dtype=np.uint8)
    for s in range(0, n_samples, chunk):
        k = min(chunk, n_samples - s)
        v = rng.normal(mean, sigma, k)
        np.clip(np.rint(v), 0, 255, out=v)
        out[s:s + k] = v.astype(np.uint8)
    return out


def ar1_adc(n_samples: int, seed: int, phi: float = 0.1, sigma: float = 20.0,
            offset: float = 128.0, chunk: int = 1 << 24) -> np.ndarray:
    """n_samples uint8 samples of the AR(1) process described above."""
    from scipy.signal import lfilter

    rng = _rng(seed)
    out = np.empty(n_samples, dtype=np.uint8)
    u_prev = rng.normal(0.0, sigma / np.sqrt(1.0 - phi * phi))
    first = True
    for s in range(0, n_samples, chunk):
        k = min(chunk, n_samples - s)
        e = rng.normal(0.0, sigma, k)
        if first:
            # u_0 is the stationary draw itself; the recursion starts at u_1
            e[0] = u_prev
            u, _ = lfilter([1.0], [1.0, -phi], e, zi=[0.0])
            first = False
        else:
            u, _ = lfilter([1.0], [1.0, -phi], e, zi=[phi * u_prev])
        u_prev = u[-1]
        v = np.clip(np.rint(offset + u), 0, 255)
        out[s:s + k] = v.astype(np.uint8)
    return out


def gaussian_adc16(n_samples: int, seed: int, mean: float = 32768.0, sigma: float = 682.0,
                   chunk: int = 1 << 23) -> np.ndarray:
    """n_samples 16-bit samples round(N(mean, sigma^2)) clipped to [0, 65535],
    as their little-endian bytes (2 * n_samples uint8).  sigma = 682 gives a
    min-entropy of about 10.74 bits per sample, the rate of the paper's
    homodyne source (Sec. 4.2): -log2 of the most likely value's probability,
    1 / (sigma * sqrt(2 pi))."""
    rng = _rng(seed)
    out = np.empty(n_samples, dtype="<u2")
    for s in range(0, n_samples, chunk):
        k = min(chunk, n_samples - s)
        v = rng.normal(mean, sigma, k)
        np.clip(np.rint(v), 0, 65535, out=v)
        out[s:s + k] = v.astype("<u2")
    return out.view(np.uint8)


@dataclass
class StreamPair:
    """One (X, Y) source pair with its block shape."""
    n_bits: int
    m_bits: int
    x: np.ndarray
    y: np.ndarray

    @property
    def n_pairs(self) -> int:
        return (8 * min(self.x.size, self.y.size)) // self.n_bits


@dataclass
class Workload:
    name: str
    streams: list = field(default_factory=list)


def plain_workload(n_bits: int, m_bits: int, n_pairs: int, seed_x: int, seed_y: int,
                   kind: str = "gaussian") -> StreamPair:
    nbytes = n_pairs * n_bits // 8
    gen = gaussian_adc if kind == "gaussian" else ar1_adc
    return StreamPair(n_bits, m_bits, gen(nbytes, seed_x), gen(nbytes, seed_y))


# The five workloads: sizes, seeds and distributions.
def tiny() -> StreamPair:
    """n = 1024-bit blocks, m = 256, 1024 pairs, i.i.d. Gaussian, seeds 1 and 2."""
    return plain_workload(1024, 256, 1024, 1, 2)


def paper_block(n_pairs: int = 65536) -> StreamPair:
    """n = 8192, m = 2048, 65536 pairs (64 MiB per source), i.i.d. Gaussian,
    seeds 11 and 12."""
    return plain_workload(8192, 2048, n_pairs, 11, 12)


def forward_block_stress(n_pairs: int = 16384) -> StreamPair:
    """n = 65536, m = 16384, 16384 pairs (128 MiB per source), AR(1) with
    phi = 0.1, seeds 21 and 22."""
    return plain_workload(65536, 16384, n_pairs, 21, 22, kind="ar1")


def paper_point(n_pairs: int = 262144) -> StreamPair:
    """The paper's own parameter point (Sec. 4.2): n_e = 71 elements of
    F_2^80 per block (n = 5680 bits = 355 samples of b = 16 bits), m = 80;
    16-bit Gaussian samples as in gaussian_adc16, seeds 31 and 32."""
    n, m = 71 * 80, 80
    samples = n_pairs * n // 16
    return StreamPair(n, m, gaussian_adc16(samples, 31), gaussian_adc16(samples, 32))


BATCHED_N_CHOICES = (2048, 4096, 8192, 16384, 32768)


def batched(n_streams: int = 64, pairs_per_stream: int = 4096, seed: int = 3) -> Workload:
    """n_streams stream pairs, block length n drawn uniformly from
    BATCHED_N_CHOICES (once per stream, seed 3), m = n/4, pairs_per_stream
    pairs each, i.i.d. Gaussian; stream s uses seeds 1000+2s and 1001+2s."""
    rng = _rng(seed)
    ns = rng.choice(np.asarray(BATCHED_N_CHOICES), size=n_streams)
    w = Workload("batched")
    for s, n in enumerate(ns):
        n = int(n)
        w.streams.append(plain_workload(n, n // 4, pairs_per_stream, 1000 + 2 * s, 1001 + 2 * s))
    return w


def served_channels(n_channels: int = 256, seed: int = 4):
    """Channel shapes of the served workload: channel c with c % 4 == 3 is an
    AR(1) forward-block-stress source (n = 65536, m = 16384); every other
    channel is i.i.d. Gaussian with n drawn uniformly from BATCHED_N_CHOICES
    (seed 4) and m = n/4.  Returns a list of (n_bits, m_bits, kind)."""
    rng = _rng(seed)
    ns = rng.choice(np.asarray(BATCHED_N_CHOICES), size=n_channels)
    out = []
    for c in range(n_channels):
        if c % 4 == 3:
            out.append((65536, 16384, "ar1"))
        else:
            out.append((int(ns[c]), int(ns[c]) // 4, "gaussian"))
    return out
