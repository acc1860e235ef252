"""Algorithm 2 (growing blocks) on the GPU through the C ABI: every block's
output against the oracle computed block by block on the oracle's own
schedule, Delta = 0 against Algorithm 1, host and device memory, bit-exact."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from oracle import params as orc_params
from paper_2402_14607_amd import binding

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    d = torch.device("cuda:0")
    torch.cuda.set_device(d)
    binding.load()
    return d


def say(msg):
    print(msg, flush=True)


def oracle_growing(x, y, n_e, q1, delta_steps, b, k):
    """Concatenated outputs of blocks 0..k-1, each Ext_IP of its own block."""
    outs = []
    for start, size, q in orc_params.schedule(q1, delta_steps, b, n_e, k):
        lo, hi = start * b // 8, (start + size) * b // 8
        outs.append(oracle.ext_blocks(x[lo:hi], y[lo:hi], q * n_e, q))
    return np.concatenate(outs)


def run(dev, g, x, y, device_memory):
    import torch

    k, nin, nout = g.blocks(x.size)
    if device_memory:
        xd = torch.from_numpy(x).to(dev)
        yd = torch.from_numpy(y).to(dev)
        out = torch.full((nout + 64,), 0xA5, dtype=torch.uint8, device=dev)
        got_k = g.extract(xd, yd, x.size, out, nout + 64)
        res = out.cpu().numpy()
    else:
        res = np.full(nout + 64, 0xA5, dtype=np.uint8)
        got_k = g.extract(x, y, x.size, res, nout + 64)
    assert got_k == k
    assert np.all(res[nout:] == 0xA5)  # nothing written past the k blocks' outputs
    return k, res[:nout]


CASES = [  # n_e, q1, Delta, b, blocks
    (4, 80, 1, 16, 30),
    (3, 64, 2, 8, 50),
    (71, 80, 1, 16, 12),
    (5, 256, 1, 32, 20),
]


@pytest.mark.parametrize("n_e,q1,delta_steps,b,k", CASES, ids=lambda v: str(v))
def test_growing_blocks_against_oracle(dev, n_e, q1, delta_steps, b, k):
    total = sum(size for _, size, _ in orc_params.schedule(q1, delta_steps, b, n_e, k)) * b // 8
    rng = np.random.Generator(np.random.PCG64(q1 + 7 * n_e + delta_steps))
    extra = 37  # a partial block after the k whole ones
    x = rng.integers(0, 256, total + extra, dtype=np.uint8)
    y = rng.integers(0, 256, total + extra, dtype=np.uint8)
    want = oracle_growing(x, y, n_e, q1, delta_steps, b, k)
    say("growing n_e=%d q1=%d delta=%d b=%d: %d blocks, %d output bytes" % (n_e, q1, delta_steps,
                                                                              b, k, want.size))
    for device_memory in (True, False):
        with binding.Growing(n_e, q1, delta_steps, sample_bits=b,
                             device_memory=device_memory) as g:
            got_k, got = run(dev, g, x, y, device_memory)
        assert got_k == k
        assert np.array_equal(got, want), "device_memory=%s" % device_memory


def test_delta_zero_is_algorithm_one(dev):
    """Delta = 0: the same bytes as the plain form over equal blocks
    (Algorithm 1), at the paper's parameter point."""
    import torch

    n_e, q = 71, 80
    pairs = 40
    rng = np.random.Generator(np.random.PCG64(99))
    x = rng.integers(0, 256, pairs * n_e * q // 8, dtype=np.uint8)
    y = rng.integers(0, 256, pairs * n_e * q // 8, dtype=np.uint8)
    with binding.Growing(n_e, q, 0, sample_bits=16) as g:
        k, got = run(dev, g, x, y, True)
    assert k == pairs
    out = torch.zeros(pairs * q // 8, dtype=torch.uint8, device=dev)
    with binding.Extractor(n_e * q, q, device_memory=True,
                           stream=torch.cuda.current_stream(dev).cuda_stream) as ex:
        ex.extract(torch.from_numpy(x).to(dev), torch.from_numpy(y).to(dev), out, pairs)
        ex.sync()
    assert np.array_equal(got, out.cpu().numpy())
    assert np.array_equal(got, oracle.ext_blocks(x, y, n_e * q, q))


def test_growing_limits_and_errors(dev):
    rng = np.random.Generator(np.random.PCG64(5))
    x = rng.integers(0, 256, 4000, dtype=np.uint8)
    with binding.Growing(4, 64, 1, sample_bits=8, device_memory=False) as g:
        k, nin, nout = g.blocks(x.size)
        assert k > 3
        out = np.zeros(nout, dtype=np.uint8)
        assert g.extract(x, x, x.size, out, nout, max_blocks=3) == 3
        want = oracle_growing(x, x, 4, 64, 1, 8, 3)
        assert np.array_equal(out[:want.size], want)
        with pytest.raises(binding.ExtError) as e:
            g.extract(x, x, x.size, out, nout - 1)
        assert e.value.code == binding.EXT_EINVAL
    for bad in [(0, 64, 1, 8), (4, 60, 1, 8), (4, 64, 1, 3), (4, 72, 1, 16)]:
        n_e, q1, d, b = bad
        with pytest.raises(binding.ExtError):
            binding.Growing(n_e, q1, d, sample_bits=b)
