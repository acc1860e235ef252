"""The allocation-free growing-block call (ext_growing_extract_noalloc) on the
GPU through the C ABI: two calls in a row, the second on a smaller input,
each byte for byte equal to ext_growing_extract on the same handle and
inputs, and to the oracle; the largest call the static scratch takes; the
refusals (too many blocks, host memory)."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from oracle import params as orc_params
from paper_2402_14607_amd import binding

pytestmark = pytest.mark.gpu

MAX_BLOCKS = 4096  # EXT_NOALLOC_MAX_BLOCKS


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
    outs = []
    for start, size, q in orc_params.schedule(q1, delta_steps, b, n_e, k):
        lo, hi = start * b // 8, (start + size) * b // 8
        outs.append(oracle.ext_blocks(x[lo:hi], y[lo:hi], q * n_e, q))
    return np.concatenate(outs)


def both_forms(dev, g, x, y, n_bytes):
    """(k, noalloc output, allocating output) on device copies of x and y,
    with canary bytes after the outputs."""
    import torch

    k, _, nout = g.blocks(n_bytes)
    xd = torch.from_numpy(x).to(dev)
    yd = torch.from_numpy(y).to(dev)
    a = torch.full((nout + 64,), 0xA5, dtype=torch.uint8, device=dev)
    b = torch.full((nout + 64,), 0x5A, dtype=torch.uint8, device=dev)
    ka = g.extract_noalloc(xd, yd, n_bytes, a, nout + 64)
    kb = g.extract(xd, yd, n_bytes, b, nout + 64)
    a, b = a.cpu().numpy(), b.cpu().numpy()
    assert ka == kb == k
    assert np.all(a[nout:] == 0xA5) and np.all(b[nout:] == 0x5A)
    return k, a[:nout], b[:nout]


@pytest.mark.parametrize("n_e,q1,delta_steps,b", [(4, 80, 1, 16), (3, 64, 2, 8)],
                         ids=lambda v: str(v))
def test_noalloc_two_calls_second_smaller(dev, n_e, q1, delta_steps, b):
    rng = np.random.Generator(np.random.PCG64(1000 + q1 + n_e))
    sizes = []
    for k in (40, 13):  # the second call takes fewer blocks (fewer bytes)
        sched = orc_params.schedule(q1, delta_steps, b, n_e, k)
        sizes.append(sum(z for _, z, _ in sched) * b // 8 + 11)  # + a partial block
    x = rng.integers(0, 256, sizes[0], dtype=np.uint8)
    y = rng.integers(0, 256, sizes[0], dtype=np.uint8)
    with binding.Growing(n_e, q1, delta_steps, sample_bits=b, device_memory=True) as g:
        for call, n_bytes in enumerate(sizes):
            say("noalloc n_e=%d q1=%d delta=%d b=%d, call %d: %d bytes per source"
                % (n_e, q1, delta_steps, b, call, n_bytes))
            xs, ys = x[:n_bytes].copy(), y[:n_bytes].copy()
            k, got, ref = both_forms(dev, g, xs, ys, n_bytes)
            assert np.array_equal(got, ref)
            assert np.array_equal(got, oracle_growing(xs, ys, n_e, q1, delta_steps, b, k))


def test_noalloc_largest_call_and_refusals(dev):
    import torch

    # q = 8, one element, Delta = 0: one byte per block, so n_bytes is the
    # block count
    n = MAX_BLOCKS
    rng = np.random.Generator(np.random.PCG64(77))
    x = rng.integers(0, 256, n + 1, dtype=np.uint8)
    y = rng.integers(0, 256, n + 1, dtype=np.uint8)
    with binding.Growing(1, 8, 0, sample_bits=8, device_memory=True) as g:
        say("noalloc: %d one-byte blocks (the static scratch's limit)" % n)
        k, got, ref = both_forms(dev, g, x[:n].copy(), y[:n].copy(), n)
        assert k == n
        assert np.array_equal(got, ref)
        assert np.array_equal(got, oracle.ext_blocks(x[:n], y[:n], 8, 8))
        xd = torch.from_numpy(x).to(dev)
        yd = torch.from_numpy(y).to(dev)
        out = torch.full((n + 64,), 0xA5, dtype=torch.uint8, device=dev)
        say("noalloc: %d blocks refused" % (n + 1))
        with pytest.raises(binding.ExtError) as e:
            g.extract_noalloc(xd, yd, n + 1, out, n + 64)
        assert e.value.code == binding.EXT_ENOMEM
        assert np.all(out.cpu().numpy() == 0xA5)  # nothing written
        # capped by max_blocks, the same input is within the limit
        assert g.extract_noalloc(xd, yd, n + 1, out, n + 64, max_blocks=n) == n
        assert np.array_equal(out.cpu().numpy()[:n], ref)
    with binding.Growing(4, 64, 1, sample_bits=8, device_memory=False) as g:
        buf = np.zeros(4096, dtype=np.uint8)
        with pytest.raises(binding.ExtError) as e:
            g.extract_noalloc(buf, buf, buf.size, buf, buf.size)
        assert e.value.code == binding.EXT_EINVAL
