"""The bit-sliced Karatsuba kernel (EXT_KERNEL_BSK) on the GPU through the C
ABI: outputs against the oracle over every field it takes (512, 1024, 2048
bits), element counts from 1 to 8, pair counts ragged against its 32 pairs
per work-group, a modulus of the caller's, the streaming form; at the
paper-scale block (n = 8192, m = 2048, 65536 pairs) the whole output against
the word-level kernel's and sampled pairs against the oracle; the
refusals."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2402_14607_amd import binding, inputs

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


def run_bsk(dev, x, y, n, m, pairs, taps=None, canary=64):
    import torch

    stream = torch.cuda.current_stream(dev)
    xd = torch.from_numpy(x).to(dev)
    yd = torch.from_numpy(y).to(dev)
    out = torch.full((pairs * m // 8 + canary,), 0xA5, dtype=torch.uint8, device=dev)
    with binding.Extractor(n, m, device_memory=True, kernel=binding.KERNEL_BSK, taps=taps,
                           stream=stream.cuda_stream) as ex:
        assert '"kernel": "bsk"' in ex.describe()
        ex.extract(xd, yd, out, pairs)
        ex.sync()
    res = out.cpu().numpy()
    assert np.all(res[pairs * m // 8:] == 0xA5), "bytes written past the output"
    return res[:pairs * m // 8]


SHAPES = [(m, n_e, pairs) for m in (512, 1024, 2048) for n_e, pairs in
          ((1, 1), (1, 33), (2, 31), (3, 32), (4, 45), (5, 64), (8, 17))]


@pytest.mark.parametrize("m,n_e,pairs", SHAPES, ids=lambda v: str(v))
def test_bsk_against_oracle(dev, m, n_e, pairs):
    n = m * n_e
    w = inputs.plain_workload(n, m, pairs, 100 + n_e, 200 + pairs)
    say("bsk m=%d n_e=%d pairs=%d" % (m, n_e, pairs))
    got = run_bsk(dev, w.x, w.y, n, m, pairs)
    assert np.array_equal(got, oracle.ext_blocks(w.x, w.y, n, m))


def test_bsk_extremes_and_custom_modulus(dev):
    """All-ones and all-zero blocks, one-hot elements, and a pentanomial of
    the caller's (not the conventional one) with every tap at most q/2."""
    m, n_e, pairs = 1024, 3, 40
    n = m * n_e
    nb = n // 8
    rng = np.random.Generator(np.random.PCG64(5))
    x = rng.integers(0, 256, pairs * nb, dtype=np.uint8)
    y = rng.integers(0, 256, pairs * nb, dtype=np.uint8)
    x[:nb] = 0xFF
    y[:nb] = 0xFF
    x[nb:2 * nb] = 0
    y[2 * nb:3 * nb] = 0
    x[3 * nb:4 * nb] = 0
    x[3 * nb] = 1
    x[3 * nb + m // 8 + 5] = 0x80
    taps = None
    for a in range(20, 500):
        cand = (a, 7, 2)
        if binding.is_irreducible(m, cand) and cand != binding.default_modulus(m)[1:-1]:
            taps = cand
            break
    assert taps is not None
    exps = (m,) + taps + (0,)
    say("bsk m=%d custom modulus %r" % (m, exps))
    got = run_bsk(dev, x, y, n, m, pairs, taps=taps)
    assert np.array_equal(got, oracle.ext_blocks(x, y, n, m, exps))
    got = run_bsk(dev, x, y, n, m, pairs)
    assert np.array_equal(got, oracle.ext_blocks(x, y, n, m))


def test_bsk_paper_block_full_against_word_kernel(dev):
    """The benchmark's workload: all 65536 pairs byte for byte equal to the
    word-level kernel's, and sampled pairs (first, last, work-group edges)
    equal to the oracle's."""
    import torch

    w = inputs.paper_block(65536)
    stream = torch.cuda.current_stream(dev)
    xd = torch.from_numpy(w.x).to(dev)
    yd = torch.from_numpy(w.y).to(dev)
    outs = {}
    for kernel in (binding.KERNEL_BSK, binding.KERNEL_WORD):
        out = torch.empty(w.n_pairs * w.m_bits // 8, dtype=torch.uint8, device=dev)
        with binding.Extractor(w.n_bits, w.m_bits, device_memory=True, kernel=kernel,
                               stream=stream.cuda_stream) as ex:
            say("paper block, kernel %s" % ex.describe())
            ex.extract(xd, yd, out, w.n_pairs)
            ex.sync()
        outs[kernel] = out.cpu().numpy()
    assert np.array_equal(outs[binding.KERNEL_BSK], outs[binding.KERNEL_WORD])
    idx = np.asarray([0, 1, 31, 32, 33, 4095, 4096, 65503, 65504, 65535], dtype=np.uint64)
    qb = w.m_bits // 8
    want = oracle.ext_sampled(w.x, w.y, idx, w.n_bits, w.m_bits)
    got = np.concatenate([outs[binding.KERNEL_BSK][int(i) * qb:(int(i) + 1) * qb] for i in idx])
    assert np.array_equal(got, want)


def test_bsk_streaming_form(dev):
    """Streaming with the bit-sliced Karatsuba kernel: chunks of any size,
    host and device memory, equal to the oracle, the tail dropped."""
    import torch

    m, n_e, pairs = 2048, 2, 70
    n = m * n_e
    w = inputs.plain_workload(n, m, pairs, 71, 72)
    want = oracle.ext_blocks(w.x, w.y, n, m)
    rng = np.random.Generator(np.random.PCG64(73))
    for device_memory in (False, True):
        stream = torch.cuda.current_stream(dev).cuda_stream if device_memory else None
        with binding.Extractor(n, m, device_memory=device_memory, kernel=binding.KERNEL_BSK,
                               stream=stream) as ex:
            s = ex.open_stream()
            xs = torch.from_numpy(w.x).to(dev) if device_memory else w.x
            ys = torch.from_numpy(w.y).to(dev) if device_memory else w.y
            got, pos = [], 0
            total = w.x.size - 100  # the last pair incomplete: dropped at close
            buf = (torch.empty(1 << 16, dtype=torch.uint8, device=dev) if device_memory
                   else np.empty(1 << 16, dtype=np.uint8))
            while pos < total:
                c = int(min(total - pos, rng.integers(1, 3 * n // 8)))
                assert s.submit(xs[pos:pos + c], c, ys[pos:pos + c], c) == binding.EXT_OK
                pos += c
                k, _ = s.poll(buf, buf.shape[0])
                if k:
                    got.append((buf[:k].cpu().numpy() if device_memory else buf[:k]).copy())
            while True:
                k, done = s.poll(buf, buf.shape[0], wait=True)
                if not k:
                    break
                got.append((buf[:k].cpu().numpy() if device_memory else buf[:k]).copy())
            dropped = s.close()
        assert dropped == 8 * (n // 8 - 100)
        assert np.array_equal(np.concatenate(got), want[:(pairs - 1) * m // 8])


def test_bsk_refusals(dev):
    """Fields it does not take and a tap above q/2 are EXT_ENOTSUP at create
    time; device inputs off 16-byte boundaries are EXT_EINVAL."""
    import torch

    for n, m in ((4096 * 2, 4096), (256 * 4, 256), (960 * 2, 960)):
        with pytest.raises(binding.ExtError) as e:
            binding.Extractor(n, m, kernel=binding.KERNEL_BSK)
        assert e.value.code == binding.EXT_ENOTSUP
    big_tap = None
    for a in range(300, 511):
        if binding.is_irreducible(512, (a, 2, 1)):
            big_tap = (a, 2, 1)
            break
    if big_tap is not None:
        with pytest.raises(binding.ExtError) as e:
            binding.Extractor(1024, 512, kernel=binding.KERNEL_BSK, taps=big_tap)
        assert e.value.code == binding.EXT_ENOTSUP
    x = torch.zeros(2 * 1024 + 16, dtype=torch.uint8, device=dev)
    out = torch.zeros(2 * 64, dtype=torch.uint8, device=dev)
    with binding.Extractor(1024, 512, device_memory=True, kernel=binding.KERNEL_BSK,
                           stream=torch.cuda.current_stream(dev).cuda_stream) as ex:
        with pytest.raises(binding.ExtError) as e:
            ex.extract(x[4:], x[:-16], out, 2)
        assert e.value.code == binding.EXT_EINVAL


def test_bsk_autotune_choice(dev):
    """With autotune, AUTO times the kernels that take the shape and keeps the
    fastest; the chosen one gives the oracle's bytes."""
    import torch

    n, m, pairs = 8192, 2048, 300
    w = inputs.plain_workload(n, m, pairs, 81, 82)
    stream = torch.cuda.current_stream(dev)
    out = torch.empty(pairs * m // 8, dtype=torch.uint8, device=dev)
    with binding.Extractor(n, m, device_memory=True, autotune=True,
                           stream=stream.cuda_stream) as ex:
        desc = ex.describe()
        say("autotuned: %s" % desc)
        ex.extract(torch.from_numpy(w.x).to(dev), torch.from_numpy(w.y).to(dev), out, pairs)
        ex.sync()
    assert '"kernel": "bsk"' in desc or '"kernel": "word"' in desc
    assert np.array_equal(out.cpu().numpy(), oracle.ext_blocks(w.x, w.y, n, m))
