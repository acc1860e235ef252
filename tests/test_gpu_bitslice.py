"""GPU parity of the bit-sliced kernel (fields of at most 128 bits, 32 block
pairs per work-group, transposed so that one 32-bit word holds one bit of 32
pairs) against the CPU oracle, bit for bit, through the C ABI.

Every case forces the kernel with kernel=EXT_KERNEL_BITSLICE.  Pair counts
are ragged against the 32-pair work-group (1, 31, 32, 33, ...), outputs are
followed by canary bytes, and at the paper's parameter point the whole
262144-pair output must equal the word-level kernel's as well as the oracle
on sampled pairs.
"""
from __future__ import annotations

import json

import numpy as np
import pytest

import oracle
from paper_2402_14607_amd import binding, inputs
from test_gpu_parity import run_stream, say, to_dev

pytestmark = pytest.mark.gpu

BS = binding.KERNEL_BITSLICE


@pytest.fixture(scope="module")
def dev():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    d = torch.device("cuda:0")
    torch.cuda.set_device(d)
    binding.load()
    return d


def run(dev, x, y, n, m, pairs, kernel=BS, taps=None, canary=64):
    import torch

    qb = m // 8
    out = torch.full((pairs * qb + canary,), 0xA5, dtype=torch.uint8, device=dev)
    with binding.Extractor(n, m, device_memory=True, taps=taps, kernel=kernel,
                           stream=torch.cuda.current_stream(dev).cuda_stream) as ex:
        d = json.loads(ex.describe())
        assert d["kernel"] == ("bitslice" if kernel == BS else "word"), d
        ex.extract(to_dev(dev, x), to_dev(dev, y), out, pairs)
        ex.sync()
    got = out.cpu().numpy()
    assert np.all(got[pairs * qb:] == 0xA5), "store past the last pair"
    return got[:pairs * qb]


# every field size the kernel takes (multiples of 8 up to 128), with one
# chunk and with many (a chunk holds at most 128 elements)
SHAPES = [(8, 1), (8, 4), (8, 150), (8, 400), (16, 3), (16, 300), (24, 3), (24, 200), (32, 1),
          (32, 4), (32, 90), (40, 7), (48, 9), (56, 2), (64, 2), (64, 33), (72, 5), (80, 1),
          (80, 4), (80, 71), (88, 5), (96, 3), (104, 9), (112, 2), (120, 6), (128, 1), (128, 4),
          (128, 40)]


@pytest.mark.parametrize("m,n_e", SHAPES, ids=lambda v: str(v))
def test_shapes_full(dev, m, n_e):
    rng = np.random.Generator(np.random.PCG64(5000 + m * 7 + n_e))
    n = m * n_e
    pairs = int(rng.integers(34, 100)) if n_e < 100 else 35
    x = rng.integers(0, 256, pairs * n // 8, dtype=np.uint8)
    y = rng.integers(0, 256, pairs * n // 8, dtype=np.uint8)
    say("bitslice m=%d n_e=%d, %d pairs, full compare" % (m, n_e, pairs))
    got = run(dev, x, y, n, m, pairs)
    assert np.array_equal(got, oracle.ext_blocks(x, y, n, m))


@pytest.mark.parametrize("pairs", [1, 2, 31, 32, 33, 63, 64, 65, 97])
def test_ragged_pair_counts(dev, pairs):
    w = inputs.plain_workload(5680, 80, pairs, 61, 62)
    say("bitslice paper shape, %d pairs" % pairs)
    got = run(dev, w.x, w.y, 5680, 80, pairs)
    assert np.array_equal(got, oracle.ext_blocks(w.x, w.y, 5680, 80))


@pytest.mark.parametrize("off_x,off_y", [(4, 12), (12, 8), (8, 0)])
def test_unaligned_device_pointers(dev, off_x, off_y):
    """x and y 4-byte aligned (the interface's requirement) but off a 16-byte
    boundary: the staging reads the units at the region's ends byte by byte
    and must neither miss nor cross them."""
    import torch

    pairs = 70
    w = inputs.plain_workload(5680, 80, pairs, 65 + off_x, 66 + off_y)
    nb = w.x.size
    bx = torch.full((nb + 32,), 0x5A, dtype=torch.uint8, device=dev)
    by = torch.full((nb + 32,), 0xC3, dtype=torch.uint8, device=dev)
    bx[off_x:off_x + nb] = to_dev(dev, w.x)
    by[off_y:off_y + nb] = to_dev(dev, w.y)
    out = torch.full((pairs * 10 + 16,), 0xA5, dtype=torch.uint8, device=dev)
    say("bitslice unaligned x+%d y+%d" % (off_x, off_y))
    with binding.Extractor(5680, 80, device_memory=True, kernel=BS,
                           stream=torch.cuda.current_stream(dev).cuda_stream) as ex:
        ex.extract(bx[off_x:off_x + nb], by[off_y:off_y + nb], out, pairs)
        ex.sync()
    got = out.cpu().numpy()
    assert np.array_equal(got[:pairs * 10], oracle.ext_blocks(w.x, w.y, 5680, 80))
    assert np.all(got[pairs * 10:] == 0xA5)


def test_extremes(dev):
    """All-zero and all-one blocks and the edge elements 1 and t^(q-1), which
    reach the lowest and the highest product planes."""
    m, n_e = 128, 4
    nb = m * n_e // 8
    one = np.zeros(nb, np.uint8)
    one[0] = 1
    top = np.zeros(nb, np.uint8)
    top[m // 8 - 1] = 0x80
    ff = np.full(nb, 255, np.uint8)
    zz = np.zeros(nb, np.uint8)
    bx = [zz, ff, ff, one, top, top, ff] * 5
    by = [ff, ff, zz, np.full(nb, 0x5A, np.uint8), top, ff, top] * 5
    x, y = np.concatenate(bx), np.concatenate(by)
    got = run(dev, x, y, m * n_e, m, len(bx))
    assert np.array_equal(got, oracle.ext_blocks(x, y, m * n_e, m))


def test_custom_taps(dev):
    """A pentanomial other than the default one (found and checked by the
    oracle), at q = 64 and q = 128."""
    for m in (64, 128):
        taps = None
        for a in range(5, m // 2):
            for b in range(2, a):
                for c in range(1, b):
                    if (a, b, c) != tuple(oracle.modulus(m)[1:4]) and \
                            oracle.is_irreducible(m, (m, a, b, c, 0)):
                        taps = (a, b, c)
                        break
                if taps:
                    break
            if taps:
                break
        rng = np.random.Generator(np.random.PCG64(m))
        n_e, pairs = 3, 45
        x = rng.integers(0, 256, pairs * m * n_e // 8, dtype=np.uint8)
        y = rng.integers(0, 256, pairs * m * n_e // 8, dtype=np.uint8)
        say("bitslice custom taps %r at m=%d" % (taps, m))
        got = run(dev, x, y, m * n_e, m, pairs, taps=taps)
        assert np.array_equal(got, oracle.ext_blocks(x, y, m * n_e, m,
                                                     exps=(m,) + taps + (0,)))


def test_paper_point_equals_word_kernel_and_oracle(dev):
    """The paper's point (n_e = 71, q = 80, 16-bit Gaussian samples, 262144
    pairs in one launch): the two kernels agree on every pair, and sampled
    pairs plus the first 200 agree with the oracle."""
    w = inputs.paper_point()
    say("paper point n=5680 m=80, %d pairs, bitslice vs word kernel" % w.n_pairs)
    got = run(dev, w.x, w.y, 5680, 80, w.n_pairs)
    word = run(dev, w.x, w.y, 5680, 80, w.n_pairs, kernel=binding.KERNEL_WORD)
    if not np.array_equal(got, word):
        k = int(np.nonzero(got != word)[0][0]) // 10
        raise AssertionError("pair %d differs between the kernels" % k)
    rng = np.random.Generator(np.random.PCG64(72))
    idx = np.unique(np.concatenate([[0, 31, 32, w.n_pairs - 33, w.n_pairs - 1],
                                    rng.integers(0, w.n_pairs, 30)])).astype(np.uint64)
    want = oracle.ext_sampled(w.x, w.y, idx, 5680, 80)
    g = np.concatenate([got[int(i) * 10:(int(i) + 1) * 10] for i in idx])
    assert np.array_equal(g, want)
    assert np.array_equal(got[:2000], oracle.ext_blocks(w.x[:200 * 710], w.y[:200 * 710],
                                                        5680, 80))


def test_streaming_form(dev):
    """The streaming form on the bit-sliced kernel, chunks splitting samples
    and blocks anywhere, host and device memory."""
    w = inputs.plain_workload(5680, 80, 70, 43, 44)
    want = oracle.ext_blocks(w.x, w.y, 5680, 80)
    rng = np.random.Generator(np.random.PCG64(10))

    def split(total, maxc):
        out = []
        while total:
            c = int(min(total, rng.integers(1, maxc)))
            out.append(c)
            total -= c
        return out

    for device_memory in (False, True):
        say("bitslice stream, device_memory=%s" % device_memory)
        got, dropped, _ = run_stream(dev, w, split(w.x.size, 3000), split(w.y.size, 9000),
                                     device_memory=device_memory, kernel=BS)
        assert np.array_equal(got, want)
        assert dropped == 0


def test_selection_errors(dev):
    with pytest.raises(binding.ExtError) as e:
        binding.Extractor(136 * 4, 136, kernel=BS)      # q above 128
    assert e.value.code == binding.EXT_ENOTSUP
    # a modulus with a tap above q/2 (the reciprocal of the conventional one
    # of degree 64) needs more than two folding passes: neither kernel takes it
    assert oracle.is_irreducible(64, (64, 63, 61, 60, 0))
    for kernel in (BS, binding.KERNEL_AUTO):
        with pytest.raises(binding.ExtError) as e:
            binding.Extractor(64 * 40, 64, taps=(63, 61, 60), kernel=kernel)
        assert e.value.code == binding.EXT_ENOTSUP, kernel
    with pytest.raises(binding.ExtError) as e:
        binding.Extractor(1024, 256, kernel=3)
    assert e.value.code == binding.EXT_EINVAL
    with binding.Extractor(2048, 256, kernel=binding.KERNEL_AUTO) as ex:
        assert json.loads(ex.describe())["kernel"] == "word"   # q above 128


def test_auto_choice(dev):
    """AUTO takes the bit-sliced kernel at the paper's point and the word
    kernel for few elements; with autotune it times both, and every choice
    gives the oracle's bytes."""
    import torch

    for m, n_e, want in ((80, 71, "bitslice"), (80, 4, "word"), (80, 16, "bitslice"),
                         (128, 40, "word"), (128, 64, "bitslice"), (24, 30, "word"),
                         (24, 40, "bitslice"), (48, 24, "bitslice"), (48, 16, "word")):
        with binding.Extractor(m * n_e, m) as ex:
            assert json.loads(ex.describe())["kernel"] == want, (m, n_e)
    w = inputs.plain_workload(5680, 80, 45, 63, 64)
    with binding.Extractor(5680, 80, device_memory=True, autotune=True,
                           stream=torch.cuda.current_stream(dev).cuda_stream) as ex:
        say("autotuned choice at the paper's point: " + ex.describe())
        out = torch.zeros(45 * 10, dtype=torch.uint8, device=dev)
        ex.extract(to_dev(dev, w.x), to_dev(dev, w.y), out, 45)
        ex.sync()
    assert np.array_equal(out.cpu().numpy(), oracle.ext_blocks(w.x, w.y, 5680, 80))


def test_random_shapes_against_oracle(dev):
    """40 seeded random cases: q any multiple of 8 up to 128, 1 to 160
    elements, 1 to 100 pairs, inputs at 4-byte offsets from a 16-byte
    boundary, canary bytes after the output; full compare with the oracle."""
    import torch

    rng = np.random.Generator(np.random.PCG64(2024))
    for case in range(40):
        m = 8 * int(rng.integers(1, 17))
        n_e = int(rng.integers(1, 161))
        pairs = int(rng.integers(1, 101))
        off_x, off_y = 4 * int(rng.integers(0, 4)), 4 * int(rng.integers(0, 4))
        n = m * n_e
        nb = pairs * n // 8
        x = rng.integers(0, 256, nb, dtype=np.uint8)
        y = rng.integers(0, 256, nb, dtype=np.uint8)
        say("random case %d: m=%d n_e=%d pairs=%d offsets %d/%d" % (case, m, n_e, pairs, off_x, off_y))
        bx = torch.zeros(nb + 32, dtype=torch.uint8, device=dev)
        by = torch.zeros(nb + 32, dtype=torch.uint8, device=dev)
        bx[off_x:off_x + nb] = to_dev(dev, x)
        by[off_y:off_y + nb] = to_dev(dev, y)
        qb = m // 8
        out = torch.full((pairs * qb + 16,), 0xA5, dtype=torch.uint8, device=dev)
        with binding.Extractor(n, m, device_memory=True, kernel=BS,
                               stream=torch.cuda.current_stream(dev).cuda_stream) as ex:
            ex.extract(bx[off_x:off_x + nb], by[off_y:off_y + nb], out, pairs)
            ex.sync()
        got = out.cpu().numpy()
        assert np.array_equal(got[:pairs * qb], oracle.ext_blocks(x, y, n, m)), case
        assert np.all(got[pairs * qb:] == 0xA5), case
