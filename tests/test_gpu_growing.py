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
    # 71 elements of 1024..1328 bits: blocks computed in element slices over
    # several work-groups, then combined
    (71, 1024, 1, 16, 20),
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


# ---------------------------------------------------------------------------
# online form: Algorithm 2 on unbounded sources fed in chunks
# ---------------------------------------------------------------------------
def oracle_blocks_parallel(x, y, n_e, q1, delta_steps, b, k):
    """Outputs of blocks 0..k-1, one oracle call per block on host threads."""
    import concurrent.futures as cf
    import os

    sched = orc_params.schedule(q1, delta_steps, b, n_e, k)

    def one(item):
        start, size, q = item
        lo, hi = start * b // 8, (start + size) * b // 8
        return oracle.ext_blocks(x[lo:hi], y[lo:hi], q * n_e, q)

    threads = max(1, min(16, len(os.sched_getaffinity(0))))
    with cf.ThreadPoolExecutor(threads) as pool:
        return np.concatenate(list(pool.map(one, sched)))


def feed(dev, st, x, y, rng, device_memory, chunk_blocks_bytes, poll_cap=1 << 16):
    """Feed x and y to a growing stream in random chunk sizes (each side its
    own sequence, sometimes both in one call), polling now and then and on
    EXT_EAGAIN; returns (concatenated output, EAGAIN count)."""
    import torch

    if device_memory:
        xs = torch.from_numpy(x).to(dev)
        ys = torch.from_numpy(y).to(dev)
        obuf = torch.empty(poll_cap, dtype=torch.uint8, device=dev)
    else:
        xs, ys = x, y
        obuf = np.empty(poll_cap, dtype=np.uint8)
    outs, px, py, eagain = [], 0, 0, 0

    def poll(wait=False):
        while True:
            n, _ = st.poll(obuf, poll_cap, wait=wait)
            if not n:
                return
            outs.append((obuf[:n].cpu().numpy() if device_memory else obuf[:n]).copy())

    while px < x.size or py < y.size:
        cap = max(2, chunk_blocks_bytes(st))
        cx = int(min(x.size - px, rng.integers(1, cap)))
        cy = int(min(y.size - py, rng.integers(1, cap)))
        mode = int(rng.integers(0, 3))  # 0: X only, 1: Y only, 2: both in one call
        if mode == 0 or cy == 0:
            cy = 0
        if mode == 1 or cx == 0:
            cx = 0
        if cx == 0 and cy == 0:
            continue
        rc = st.submit(xs[px:px + cx] if cx else None, cx, ys[py:py + cy] if cy else None, cy)
        if rc == binding.EXT_EAGAIN:
            eagain += 1
            poll(wait=True)
            continue
        px += cx
        py += cy
        if rng.integers(0, 4) == 0:
            poll()
    poll(wait=True)
    return (np.concatenate(outs) if outs else np.zeros(0, np.uint8)), eagain


GROWING_STREAMS = [  # n_e, q1, Delta, b, blocks -- the first runs q_l past 4096 (to 5184)
    (3, 80, 1, 16, 320),
    (71, 80, 1, 16, 40),
    (4, 64, 2, 8, 120),
    # the paper's 71 elements to q = 1984: from about q = 1100 on, blocks are
    # computed in element slices (beyond about 1800 no single work-group could)
    (71, 80, 1, 16, 120),
]


@pytest.mark.parametrize("n_e,q1,delta_steps,b,k", GROWING_STREAMS, ids=lambda v: str(v))
def test_growing_stream_random_chunks(dev, n_e, q1, delta_steps, b, k):
    sched = orc_params.schedule(q1, delta_steps, b, n_e, k)
    total = sum(size for _, size, _ in sched) * b // 8
    next_block = (q1 + k * delta_steps * b) * n_e // 8
    tail = next_block // 3  # part of block k: pending at the end, dropped at close
    rng = np.random.Generator(np.random.PCG64(4000 + q1 + n_e + k))
    x = rng.integers(0, 256, total + tail, dtype=np.uint8)
    y = rng.integers(0, 256, total + tail, dtype=np.uint8)
    say("growing stream n_e=%d q1=%d delta=%d b=%d: %d blocks (q up to %d), %d bytes per source"
        % (n_e, q1, delta_steps, b, k, sched[-1][2], total + tail))
    want = oracle_blocks_parallel(x, y, n_e, q1, delta_steps, b, k)
    m_k = orc_params.output_bits(q1, delta_steps, b, k)
    assert want.size * 8 == m_k == binding.output_bits(q1, delta_steps, b, k)
    import torch

    # host memory; device memory on the handle's own stream (poll waits for
    # its copies); device memory on torch's current stream (poll's copies are
    # stream-ordered, and feed reads them on that stream)
    for device_memory, on_current in ((False, False), (True, False), (True, True)):
        say("  device_memory=%s, caller's stream=%s" % (device_memory, on_current))
        stream = torch.cuda.current_stream(dev).cuda_stream if on_current else None
        with binding.Growing(n_e, q1, delta_steps, sample_bits=b,
                             device_memory=device_memory, stream=stream) as g:
            st = g.open_stream()

            def chunk_cap(s):
                _, q, _ = s.state()
                return 3 * q * n_e // 8  # up to three blocks of the current size

            got, _ = feed(dev, st, x, y, rng, device_memory, chunk_cap)
            l, q, consumed = st.state()
            dropped = st.close()
        assert l == k and q == q1 + k * delta_steps * b and consumed == total
        assert dropped == 8 * tail
        assert got.size * 8 == m_k
        assert np.array_equal(got, want)


def test_growing_stream_delta_zero_is_algorithm_one(dev):
    """Delta = 0 in small chunks: the plain form's bytes (Algorithm 1)."""
    import torch

    n_e, q, pairs = 71, 80, 300
    rng = np.random.Generator(np.random.PCG64(515))
    x = rng.integers(0, 256, pairs * n_e * q // 8, dtype=np.uint8)
    y = rng.integers(0, 256, pairs * n_e * q // 8, dtype=np.uint8)
    with binding.Growing(n_e, q, 0, sample_bits=16, device_memory=False) as g:
        st = g.open_stream()
        got, _ = feed(dev, st, x, y, rng, False, lambda s: 700)
        assert st.close() == 0
    out = torch.zeros(pairs * q // 8, dtype=torch.uint8, device=dev)
    with binding.Extractor(n_e * q, q, device_memory=True,
                           stream=torch.cuda.current_stream(dev).cuda_stream) as ex:
        ex.extract(torch.from_numpy(x).to(dev), torch.from_numpy(y).to(dev), out, pairs)
        ex.sync()
    assert np.array_equal(got, out.cpu().numpy())


def test_growing_stream_admission(dev):
    """A small device_bytes_cap: one side far ahead is refused with EXT_EAGAIN
    and nothing consumed; the stream still produces every block."""
    n_e, q1, d, b, k = 4, 64, 1, 8, 60
    sched = orc_params.schedule(q1, d, b, n_e, k)
    total = sum(size for _, size, _ in sched) * b // 8
    rng = np.random.Generator(np.random.PCG64(616))
    x = rng.integers(0, 256, total, dtype=np.uint8)
    y = rng.integers(0, 256, total, dtype=np.uint8)
    want = oracle_blocks_parallel(x, y, n_e, q1, d, b, k)
    with binding.Growing(n_e, q1, d, sample_bits=b, device_memory=False,
                         device_bytes_cap=4096) as g:
        st = g.open_stream()
        # all of X at once is more than the cap allows (and than two blocks)
        assert st.submit(x, x.size, None, 0) == binding.EXT_EAGAIN
        assert st.state() == (0, q1, 0)
        got, eagain = feed(dev, st, x, y, rng, False, lambda s: 5000)
        assert st.close() == 0
    assert np.array_equal(got, want)


def test_growing_stream_poll_whole_blocks_and_errors(dev):
    """poll returns whole blocks only (a buffer smaller than the next block's
    output gets nothing); a stream closed before any block drops its bytes."""
    n_e, q1, d, b = 2, 256, 1, 32
    rng = np.random.Generator(np.random.PCG64(717))
    sched = orc_params.schedule(q1, d, b, n_e, 5)
    total = sum(size for _, size, _ in sched) * b // 8
    x = rng.integers(0, 256, total, dtype=np.uint8)
    y = rng.integers(0, 256, total, dtype=np.uint8)
    want = oracle_blocks_parallel(x, y, n_e, q1, d, b, 5)
    with binding.Growing(n_e, q1, d, sample_bits=b, device_memory=False) as g:
        st = g.open_stream()
        assert st.submit(x, x.size, y, y.size) == binding.EXT_OK
        small = np.zeros(q1 // 8 - 1, dtype=np.uint8)
        n, done = st.poll(small, small.size, wait=True)
        assert n == 0 and done == 0
        buf = np.zeros(want.size, dtype=np.uint8)
        n, done = st.poll(buf, buf.size, wait=True)
        assert n == want.size and done == 5
        assert np.array_equal(buf, want)
        assert st.close() == 0
        st2 = g.open_stream()
        assert st2.submit(x[:100], 100, y[:40], 40) == binding.EXT_OK
        assert st2.state() == (0, q1, 0)
        assert st2.close() == 800
