"""GPU parity: the HIP path through the C ABI against the CPU oracle, bit for
bit (exact GF(2) arithmetic, so any difference is a failure).

Small cases are compared in full; the full-size workloads, run in the same
launch configuration the benchmark times (one ext_extract over every pair,
device memory), are compared on sampled pairs that include the first and last
pair and both sides of work-group boundaries, and through properties that
hold at any size (symmetry, independence of the batch split).
"""
from __future__ import annotations

import json

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


def to_dev(dev, arr):
    import torch

    return torch.from_numpy(np.ascontiguousarray(arr)).to(dev)


def gpu_extract(dev, x_np, y_np, n_bits, m_bits, n_pairs=None, taps=None, ex=None):
    import torch

    if n_pairs is None:
        n_pairs = (8 * min(x_np.size, y_np.size)) // n_bits
    x = torch.from_numpy(np.ascontiguousarray(x_np)).to(dev)
    y = torch.from_numpy(np.ascontiguousarray(y_np)).to(dev)
    out = torch.full((max(1, n_pairs * m_bits // 8),), 0xA5, dtype=torch.uint8, device=dev)
    own = ex is None
    if own:
        ex = binding.Extractor(n_bits, m_bits, device_memory=True,
                               stream=torch.cuda.current_stream(dev).cuda_stream, taps=taps)
    try:
        ex.extract(x, y, out, n_pairs)
        ex.sync()
        return out[: n_pairs * m_bits // 8].cpu().numpy()
    finally:
        if own:
            ex.close()


def sample_indices(n_pairs, ppw, rng, extra=24):
    idx = {0, n_pairs - 1, min(1, n_pairs - 1)}
    for b in (ppw - 1, ppw, ppw + 1, n_pairs - ppw - 1, n_pairs - ppw, (n_pairs // ppw) * ppw - 1):
        if 0 <= b < n_pairs:
            idx.add(b)
    idx.update(int(v) for v in rng.integers(0, n_pairs, extra))
    return np.asarray(sorted(idx), dtype=np.uint64)


def compare_sampled(got, w, idx, m_bits):
    want = oracle.ext_sampled(w.x, w.y, idx, w.n_bits, m_bits)
    qb = m_bits // 8
    g = np.concatenate([got[int(i) * qb:(int(i) + 1) * qb] for i in idx])
    if not np.array_equal(g, want):
        k = int(np.nonzero(g != want)[0][0]) // qb
        raise AssertionError("pair %d differs from the oracle" % int(idx[k]))


# ---------------------------------------------------------------------------
def test_modulus_agrees_with_oracle(dev):
    for m in (32, 64, 96, 128, 160, 192, 224, 256, 320, 384, 512, 768, 1024, 1536, 2048,
              4096, 8192, 16384):
        assert binding.default_modulus(m) == oracle.modulus(m), m


def test_tiny_full(dev):
    w = inputs.tiny()
    say("tiny workload: n=1024 m=256, %d pairs, full compare" % w.n_pairs)
    got = gpu_extract(dev, w.x, w.y, w.n_bits, w.m_bits)
    want = oracle.ext_blocks(w.x, w.y, w.n_bits, w.m_bits)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("n_pairs", [1, 2, 8, 9, 10, 37, 100])
def test_paper_block_shape_ragged_full(dev, n_pairs):
    w = inputs.plain_workload(8192, 2048, n_pairs, 11, 12)
    say("n=8192 m=2048, %d pairs, full compare" % n_pairs)
    got = gpu_extract(dev, w.x, w.y, 8192, 2048)
    want = oracle.ext_blocks(w.x, w.y, 8192, 2048)
    assert np.array_equal(got, want)


def test_paper_block_full_size_sampled(dev):
    import torch

    w = inputs.paper_block()
    say("paper block: n=8192 m=2048, %d pairs (bench launch), sampled compare" % w.n_pairs)
    with binding.Extractor(8192, 2048, device_memory=True,
                           stream=torch.cuda.current_stream(dev).cuda_stream) as ex:
        ppw = json.loads(ex.describe())["pairs_per_workgroup"]
        got = gpu_extract(dev, w.x, w.y, 8192, 2048, ex=ex)
        # any-size properties: symmetry, and the same bytes from a split batch
        sym = gpu_extract(dev, w.y, w.x, 8192, 2048, ex=ex)
        assert np.array_equal(got, sym), "Ext(x, y) != Ext(y, x) at full size"
        k = 12345
        nb = 8192 // 8
        part = gpu_extract(dev, w.x[k * nb:], w.y[k * nb:], 8192, 2048, ex=ex)
        assert np.array_equal(got[k * 256:], part), "batch split changes the output"
    rng = np.random.Generator(np.random.PCG64(7))
    compare_sampled(got, w, sample_indices(w.n_pairs, ppw, rng, extra=40), 2048)


def test_forward_block_stress_sampled(dev):
    import torch

    w = inputs.forward_block_stress()
    say("forward-block stress: n=65536 m=16384 AR(1), %d pairs, sampled compare" % w.n_pairs)
    with binding.Extractor(65536, 16384, device_memory=True,
                           stream=torch.cuda.current_stream(dev).cuda_stream) as ex:
        ppw = json.loads(ex.describe())["pairs_per_workgroup"]
        got = gpu_extract(dev, w.x, w.y, 65536, 16384, ex=ex)
    rng = np.random.Generator(np.random.PCG64(8))
    idx = sample_indices(w.n_pairs, ppw, rng, extra=2)
    compare_sampled(got, w, idx, 16384)


def test_forward_block_stress_small_full(dev):
    w = inputs.plain_workload(65536, 16384, 3, 21, 22, kind="ar1")
    say("n=65536 m=16384 AR(1), 3 pairs, full compare")
    got = gpu_extract(dev, w.x, w.y, 65536, 16384)
    assert np.array_equal(got, oracle.ext_blocks(w.x, w.y, 65536, 16384))


# every base-product size and Karatsuba depth the planner can choose
FUZZ_SHAPES = [(32, 1), (32, 4), (64, 2), (96, 3), (128, 4), (160, 2), (192, 5), (224, 1),
               (256, 1), (256, 8), (320, 4), (384, 2), (512, 4), (768, 3), (1024, 4),
               (1024, 1), (1536, 2), (2048, 2), (4096, 4), (8192, 4), (8192, 1)]


@pytest.mark.parametrize("m,n_e", FUZZ_SHAPES, ids=lambda v: str(v))
def test_shapes_full(dev, m, n_e):
    rng = np.random.Generator(np.random.PCG64(1000 + m + n_e))
    n = m * n_e
    pairs = int(rng.integers(1, 40)) if m <= 1024 else 3
    x = rng.integers(0, 256, pairs * n // 8, dtype=np.uint8)
    y = rng.integers(0, 256, pairs * n // 8, dtype=np.uint8)
    say("shape m=%d n_e=%d, %d pairs, full compare" % (m, n_e, pairs))
    got = gpu_extract(dev, x, y, n, m)
    assert np.array_equal(got, oracle.ext_blocks(x, y, n, m))


# deep Karatsuba trees reached with small fixed bases: up to 7 levels take the
# sub-products in the ranked order (by number of sum-of-halves levels), 8 in
# base-3 digit order; a fixed base also keeps the default plan (no latency
# plan) whatever the pair count
RANKED_SHAPES = [(1024, 2, 32), (2048, 2, 64), (2048, 1, 32), (4096, 2, 32), (8192, 1, 32),
                 (1024, 3, 64)]


@pytest.mark.parametrize("m,n_e,base", RANKED_SHAPES, ids=lambda v: str(v))
def test_deep_karatsuba_levels(dev, m, n_e, base):
    import json

    import torch

    rng = np.random.Generator(np.random.PCG64(5000 + m + n_e + base))
    n = m * n_e
    pairs = 3
    x = rng.integers(0, 256, pairs * n // 8, dtype=np.uint8)
    y = rng.integers(0, 256, pairs * n // 8, dtype=np.uint8)
    with binding.Extractor(n, m, device_memory=True, base_bits=base,
                           stream=torch.cuda.current_stream(dev).cuda_stream) as ex:
        plan = json.loads(ex.describe())
        say("m=%d n_e=%d base %d bits: %d levels, %s" % (m, n_e, base, plan["karatsuba_levels"],
                                                      ex.describe()))
        assert plan["base_bits"] == base and "small_launch" not in plan
        got = gpu_extract(dev, x, y, n, m, ex=ex)
    assert np.array_equal(got, oracle.ext_blocks(x, y, n, m))


@pytest.mark.parametrize("m,n_e", [(256, 4), (2048, 4), (1024, 1), (512, 8)],
                         ids=lambda v: str(v))
def test_latency_plan_equals_default_plan(dev, m, n_e):
    """A launch with fewer work-groups than CUs takes the context's latency
    plan (ext_describe's small_launch); its bytes equal the default plan's
    (a context with the base fixed at its default size has no latency plan)
    and the oracle's.  The plan's base is half the default's, or smaller
    while a pair's n_e * 3^levels items fit in one round of the lanes."""
    import json

    import torch

    rng = np.random.Generator(np.random.PCG64(6000 + m + n_e))
    n = m * n_e
    pairs = 37
    x = rng.integers(0, 256, pairs * n // 8, dtype=np.uint8)
    y = rng.integers(0, 256, pairs * n // 8, dtype=np.uint8)
    st = torch.cuda.current_stream(dev).cuda_stream
    with binding.Extractor(n, m, device_memory=True, stream=st) as ex:
        plan = json.loads(ex.describe())
        say("m=%d n_e=%d: %s" % (m, n_e, ex.describe()))
        assert "small_launch" in plan
        assert (pairs + plan["pairs_per_workgroup"] - 1) // plan["pairs_per_workgroup"] < \
            plan["small_launch"]["below_workgroups"]
        small = gpu_extract(dev, x, y, n, m, ex=ex)
        base = plan["base_bits"]
        sl = plan["small_launch"]
        assert sl["element_groups"] == n_e and sl["base_bits"] <= max(32, base // 2)
        fits = lambda levels: n_e * 3 ** levels <= plan["threads"]  # noqa: E731
        if sl["base_bits"] < base // 2:
            assert fits(sl["karatsuba_levels"])
        if sl["base_bits"] > 32 and fits(sl["karatsuba_levels"]):
            assert not fits(sl["karatsuba_levels"] + 1)
    with binding.Extractor(n, m, device_memory=True, stream=st, base_bits=base) as ex:
        assert "small_launch" not in json.loads(ex.describe())
        default = gpu_extract(dev, x, y, n, m, ex=ex)
    assert np.array_equal(small, default)
    assert np.array_equal(small, oracle.ext_blocks(x, y, n, m))


@pytest.mark.parametrize("pairs", [512, 3000, 20000])
def test_latency_plans_by_launch_size(dev, pairs):
    """n = 1024, m = 256: the default plan packs 256 pairs per work-group, so
    launches up to 65279 pairs are below one work-group per CU (256 on
    MI355X) and take a latency plan: the 32-bit base while its launch stays
    within two work-groups per CU (512 pairs: 256 work-groups), the 64-bit
    one at 3000 pairs (429), the half-size 128-bit one at 20000 (953).
    Every launch size gives the default plan's bytes, and sampled pairs the
    oracle's."""
    import json

    import torch

    n, m = 1024, 256
    rng = np.random.Generator(np.random.PCG64(7100 + pairs))
    x = rng.integers(0, 256, pairs * n // 8, dtype=np.uint8)
    y = rng.integers(0, 256, pairs * n // 8, dtype=np.uint8)
    st = torch.cuda.current_stream(dev).cuda_stream
    with binding.Extractor(n, m, device_memory=True, stream=st) as ex:
        plan = json.loads(ex.describe())
        say("pairs=%d: %s" % (pairs, plan))
        assert plan["small_launch"]["bases"] == [128, 64, 32]
        assert plan["small_launch"]["smallest_within_workgroups"] == \
            2 * plan["small_launch"]["below_workgroups"]
        got = gpu_extract(dev, x, y, n, m, ex=ex)
    with binding.Extractor(n, m, device_memory=True, stream=st, base_bits=256) as ex:
        assert "small_launch" not in json.loads(ex.describe())
        default = gpu_extract(dev, x, y, n, m, ex=ex)
    assert np.array_equal(got, default)
    idx = np.unique(np.concatenate([[0, pairs - 1], rng.integers(0, pairs, 30)])).astype(np.uint64)
    want = oracle.ext_sampled(x, y, idx, n, m)
    qb = m // 8
    assert np.array_equal(np.concatenate([got[int(i) * qb:(int(i) + 1) * qb] for i in idx]), want)


# degrees that are not multiples of 32: elements sit at byte (not word)
# offsets, are re-laid out in zero-padded 32-bit slots, and outputs are
# q/8 bytes per pair at byte offsets; and multiples of 32 whose word count
# has an odd part above 15 (544 = 17 words, 1056 = 33 words), computed in
# wider zero-padded slots (18 and 36 words)
PADDED_SHAPES = [(8, 4), (24, 3), (40, 7), (80, 4), (80, 71), (88, 5), (104, 9), (200, 3),
                 (1000, 4), (1016, 2), (544, 3), (1056, 2)]


@pytest.mark.parametrize("m,n_e", PADDED_SHAPES, ids=lambda v: str(v))
def test_padded_shapes_full(dev, m, n_e):
    """Full compare against the oracle, with canary bytes after the output
    (no store may pass the last pair's q/8 bytes)."""
    import torch

    rng = np.random.Generator(np.random.PCG64(3000 + m + n_e))
    n = m * n_e
    pairs = int(rng.integers(1, 40)) if m < 1000 else 3
    x = rng.integers(0, 256, pairs * n // 8, dtype=np.uint8)
    y = rng.integers(0, 256, pairs * n // 8, dtype=np.uint8)
    say("padded shape m=%d n_e=%d, %d pairs, full compare" % (m, n_e, pairs))
    qb = m // 8
    out = torch.full((pairs * qb + 64,), 0xA5, dtype=torch.uint8, device=dev)
    with binding.Extractor(n, m, device_memory=True,
                           stream=torch.cuda.current_stream(dev).cuda_stream) as ex:
        say(ex.describe())
        ex.extract(to_dev(dev, x), to_dev(dev, y), out, pairs)
        ex.sync()
    got = out.cpu().numpy()
    assert np.array_equal(got[:pairs * qb], oracle.ext_blocks(x, y, n, m))
    assert np.all(got[pairs * qb:] == 0xA5)


def test_paper_point_sampled(dev):
    """The paper's parameter point, n_e = 71 elements of F_2^80 over 16-bit
    Gaussian samples, 262144 pairs in one launch: sampled pairs against the
    oracle, plus the first 300 pairs in full."""
    import torch

    w = inputs.paper_point()
    say("paper point n=5680 m=80, %d pairs" % w.n_pairs)
    x, y = to_dev(dev, w.x), to_dev(dev, w.y)
    out = torch.zeros(w.n_pairs * 10, dtype=torch.uint8, device=dev)
    with binding.Extractor(5680, 80, device_memory=True, sample_bits=16,
                           stream=torch.cuda.current_stream(dev).cuda_stream) as ex:
        say(ex.describe())
        ex.extract(x, y, out, w.n_pairs)
        ex.sync()
    got = out.cpu().numpy()
    rng = np.random.Generator(np.random.PCG64(71))
    idx = np.unique(np.concatenate([[0, w.n_pairs - 1],
                                    rng.integers(0, w.n_pairs, 30)])).astype(np.uint64)
    want = oracle.ext_sampled(w.x, w.y, idx, 5680, 80)
    g = np.concatenate([got[int(i) * 10:(int(i) + 1) * 10] for i in idx])
    assert np.array_equal(g, want)
    assert np.array_equal(got[:3000], oracle.ext_blocks(w.x[:300 * 710], w.y[:300 * 710], 5680, 80))


def test_paper_point_streaming_chunks(dev):
    """Streaming form at q = 80 (710-byte blocks) with chunk lengths that
    split samples and blocks anywhere, host and device memory: equal to the
    oracle over the whole stream."""
    w = inputs.plain_workload(5680, 80, 60, 41, 42)
    want = oracle.ext_blocks(w.x, w.y, 5680, 80)
    rng = np.random.Generator(np.random.PCG64(8))

    def split(total, maxc):
        out = []
        while total:
            c = int(min(total, rng.integers(1, maxc)))
            out.append(c)
            total -= c
        return out

    for device_memory in (False, True):
        say("paper-point stream, device_memory=%s" % device_memory)
        got, dropped, _ = run_stream(dev, w, split(w.x.size, 1500), split(w.y.size, 4000),
                                     device_memory=device_memory)
        assert np.array_equal(got, want)
        assert dropped == 0


def test_custom_taps(dev):
    # another irreducible pentanomial of degree 256 (checked by the oracle)
    m, n_e = 256, 4
    taps = None
    for a in range(11, 40):
        for b in range(2, a):
            for c in range(1, b):
                if oracle.is_irreducible(m, (m, a, b, c, 0)):
                    taps = (a, b, c)
                    break
            if taps:
                break
        if taps:
            break
    rng = np.random.Generator(np.random.PCG64(5))
    x = rng.integers(0, 256, 20 * m * n_e // 8, dtype=np.uint8)
    y = rng.integers(0, 256, 20 * m * n_e // 8, dtype=np.uint8)
    say("custom taps %r at m=256" % (taps,))
    got = gpu_extract(dev, x, y, m * n_e, m, taps=taps)
    assert np.array_equal(got, oracle.ext_blocks(x, y, m * n_e, m, exps=(m,) + taps + (0,)))


def test_extremes(dev):
    """All-zero and all-one blocks, and the edge elements (0, 1, t^(q-1))."""
    m, n_e = 2048, 4
    nb = m * n_e // 8
    blocks_x = [np.zeros(nb, np.uint8), np.full(nb, 255, np.uint8), np.full(nb, 255, np.uint8)]
    blocks_y = [np.full(nb, 255, np.uint8), np.full(nb, 255, np.uint8), np.zeros(nb, np.uint8)]
    one = np.zeros(nb, np.uint8)
    one[0] = 1                       # x_1 = 1
    top = np.zeros(nb, np.uint8)
    top[m // 8 - 1] = 0x80           # x_1 = t^(q-1)
    blocks_x += [one, top, top]
    blocks_y += [np.full(nb, 0x5A, np.uint8), top, np.full(nb, 255, np.uint8)]
    x = np.concatenate(blocks_x)
    y = np.concatenate(blocks_y)
    got = gpu_extract(dev, x, y, m * n_e, m)
    assert np.array_equal(got, oracle.ext_blocks(x, y, m * n_e, m))


def test_host_memory_path_equals_device_path(dev):
    w = inputs.plain_workload(8192, 2048, 50, 31, 32)
    with binding.Extractor(8192, 2048, device_memory=False) as ex:
        out = np.zeros(50 * 256, dtype=np.uint8)
        ex.extract(w.x, w.y, out, 50)
    assert np.array_equal(out, oracle.ext_blocks(w.x, w.y, 8192, 2048))


def test_zero_pairs_and_errors(dev):
    import torch

    with binding.Extractor(1024, 256, device_memory=True,
                           stream=torch.cuda.current_stream(dev).cuda_stream) as ex:
        x = torch.zeros(4096, dtype=torch.uint8, device=dev)
        out = torch.full((256,), 7, dtype=torch.uint8, device=dev)
        ex.extract(x, x, out, 0)
        ex.sync()
        assert int(out.sum()) == 7 * 256  # untouched
        with pytest.raises(binding.ExtError) as e:
            ex.extract(x[1:], x, out, 1)  # misaligned
        assert e.value.code == binding.EXT_EINVAL
    with pytest.raises(binding.ExtError) as e:
        binding.Extractor(48, 12, sample_bits=4)  # m not a multiple of 8: not on this path
    assert e.value.code == binding.EXT_ENOTSUP
    with pytest.raises(binding.ExtError) as e:
        binding.Extractor(1000, 256)      # n not a multiple of m
    assert e.value.code == binding.EXT_EINVAL
    with pytest.raises(binding.ExtError) as e:
        binding.Extractor(1024, 256, taps=(4, 3, 2))  # reducible at degree 256
    assert e.value.code == binding.EXT_EINVAL


# ---------------------------------------------------------------------------
# streaming form
# ---------------------------------------------------------------------------
def run_stream(dev, w, chunks_x, chunks_y, device_memory=False, cap=0, poll_every=1,
               combined=True, kernel=0, ctx_shape=None, ctx_taps=None, sample_bits=8):
    """Feed X and Y in the given chunk sizes (in one ext_submit per step when
    combined, else one side per call), poll as it goes, then drain.  With
    ctx_shape = (n, m) the context has that shape and the stream is opened
    with w's own.  Returns (output bytes, dropped bits, EAGAIN count)."""
    import torch

    cn, cm = ctx_shape if ctx_shape else (w.n_bits, w.m_bits)
    ex = binding.Extractor(cn, cm, device_memory=device_memory,
                           stream=torch.cuda.current_stream(dev).cuda_stream if device_memory else None,
                           device_bytes_cap=cap, kernel=kernel, taps=ctx_taps,
                           sample_bits=sample_bits)
    s = ex.open_stream(w.n_bits, w.m_bits) if ctx_shape else ex.open_stream()
    qb = w.m_bits // 8
    collected = []
    xs = torch.from_numpy(w.x).to(dev) if device_memory else w.x
    ys = torch.from_numpy(w.y).to(dev) if device_memory else w.y
    buf = torch.empty(1 << 20, dtype=torch.uint8, device=dev) if device_memory \
        else np.empty(1 << 20, dtype=np.uint8)

    def poll(wait):
        n, _ = s.poll(buf, len(buf) // qb * qb, wait=wait)
        collected.append(buf[:n].cpu().numpy() if device_memory else np.array(buf[:n]))
        return n

    kx = ky = ox = oy = 0
    eagain = stuck = steps = 0
    while kx < len(chunks_x) or ky < len(chunks_y):
        progressed = False
        lx = chunks_x[kx] if kx < len(chunks_x) else 0
        ly = chunks_y[ky] if ky < len(chunks_y) else 0
        sides = [(lx, ly)] if combined else [(lx, 0), (0, ly)]
        for a, b in sides:
            if not a and not b:
                continue
            rc = s.submit(xs[ox:ox + a] if a else None, a, ys[oy:oy + b] if b else None, b)
            if rc == binding.EXT_EAGAIN:
                eagain += 1
                continue
            progressed = True
            if a:
                ox += a
                kx += 1
            if b:
                oy += b
                ky += 1
        steps += 1
        if not progressed:
            poll(True)
            stuck += 1
            assert stuck < 1000, "stream made no progress"
        elif steps % poll_every == 0:
            poll(False)
    while poll(True):
        pass
    dropped = s.close()
    ex.close()
    return np.concatenate(collected) if collected else np.zeros(0, np.uint8), dropped, eagain


def test_stream_chunk_split_invariance(dev):
    w = inputs.plain_workload(1024, 256, 300, 41, 42)
    tail = 77  # bytes of a partial block at the end of X
    w.x = np.concatenate([w.x, np.arange(tail, dtype=np.uint8)])
    want = oracle.ext_blocks(w.x, w.y, 1024, 256)
    rng = np.random.Generator(np.random.PCG64(9))

    def split(total, maxc):
        out = []
        while total:
            c = int(min(total, rng.integers(1, maxc)))
            out.append(c)
            total -= c
        return out

    for device_memory in (False, True):
        for maxc in (2, 300, 5000):
            cx = split(w.x.size, maxc)
            cy = split(w.y.size, maxc * 3)
            say("stream: chunks <= %d (x) / %d (y), device_memory=%s" % (maxc, 3 * maxc, device_memory))
            got, dropped, _ = run_stream(dev, w, cx, cy, device_memory=device_memory,
                                         combined=(maxc != 300))
            assert np.array_equal(got, want)
            assert dropped == 8 * tail


def test_stream_admission_backpressure(dev):
    w = inputs.plain_workload(8192, 2048, 64, 51, 52)
    want = oracle.ext_blocks(w.x, w.y, 8192, 2048)
    nb = 1024
    # X arrives in 3-block chunks, Y in 1-block chunks: X runs ahead until the
    # cap (4 blocks pending) answers EAGAIN, and resumes when Y catches up
    cx = [3 * nb] * 21 + [nb]
    cy = [nb] * 64
    got, dropped, eagain = run_stream(dev, w, cx, cy, cap=4 * nb, poll_every=3, combined=False)
    assert eagain > 0
    assert dropped == 0
    assert np.array_equal(got, want)


# (context n, m, taps), (stream n, m): streams whose shape is not their
# context's -- another field (the conventional modulus of its degree),
# the same field with more elements (the context's own modulus, here a
# non-conventional one), and the paper's point on a bit-sliced-capable shape
STREAM_SHAPES = [((8192, 2048, None), (1024, 256)),
                 ((1024, 256, (16, 3, 1)), (4096, 256)),
                 ((8192, 2048, None), (5680, 80)),
                 ((512, 128, None), (65536, 16384))]


@pytest.mark.parametrize("ctx,shape", STREAM_SHAPES, ids=lambda v: str(v))
def test_stream_shape_of_its_own(dev, ctx, shape):
    n, m = shape
    cn, cm, taps = ctx
    if taps is not None:
        assert binding.is_irreducible(cm, taps)
    pairs = 3 if n >= 65536 else 40
    w = inputs.plain_workload(n, m, pairs, 61, 62)
    tail = 5
    w.x = np.concatenate([w.x, np.arange(tail, dtype=np.uint8)])
    exps = (cm,) + tuple(sorted(taps, reverse=True)) + (0,) if (taps and cm == m) else None
    want = oracle.ext_blocks(w.x, w.y, n, m, exps)
    rng = np.random.Generator(np.random.PCG64(n + m))
    cx, cy = [], []
    for total, out in ((w.x.size, cx), (w.y.size, cy)):
        while total:
            c = int(min(total, rng.integers(1, 3 * n // 8)))
            out.append(c)
            total -= c
    for device_memory in (False, True):
        say("stream n=%d m=%d on a context n=%d m=%d taps=%s, device_memory=%s"
            % (n, m, cn, cm, taps, device_memory))
        got, dropped, _ = run_stream(dev, w, cx, cy, device_memory=device_memory,
                                     ctx_shape=(cn, cm), ctx_taps=taps)
        assert np.array_equal(got, want)
        assert dropped == 8 * tail


def test_stream_shape_refusals(dev):
    with binding.Extractor(8192, 2048, device_memory=False) as ex:
        for n, m, code in ((1000, 256, binding.EXT_EINVAL), (48, 12, binding.EXT_EINVAL),
                           (1024, 8, binding.EXT_OK)):
            if code == binding.EXT_OK:
                ex.open_stream(n, m).close()
                continue
            with pytest.raises(binding.ExtError) as e:
                ex.open_stream(n, m)
            assert e.value.code == code, (n, m)
