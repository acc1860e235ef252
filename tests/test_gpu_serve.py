"""Served form on the GPU: continuous batching over many channels.

Each channel's output from the server must equal the CPU oracle's and the
plain form's on the same input (alone vs in the mix, bit-exact), however the
chunks were cut and interleaved; admission answers EAGAIN and recovers; the
load generator's captured outputs match the plain form channel by channel.
"""
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


def plain(n, m, x, y):
    pairs = (8 * min(x.size, y.size)) // n
    out = np.zeros(max(1, pairs * m // 8), dtype=np.uint8)
    with binding.Extractor(n, m, device_memory=False) as ex:
        ex.extract(np.ascontiguousarray(x), np.ascontiguousarray(y), out, pairs)
    return out[: pairs * m // 8]


def drain(srv, chans, expect_bytes, timeout_s=30.0):
    import time

    got = {c: [] for c in chans}
    have = {c: 0 for c in chans}
    t_end = time.time() + timeout_s
    while any(have[c] < expect_bytes[c] for c in chans):
        assert time.time() < t_end, "server did not return every block"
        for c in chans:
            buf = np.empty(1 << 16, dtype=np.uint8)
            n, _ = srv.poll(c, buf)
            if n:
                got[c].append(buf[:n].copy())
                have[c] += n
    return {c: np.concatenate(got[c]) if got[c] else np.zeros(0, np.uint8) for c in chans}


SHAPES = [(1024, 256, "gaussian"), (8192, 2048, "gaussian"), (2048, 512, "gaussian"),
          (65536, 16384, "ar1"), (480, 96, "gaussian"), (32768, 8192, "gaussian"),
          (5680, 80, "gaussian")]  # the paper's point: 710-byte blocks, 10-byte outputs


def test_server_interleaved_random_chunks(dev):
    """X and Y of six channels cut independently into random byte lengths,
    submissions of all channels interleaved at random, small rings so that
    admission refuses and recovers: every channel's output equals the
    oracle's."""
    rng = np.random.Generator(np.random.PCG64(21))
    streams = []
    for i, (n, m, kind) in enumerate(SHAPES):
        pairs = 3 if n >= 32768 else 25
        streams.append(inputs.plain_workload(n, m, pairs, 300 + 2 * i, 301 + 2 * i, kind=kind))
    with binding.Server(config=binding.server_config(ring_blocks=6)) as srv:
        chans = [srv.open(w.n_bits, w.m_bits) for w in streams]
        outs = {c: [] for c in chans}
        pos = [[0, 0] for _ in streams]
        empty = np.zeros(0, np.uint8)
        todo = list(range(len(streams)))
        refused = 0
        while todo:
            i = int(rng.choice(todo))
            w, c = streams[i], chans[i]
            side = int(rng.integers(0, 2))
            if pos[i][side] == (w.x.size if side == 0 else w.y.size):
                side = 1 - side
            arr = w.x if side == 0 else w.y
            p = pos[i][side]
            k = int(min(arr.size - p, rng.integers(1, 3 * w.n_bits // 8)))
            chunk = arr[p:p + k]
            rc = srv.submit(c, chunk if side == 0 else empty, chunk if side == 1 else empty)
            if rc == binding.EXT_OK:
                pos[i][side] += k
            else:
                refused += 1
            buf = np.empty(1 << 16, dtype=np.uint8)
            got, _ = srv.poll(c, buf)
            if got:
                outs[c].append(buf[:got].copy())
            if pos[i][0] == w.x.size and pos[i][1] == w.y.size:
                todo.remove(i)
        want_bytes = {c: w.n_pairs * w.m_bits // 8 - sum(a.size for a in outs[c])
                      for c, w in zip(chans, streams)}
        rest = drain(srv, chans, want_bytes)
        say("server stats: %s, refused %d" % (srv.stats(), refused))
        assert refused > 0
        for c, w in zip(chans, streams):
            got = np.concatenate(outs[c] + [rest[c]])
            assert np.array_equal(got, oracle.ext_blocks(w.x, w.y, w.n_bits, w.m_bits)), \
                (w.n_bits, w.m_bits)


@pytest.mark.parametrize("split", [1, 0])
def test_server_outputs_equal_plain_form_any_chunking(dev, split):
    """Random chunking of six channels; outputs equal the plain form's.  With
    split = 1 (the default) pairs of the m = 4096 .. 16384 channels are cut
    into slices over several work-groups and combined; with 0 every pair is
    one work-group's."""
    rng = np.random.Generator(np.random.PCG64(22))
    streams = [inputs.plain_workload(n, m, 40 if n < 32768 else 4, 400 + i, 500 + i, kind=kind)
               for i, (n, m, kind) in enumerate(SHAPES)]
    with binding.Server(config=binding.server_config(split_pairs=split)) as srv:
        chans = [srv.open(w.n_bits, w.m_bits) for w in streams]
        for c, w in zip(chans, streams):
            px = py = 0
            while px < w.x.size or py < w.y.size:
                kx = int(min(w.x.size - px, rng.integers(0, 5 * w.n_bits // 8)))
                ky = int(min(w.y.size - py, rng.integers(0, 5 * w.n_bits // 8)))
                assert srv.submit(c, w.x[px:px + kx], w.y[py:py + ky]) == binding.EXT_OK
                px += kx
                py += ky
        outs = drain(srv, chans, {c: w.n_pairs * w.m_bits // 8 for c, w in zip(chans, streams)})
        for c, w in zip(chans, streams):
            assert np.array_equal(outs[c], plain(w.n_bits, w.m_bits, w.x, w.y)), w.n_bits
        st = srv.stats()
        say("server stats: %s" % st)
        assert st["pairs"] == sum(w.n_pairs for w in streams)
        sliced = sum(w.n_pairs for w in streams if w.n_bits >= 32768)
        assert st["split_pairs"] == (sliced if split else 0)


def test_server_admission_and_close(dev):
    n, m = 8192, 2048
    nb = n // 8
    w = inputs.plain_workload(n, m, 20, 61, 62)
    tail = np.arange(100, dtype=np.uint8)
    with binding.Server(config=binding.server_config(ring_blocks=4)) as srv:
        c = srv.open(n, m)
        empty = np.zeros(0, np.uint8)
        # X alone runs ahead until the 4-block ring is full
        sent = 0
        while srv.submit(c, w.x[sent * nb:(sent + 1) * nb], empty) == binding.EXT_OK:
            sent += 1
        assert sent == 4
        # Y catches up; outputs come back; ring space returns after polling
        got = []
        py = 0
        px = sent
        while py < 20:
            if srv.submit(c, empty, w.y[py * nb:(py + 1) * nb]) == binding.EXT_OK:
                py += 1
            if px < 20 and srv.submit(c, w.x[px * nb:(px + 1) * nb], empty) == binding.EXT_OK:
                px += 1
            buf = np.empty(1 << 16, dtype=np.uint8)
            k, _ = srv.poll(c, buf)
            if k:
                got.append(buf[:k].copy())
        rest = drain(srv, [c], {c: 20 * 256 - sum(g.size for g in got)})
        out = np.concatenate(got + [rest[c]])
        assert np.array_equal(out, oracle.ext_blocks(w.x, w.y, n, m))
        assert srv.submit(c, tail, empty) == binding.EXT_OK
        assert srv.close_channel(c) == 8 * tail.size
        with pytest.raises(binding.ExtError):
            srv.submit(c, tail, tail)


def test_load_generator_alone_vs_mix(dev):
    """Poisson chunk arrivals on 12 channels of mixed shapes through the
    server: every channel's captured output equals the plain form on the
    bytes it was fed (pools large enough that they are read once)."""
    specs = [(2048, 512), (4096, 1024), (8192, 2048), (16384, 4096), (32768, 8192),
             (65536, 16384)] * 2
    rate = 150e6  # raw bytes/s, X + Y, all channels
    horizon = 1.3
    chans = []
    for i, (n, m) in enumerate(specs):
        share = rate / len(specs) * horizon / 2 * 2.5  # bytes per side, generous
        pairs = int(share // (n // 8)) + 64
        kind = "ar1" if n == 65536 else "gaussian"
        w = inputs.plain_workload(n, m, pairs, 700 + i, 800 + i, kind=kind)
        chans.append((n, m, w.x, w.y))
    say("load generator: %d channels, %.0f MB/s" % (len(chans), rate / 1e6))
    res, cap = binding.simulate(chans, raw_bytes_per_s=rate, warmup_s=0.3, duration_s=1.0,
                                grace_s=3.0, seed=9, capture=True)
    say("result: %s" % res)
    assert res["blocks_missing"] == 0
    assert not res["admission_gave_up"]
    for (n, m, x, y), c in zip(chans, cap):
        blocks = c.size // (m // 8)
        assert blocks > 0
        nb = n // 8
        assert np.array_equal(c, plain(n, m, x[:blocks * nb], y[:blocks * nb])), (n, m)


def test_load_generator_plain_mode_runs(dev):
    specs = [(2048, 512), (8192, 2048), (65536, 16384)]
    rate = 30e6
    chans = []
    for i, (n, m) in enumerate(specs):
        share = rate / len(specs) * 0.7 / 2 * 2.5  # bytes per side, generous
        w = inputs.plain_workload(n, m, int(share // (n // 8)) + 64, 900 + i, 950 + i)
        chans.append((n, m, w.x, w.y))
    res, cap = binding.simulate(chans, mode=binding.EXT_SIM_PLAIN, raw_bytes_per_s=rate,
                                warmup_s=0.2, duration_s=0.5, grace_s=2.0, seed=3, capture=True)
    say("plain mode: %s" % res)
    assert res["blocks_measured"] > 0
    for (n, m, x, y), c in zip(chans, cap):
        blocks = c.size // (m // 8)
        nb = n // 8
        assert np.array_equal(c, plain(n, m, x[:blocks * nb], y[:blocks * nb]))


def test_close_with_pending_partial_block_while_others_stream(dev):
    """Channels that hold a pending partial block (bytes in the current
    cycle's staging, no complete pair) are opened and closed over and over
    while other channels keep streaming from another thread: the closes
    report the dropped bits, the slots are reused, and the streaming
    channels' outputs still equal the plain form's."""
    import threading

    live = [inputs.plain_workload(2048, 512, 600, 950 + i, 960 + i) for i in range(3)]
    with binding.Server(config=binding.server_config(ring_blocks=32)) as srv:
        chans = [srv.open(w.n_bits, w.m_bits) for w in live]
        stop = threading.Event()
        errors = []

        def feed():
            try:
                nb = 256
                pos = [0] * len(live)
                while not stop.is_set() and any(p < 600 for p in pos):
                    for i, (c, w) in enumerate(zip(chans, live)):
                        if pos[i] >= 600:
                            continue
                        k = min(3, 600 - pos[i])
                        sl = slice(pos[i] * nb, (pos[i] + k) * nb)
                        if srv.submit(c, w.x[sl], w.y[sl]) == binding.EXT_OK:
                            pos[i] += k
            except Exception as e:  # surfaced below
                errors.append(e)

        got = {c: [] for c in chans}
        t = threading.Thread(target=feed)
        t.start()
        closes = 0
        part = inputs.plain_workload(8192, 2048, 1, 970, 971)
        try:
            while t.is_alive() or closes < 40:
                c = srv.open(8192, 2048)
                # 700 of 1024 bytes of X, all of Y: a partial block, no pair
                assert srv.submit(c, part.x[:700], part.y) == binding.EXT_OK
                assert srv.close_channel(c) == 8 * 1024
                closes += 1
                for cc in chans:
                    buf = np.empty(1 << 16, dtype=np.uint8)
                    n, _ = srv.poll(cc, buf)
                    if n:
                        got[cc].append(buf[:n].copy())
        finally:
            stop.set()
            t.join()
        assert not errors, errors
        have = {c: sum(g.size for g in got[c]) for c in chans}
        rest = drain(srv, chans, {c: 600 * 64 - have[c] for c in chans})
    say("closed %d channels holding partial blocks while 3 channels streamed" % closes)
    for c, w in zip(chans, live):
        out = np.concatenate(got[c] + [rest[c]])
        assert np.array_equal(out, plain(w.n_bits, w.m_bits, w.x, w.y))


def test_admission_by_free_device_memory(dev):
    """Channels are admitted by device memory: with a reserve above what the
    device has free every open is refused with EXT_EAGAIN and nothing is
    allocated; under a cap on all rings the fourth channel waits until one
    closes, and the admitted channels' outputs equal the plain form's."""
    import torch

    free, total = torch.cuda.mem_get_info()
    say("device memory: %.1f GiB free of %.1f GiB" % (free / 2**30, total / 2**30))
    with binding.Server(config=binding.server_config(device_reserve_bytes=total + 1)) as srv:
        for n, m in ((2048, 512), (65536, 16384)):
            with pytest.raises(binding.ExtError) as e:
                srv.open(n, m)
            assert e.value.code == binding.EXT_EAGAIN
        st = srv.stats()
        assert st["eagain_mem"] == 2 and st["rings_bytes"] == 0
        assert 0 < st["free_bytes"] <= total
    ring = 2 * 128 * (2048 // 8)  # two rings of 128 blocks of 256 bytes
    cfg = binding.server_config(ring_blocks=128, rings_bytes_cap=3 * ring)
    w = inputs.plain_workload(2048, 512, 100, 990, 991)
    with binding.Server(config=cfg) as srv:
        chans = [srv.open(2048, 512) for _ in range(3)]
        with pytest.raises(binding.ExtError) as e:
            srv.open(2048, 512)
        assert e.value.code == binding.EXT_EAGAIN
        st = srv.stats()
        assert st["eagain_mem"] == 1 and st["rings_bytes"] == 3 * ring
        assert srv.close_channel(chans[1]) == 0
        assert srv.stats()["rings_bytes"] == 2 * ring
        c = srv.open(2048, 512)  # admitted now
        chans = [chans[0], chans[2], c]
        assert srv.stats()["rings_bytes"] == 3 * ring
        for ch in chans:
            assert srv.submit(ch, w.x, w.y) == binding.EXT_OK
        got = drain(srv, chans, {ch: 100 * 64 for ch in chans})
    want = plain(2048, 512, w.x, w.y)
    for ch in chans:
        assert np.array_equal(got[ch], want)
