"""Thin ctypes binding of libqrngext.so (include/qrng_ext.h).

Argument marshalling only: every step of the extraction runs in the HIP
library.  PyTorch supplies device memory (tensors) and streams
(``torch.cuda.current_stream()``).  If the library is not built, loading
fails with an error -- there is no other implementation to fall back to.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libqrngext.so")

EXT_OK = 0
EXT_EINVAL = -1
EXT_ENOTSUP = -2
EXT_ENOMEM = -3
EXT_EAGAIN = -4
EXT_EDEVICE = -5
EXT_ECLOSED = -6

EXT_MEM_HOST = 0
EXT_MEM_DEVICE = 1

EXPORTED = (
    "ext_params_init", "ext_create", "ext_destroy", "ext_get_modulus", "ext_default_modulus",
    "ext_is_irreducible", "ext_extract", "ext_sync", "ext_stream_open", "ext_submit",
    "ext_poll", "ext_drain", "ext_stream_close", "ext_describe", "ext_strerror",
    "ext_batch_create", "ext_batch_run", "ext_batch_sync", "ext_batch_describe",
    "ext_batch_destroy", "ext_server_config_init", "ext_server_create", "ext_server_open",
    "ext_server_submit", "ext_server_poll", "ext_server_close", "ext_server_stats_get",
    "ext_server_destroy", "ext_serve_simulate", "ext_server_ready",
    "ext_choose_params", "ext_block_error_log2", "ext_stream_error_log2", "ext_output_bits",
    "ext_growing_create", "ext_growing_blocks", "ext_growing_extract",
    "ext_growing_extract_noalloc", "ext_growing_destroy", "ext_growing_open",
    "ext_growing_submit", "ext_growing_poll", "ext_growing_drain", "ext_growing_state",
    "ext_growing_close",
    "ext_probe_valu_rate",
)

EXT_SIM_SERVED = 0
KERNEL_AUTO, KERNEL_WORD, KERNEL_BITSLICE = 0, 1, 2
EXT_SIM_PLAIN = 1


class ExtError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        super().__init__("%s: %s (%d)" % (what, strerror(code), code))


class ExtParams(ctypes.Structure):
    _fields_ = [
        ("sample_bits", ctypes.c_uint32),
        ("n_taps", ctypes.c_uint32),
        ("taps", ctypes.c_uint32 * 3),
        ("mem_kind", ctypes.c_uint32),
        ("hip_stream", ctypes.c_void_p),
        ("use_hip_stream", ctypes.c_uint32),
        ("device_bytes_cap", ctypes.c_uint64),
        ("device", ctypes.c_int32),
        ("base_bits", ctypes.c_uint32),
        ("groups", ctypes.c_uint32),
        ("pairs_per_group", ctypes.c_uint32),
        ("autotune", ctypes.c_uint32),
        ("threads", ctypes.c_uint32),
        ("kernel", ctypes.c_uint32),
        ("reserved", ctypes.c_uint32 * 2),
    ]


class BatchItem(ctypes.Structure):
    _fields_ = [
        ("n_bits", ctypes.c_uint64),
        ("m_bits", ctypes.c_uint32),
        ("reserved", ctypes.c_uint32),
        ("x", ctypes.c_void_p),
        ("y", ctypes.c_void_p),
        ("out", ctypes.c_void_p),
        ("n_pairs", ctypes.c_uint64),
    ]


class ServerConfig(ctypes.Structure):
    _fields_ = [
        ("max_channels", ctypes.c_uint32),
        ("ring_blocks", ctypes.c_uint32),
        ("stage_bytes", ctypes.c_uint64),
        ("outbox_bytes", ctypes.c_uint64),
        ("max_tiles", ctypes.c_uint32),
        ("max_descs", ctypes.c_uint32),
        ("poll_us", ctypes.c_uint32),
        ("wg_per_cu", ctypes.c_uint32),
        ("ring_bytes", ctypes.c_uint64),
        ("max_inflight", ctypes.c_uint32),
        ("split_pairs", ctypes.c_uint32),
        ("timing", ctypes.c_uint32),
        ("reserved", ctypes.c_uint32),
        ("device_reserve_bytes", ctypes.c_uint64),
        ("rings_bytes_cap", ctypes.c_uint64),
    ]


class ServerStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in
                ("cycles", "tiles", "pairs", "bytes_in", "eagain_ring", "eagain_stage",
                 "gpu_busy_ns", "split_pairs", "build_ns", "launch_ns", "max_cycle_ns",
                 "gpu_ns", "stage_ns", "extract_ns", "eagain_mem", "rings_bytes",
                 "free_bytes")]


class SimConfig(ctypes.Structure):
    _fields_ = [
        ("n_channels", ctypes.c_uint32),
        ("mode", ctypes.c_uint32),
        ("n_bits", ctypes.POINTER(ctypes.c_uint64)),
        ("m_bits", ctypes.POINTER(ctypes.c_uint32)),
        ("pool_x", ctypes.POINTER(ctypes.c_void_p)),
        ("pool_y", ctypes.POINTER(ctypes.c_void_p)),
        ("pool_bytes", ctypes.POINTER(ctypes.c_uint64)),
        ("raw_bytes_per_s", ctypes.c_double),
        ("min_chunk_blocks", ctypes.c_uint32),
        ("max_chunk_blocks", ctypes.c_uint32),
        ("warmup_s", ctypes.c_double),
        ("duration_s", ctypes.c_double),
        ("grace_s", ctypes.c_double),
        ("max_lag_s", ctypes.c_double),
        ("seed", ctypes.c_uint64),
        ("producer_threads", ctypes.c_uint32),
        ("reserved0", ctypes.c_uint32),
        ("capture", ctypes.POINTER(ctypes.c_void_p)),
        ("capture_cap", ctypes.POINTER(ctypes.c_uint64)),
        ("server_cfg", ctypes.POINTER(ServerConfig)),
        ("params", ctypes.POINTER(ExtParams)),
    ]


class SimResult(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in
                ("window_s", "out_gbps", "in_gbps", "offered_in_gbps", "lat_p50_us",
                 "lat_p99_us", "lat_max_us", "lat_mean_us")] + \
               [(n, ctypes.c_uint64) for n in ("blocks_measured", "blocks_missing", "chunks",
                                               "eagain")] + \
               [("max_submit_lag_us", ctypes.c_double), ("cycles", ctypes.c_uint64),
                ("eagain_ring", ctypes.c_uint64), ("eagain_stage", ctypes.c_uint64),
                ("mean_cycle_us", ctypes.c_double), ("submit_lag_p99_us", ctypes.c_double),
                ("service_p50_us", ctypes.c_double), ("service_p99_us", ctypes.c_double),
                ("ready_p50_us", ctypes.c_double), ("ready_p99_us", ctypes.c_double),
                ("mean_build_us", ctypes.c_double), ("mean_launch_us", ctypes.c_double),
                ("max_cycle_us", ctypes.c_double), ("mean_gpu_us", ctypes.c_double),
                ("mean_tiles", ctypes.c_double), ("mean_stage_us", ctypes.c_double),
                ("mean_extract_us", ctypes.c_double), ("rings_bytes", ctypes.c_uint64),
                ("free_bytes", ctypes.c_uint64), ("eagain_mem", ctypes.c_uint64)]


_lib = None


def load() -> ctypes.CDLL:
    """Load libqrngext.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libqrngext.so is not built; run __graft_entry__.build() "
                          "or python -m paper_2402_14607_amd.build")
    lib = ctypes.CDLL(LIB_PATH)
    vp, u32, u64, sz = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_size_t
    u32p = ctypes.POINTER(u32)
    u64p = ctypes.POINTER(u64)
    szp = ctypes.POINTER(sz)
    sig = {
        "ext_params_init": (None, [ctypes.POINTER(ExtParams)]),
        "ext_create": (ctypes.c_int, [u64, u32, ctypes.POINTER(ExtParams), ctypes.POINTER(vp)]),
        "ext_destroy": (ctypes.c_int, [vp]),
        "ext_get_modulus": (ctypes.c_int, [vp, u32p, u32, u32p]),
        "ext_default_modulus": (ctypes.c_int, [u32, u32p, u32, u32p]),
        "ext_is_irreducible": (ctypes.c_int, [u32, u32p, u32]),
        "ext_extract": (ctypes.c_int, [vp, vp, vp, u64, vp]),
        "ext_sync": (ctypes.c_int, [vp]),
        "ext_stream_open": (ctypes.c_int, [vp, ctypes.c_uint64, ctypes.c_uint32,
                                           ctypes.POINTER(vp)]),
        "ext_submit": (ctypes.c_int, [vp, vp, sz, vp, sz, u64p]),
        "ext_poll": (ctypes.c_int, [vp, vp, sz, szp, u64p]),
        "ext_drain": (ctypes.c_int, [vp, vp, sz, szp, u64p]),
        "ext_stream_close": (ctypes.c_int, [vp, u64p]),
        "ext_describe": (ctypes.c_int, [vp, ctypes.c_char_p, sz]),
        "ext_strerror": (ctypes.c_char_p, [ctypes.c_int]),
        "ext_batch_create": (ctypes.c_int, [ctypes.POINTER(BatchItem), u32,
                                            ctypes.POINTER(ExtParams), ctypes.POINTER(vp)]),
        "ext_batch_run": (ctypes.c_int, [vp]),
        "ext_batch_sync": (ctypes.c_int, [vp]),
        "ext_batch_describe": (ctypes.c_int, [vp, ctypes.c_char_p, sz]),
        "ext_batch_destroy": (ctypes.c_int, [vp]),
        "ext_server_config_init": (None, [ctypes.POINTER(ServerConfig)]),
        "ext_server_create": (ctypes.c_int, [ctypes.POINTER(ServerConfig), ctypes.POINTER(ExtParams),
                                             ctypes.POINTER(vp)]),
        "ext_server_open": (ctypes.c_int, [vp, u64, u32, ctypes.POINTER(u32)]),
        "ext_server_submit": (ctypes.c_int, [vp, u32, vp, sz, vp, sz]),
        "ext_server_poll": (ctypes.c_int, [vp, u32, vp, sz, szp, u64p, u64p]),
        "ext_server_close": (ctypes.c_int, [vp, u32, u64p]),
        "ext_server_ready": (ctypes.c_int, [vp, ctypes.POINTER(u32), u32, ctypes.POINTER(u32), u32]),
        "ext_choose_params": (ctypes.c_int, [u32, u64, u64, ctypes.c_double, ctypes.c_double,
                                             ctypes.POINTER(u32), ctypes.POINTER(u32)]),
        "ext_block_error_log2": (ctypes.c_double, [u32, u32, ctypes.c_double]),
        "ext_stream_error_log2": (ctypes.c_int, [u32, u32, u32, u32, ctypes.c_double, u64,
                                                 ctypes.POINTER(ctypes.c_double),
                                                 ctypes.POINTER(ctypes.c_double)]),
        "ext_output_bits": (ctypes.c_int, [u32, u32, u32, u64, u64p]),
        "ext_growing_create": (ctypes.c_int, [u32, u32, u32, ctypes.POINTER(ExtParams),
                                              ctypes.POINTER(vp)]),
        "ext_growing_blocks": (ctypes.c_int, [vp, u64, u64p, u64p, u64p]),
        "ext_growing_extract": (ctypes.c_int, [vp, vp, vp, u64, u64, vp, u64, u64p]),
        "ext_growing_extract_noalloc": (ctypes.c_int, [vp, vp, vp, u64, u64, vp, u64, u64p]),
        "ext_growing_destroy": (ctypes.c_int, [vp]),
        "ext_growing_open": (ctypes.c_int, [vp, ctypes.POINTER(vp)]),
        "ext_growing_submit": (ctypes.c_int, [vp, vp, sz, vp, sz, u64p]),
        "ext_growing_poll": (ctypes.c_int, [vp, vp, sz, szp, u64p]),
        "ext_growing_drain": (ctypes.c_int, [vp, vp, sz, szp, u64p]),
        "ext_growing_state": (ctypes.c_int, [vp, u64p, u64p, u64p]),
        "ext_growing_close": (ctypes.c_int, [vp, u64p]),
        "ext_probe_valu_rate": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(ctypes.c_double)]),
        "ext_server_stats_get": (ctypes.c_int, [vp, ctypes.POINTER(ServerStats)]),
        "ext_server_destroy": (ctypes.c_int, [vp]),
        "ext_serve_simulate": (ctypes.c_int, [ctypes.POINTER(SimConfig), ctypes.POINTER(SimResult),
                                              u64p]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def strerror(code: int) -> str:
    try:
        return load().ext_strerror(code).decode()
    except ImportError:
        return "status %d" % code


def _check(rc: int, what: str) -> int:
    if rc < 0:
        raise ExtError(rc, what)
    return rc


def default_modulus(m_bits: int) -> tuple:
    lib = load()
    exps = (ctypes.c_uint32 * 8)()
    n = ctypes.c_uint32()
    _check(lib.ext_default_modulus(m_bits, exps, 8, ctypes.byref(n)), "ext_default_modulus")
    return tuple(int(exps[i]) for i in range(n.value))


def is_irreducible(m_bits: int, taps) -> bool:
    lib = load()
    arr = (ctypes.c_uint32 * 3)(*taps)
    return bool(_check(lib.ext_is_irreducible(m_bits, arr, len(taps)), "ext_is_irreducible"))


def _ptr(buf) -> int:
    """Raw address of a torch tensor or numpy array (an int is taken as an
    address already)."""
    if isinstance(buf, int):
        return buf
    if hasattr(buf, "data_ptr"):
        return buf.data_ptr()
    if isinstance(buf, np.ndarray):
        return buf.ctypes.data
    raise TypeError("expected a torch tensor or numpy array, got %r" % type(buf))


def make_params(lib, *, device_memory=True, stream=None, taps=None, sample_bits=8,
                device_bytes_cap=0, device=-1, autotune=False, base_bits=0, groups=0,
                pairs_per_group=0, threads=0, kernel=0) -> ExtParams:
    p = ExtParams()
    lib.ext_params_init(ctypes.byref(p))
    p.sample_bits = sample_bits
    p.mem_kind = EXT_MEM_DEVICE if device_memory else EXT_MEM_HOST
    if taps:
        p.n_taps = len(taps)
        for i, t in enumerate(taps):
            p.taps[i] = int(t)
    if stream is not None:
        p.hip_stream = ctypes.c_void_p(int(stream))
        p.use_hip_stream = 1
    if device_bytes_cap:
        p.device_bytes_cap = device_bytes_cap
    p.device = device
    p.autotune = 1 if autotune else 0
    p.base_bits = base_bits
    p.groups = groups
    p.pairs_per_group = pairs_per_group
    p.kernel = kernel
    p.threads = threads
    return p


class Extractor:
    """One ext_ctx: block length n_bits, m_bits output bits per block pair."""

    def __init__(self, n_bits: int, m_bits: int, *, device_memory: bool = True, stream=None,
                 taps=None, sample_bits: int = 8, device_bytes_cap: int = 0, device: int = -1,
                 autotune: bool = False, base_bits: int = 0, groups: int = 0,
                 pairs_per_group: int = 0, threads: int = 0, kernel: int = 0):
        self.lib = load()
        p = make_params(self.lib, device_memory=device_memory, stream=stream, taps=taps,
                        sample_bits=sample_bits, device_bytes_cap=device_bytes_cap,
                        device=device, autotune=autotune, base_bits=base_bits, groups=groups,
                        pairs_per_group=pairs_per_group, threads=threads, kernel=kernel)
        self.n_bits = n_bits
        self.m_bits = m_bits
        self.device_memory = device_memory
        self.handle = ctypes.c_void_p()
        _check(self.lib.ext_create(n_bits, m_bits, ctypes.byref(p), ctypes.byref(self.handle)),
               "ext_create")

    def close(self):
        if self.handle:
            self.lib.ext_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def modulus(self) -> tuple:
        exps = (ctypes.c_uint32 * 8)()
        n = ctypes.c_uint32()
        _check(self.lib.ext_get_modulus(self.handle, exps, 8, ctypes.byref(n)), "ext_get_modulus")
        return tuple(int(exps[i]) for i in range(n.value))

    def describe(self) -> str:
        buf = ctypes.create_string_buffer(1024)
        _check(self.lib.ext_describe(self.handle, buf, 1024), "ext_describe")
        return buf.value.decode()

    def extract(self, x, y, out, n_pairs: int) -> None:
        """Queue (device memory) or run (host memory) the plain form."""
        _check(self.lib.ext_extract(self.handle, _ptr(x), _ptr(y), n_pairs, _ptr(out)),
               "ext_extract")

    def sync(self) -> None:
        _check(self.lib.ext_sync(self.handle), "ext_sync")

    def open_stream(self, n_bits: int = 0, m_bits: int = 0) -> "Stream":
        """A stream of the context's shape, or of its own (n_bits, m_bits)."""
        return Stream(self, n_bits, m_bits)


class Stream:
    """One ext_stream (an (X, Y) channel pair) of an Extractor; n_bits and
    m_bits of 0 take the Extractor's shape."""

    def __init__(self, ex: Extractor, n_bits: int = 0, m_bits: int = 0):
        self.ex = ex
        self.lib = ex.lib
        self.handle = ctypes.c_void_p()
        self.n_bits = n_bits or ex.n_bits
        self.m_bits = m_bits or ex.m_bits
        _check(self.lib.ext_stream_open(ex.handle, n_bits, m_bits, ctypes.byref(self.handle)),
               "ext_stream_open")

    def submit(self, x, x_len: int, y, y_len: int) -> int:
        """Returns EXT_OK or EXT_EAGAIN; raises on other errors."""
        seq = ctypes.c_uint64()
        xp = _ptr(x) if x_len else None
        yp = _ptr(y) if y_len else None
        rc = self.lib.ext_submit(self.handle, xp, x_len, yp, y_len, ctypes.byref(seq))
        if rc == EXT_EAGAIN:
            return rc
        _check(rc, "ext_submit")
        return rc

    def poll(self, out, out_cap: int, wait: bool = False):
        """(bytes written, blocks returned so far)."""
        n = ctypes.c_size_t()
        done = ctypes.c_uint64()
        f = self.lib.ext_drain if wait else self.lib.ext_poll
        _check(f(self.handle, _ptr(out) if out_cap else None, out_cap, ctypes.byref(n),
                 ctypes.byref(done)), "ext_poll")
        return n.value, done.value

    def close(self) -> int:
        """Closes the stream; returns the dropped tail in bits."""
        if not self.handle:
            return 0
        dropped = ctypes.c_uint64()
        _check(self.lib.ext_stream_close(self.handle, ctypes.byref(dropped)), "ext_stream_close")
        self.handle = ctypes.c_void_p()
        return dropped.value


class Batch:
    """One ext_batch: many (x, y, out) device-memory stream pairs with their
    own n_bits and m_bits, run by one persistent launch per base size."""

    def __init__(self, items, *, stream=None, autotune=False, base_bits=0, device=-1):
        """items: iterable of (n_bits, m_bits, x, y, out, n_pairs) with torch
        device tensors (kept alive by this object)."""
        self.lib = load()
        self._keep = []
        arr = (BatchItem * max(1, len(items)))()
        for i, (n, m, x, y, out, n_pairs) in enumerate(items):
            arr[i].n_bits = n
            arr[i].m_bits = m
            arr[i].x = _ptr(x)
            arr[i].y = _ptr(y)
            arr[i].out = _ptr(out)
            arr[i].n_pairs = n_pairs
            self._keep.append((x, y, out))
        p = make_params(self.lib, device_memory=True, stream=stream, autotune=autotune,
                        base_bits=base_bits, device=device)
        self.handle = ctypes.c_void_p()
        _check(self.lib.ext_batch_create(arr, len(items), ctypes.byref(p), ctypes.byref(self.handle)),
               "ext_batch_create")

    def run(self):
        _check(self.lib.ext_batch_run(self.handle), "ext_batch_run")

    def sync(self):
        _check(self.lib.ext_batch_sync(self.handle), "ext_batch_sync")

    def describe(self) -> str:
        buf = ctypes.create_string_buffer(4096)
        _check(self.lib.ext_batch_describe(self.handle, buf, 4096), "ext_batch_describe")
        return buf.value.decode()

    def close(self):
        if self.handle:
            self.lib.ext_batch_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def server_config(**kw) -> ServerConfig:
    lib = load()
    c = ServerConfig()
    lib.ext_server_config_init(ctypes.byref(c))
    names = {f for f, _ in ServerConfig._fields_}
    for k, v in kw.items():
        if k not in names or k == "reserved":
            raise TypeError("ext_server_config has no field %r" % k)
        setattr(c, k, v)
    return c


class Server:
    """One ext_server (continuous batching over many channels).  Host-memory
    numpy arrays in and out."""

    def __init__(self, *, config: ServerConfig | None = None, autotune=False, device=-1):
        self.lib = load()
        self.cfg = config or server_config()
        p = make_params(self.lib, device_memory=False, autotune=autotune, device=device)
        self.handle = ctypes.c_void_p()
        _check(self.lib.ext_server_create(ctypes.byref(self.cfg), ctypes.byref(p),
                                          ctypes.byref(self.handle)), "ext_server_create")

    def open(self, n_bits: int, m_bits: int) -> int:
        ch = ctypes.c_uint32()
        _check(self.lib.ext_server_open(self.handle, n_bits, m_bits, ctypes.byref(ch)),
               "ext_server_open")
        return ch.value

    def submit(self, ch: int, x: np.ndarray, y: np.ndarray) -> int:
        x = np.ascontiguousarray(x, dtype=np.uint8)
        y = np.ascontiguousarray(y, dtype=np.uint8)
        rc = self.lib.ext_server_submit(self.handle, ch, x.ctypes.data if x.size else None, x.size,
                                        y.ctypes.data if y.size else None, y.size)
        if rc == EXT_EAGAIN:
            return rc
        return _check(rc, "ext_server_submit")

    def poll(self, ch: int, out: np.ndarray):
        n = ctypes.c_size_t()
        done = ctypes.c_uint64()
        _check(self.lib.ext_server_poll(self.handle, ch, out.ctypes.data, out.size, ctypes.byref(n),
                                        None, ctypes.byref(done)), "ext_server_poll")
        return n.value, done.value

    def close_channel(self, ch: int) -> int:
        d = ctypes.c_uint64()
        _check(self.lib.ext_server_close(self.handle, ch, ctypes.byref(d)), "ext_server_close")
        return d.value

    def stats(self) -> dict:
        st = ServerStats()
        _check(self.lib.ext_server_stats_get(self.handle, ctypes.byref(st)), "ext_server_stats_get")
        return {n: getattr(st, n) for n, _ in ServerStats._fields_ if n != "reserved"}

    def close(self):
        if self.handle:
            self.lib.ext_server_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def simulate(channels, *, mode=EXT_SIM_SERVED, raw_bytes_per_s, min_chunk=1, max_chunk=64,
             warmup_s=1.0, duration_s=5.0, grace_s=2.0, max_lag_s=0.0, seed=4, capture=False,
             producer_threads=4,
             config: ServerConfig | None = None, autotune=False):
    """Run the load generator.  channels: list of (n_bits, m_bits, pool_x, pool_y)
    with uint8 numpy pools, each read cyclically from its start.  capture: False,
    True (every channel) or the indices of the channels whose whole output is
    kept.  Returns (result dict, per-channel captured outputs (None for a
    channel not captured) or None)."""
    lib = load()
    n = len(channels)
    nbits = (ctypes.c_uint64 * n)(*[c[0] for c in channels])
    mbits = (ctypes.c_uint32 * n)(*[c[1] for c in channels])
    pools = [(np.ascontiguousarray(c[2], dtype=np.uint8), np.ascontiguousarray(c[3], dtype=np.uint8))
             for c in channels]
    px = (ctypes.c_void_p * n)(*[p[0].ctypes.data for p in pools])
    py = (ctypes.c_void_p * n)(*[p[1].ctypes.data for p in pools])
    plen = (ctypes.c_uint64 * n)(*[min(p[0].size, p[1].size) for p in pools])
    cfg = SimConfig()
    cfg.n_channels = n
    cfg.mode = mode
    cfg.n_bits = nbits
    cfg.m_bits = mbits
    cfg.pool_x = px
    cfg.pool_y = py
    cfg.pool_bytes = plen
    cfg.raw_bytes_per_s = raw_bytes_per_s
    cfg.min_chunk_blocks = min_chunk
    cfg.max_chunk_blocks = max_chunk
    cfg.warmup_s = warmup_s
    cfg.duration_s = duration_s
    cfg.grace_s = grace_s
    cfg.max_lag_s = max_lag_s
    cfg.seed = seed
    cfg.producer_threads = producer_threads
    caps = None
    if capture is not False and capture is not None:
        # capture=True: every channel; else an iterable of channel indices
        which = set(range(n)) if capture is True else {int(c) for c in capture}
        bufs = []
        for i, (nb_, mb_, _, _) in enumerate(channels):
            if i not in which:
                bufs.append(None)
                continue
            # generous: every chunk of the horizon at the channel's share of the rate
            share = (raw_bytes_per_s / n * (warmup_s + duration_s + grace_s) * 3.0
                     + 64 * nb_ // 8 * 4)
            bufs.append(np.zeros(int(share * mb_ / (2 * nb_)) + 1024, dtype=np.uint8))
        caps = bufs
        cfg.capture = (ctypes.c_void_p * n)(*[b.ctypes.data if b is not None else None
                                              for b in bufs])
        cfg.capture_cap = (ctypes.c_uint64 * n)(*[b.size if b is not None else 0 for b in bufs])
    sc = config or server_config()
    cfg.server_cfg = ctypes.pointer(sc)
    p = make_params(lib, device_memory=False, autotune=autotune)
    cfg.params = ctypes.pointer(p)
    res = SimResult()
    clen = (ctypes.c_uint64 * n)()
    rc = lib.ext_serve_simulate(ctypes.byref(cfg), ctypes.byref(res), clen)
    if rc not in (EXT_OK, EXT_EAGAIN):
        raise ExtError(rc, "ext_serve_simulate")
    out = {n_: getattr(res, n_) for n_, _ in SimResult._fields_ if n_ != "reserved"}
    out["admission_gave_up"] = rc == EXT_EAGAIN
    captured = ([b[: clen[i]] if b is not None else None for i, b in enumerate(caps)]
                if caps is not None else None)
    return out, captured


# ---------------------------------------------------------------------------
# parameters and security bounds (host only)
# ---------------------------------------------------------------------------
def choose_params(sample_bits: int, delta_num: int, delta_den: int, log2_n_samples: float,
                  log2_eps: float) -> tuple[int, int]:
    """Algorithm 1's (n_e, q) for min-entropy rate delta_num/delta_den."""
    lib = load()
    n_e, q = ctypes.c_uint32(), ctypes.c_uint32()
    _check(lib.ext_choose_params(sample_bits, delta_num, delta_den, float(log2_n_samples),
                                 float(log2_eps), ctypes.byref(n_e), ctypes.byref(q)),
           "ext_choose_params")
    return n_e.value, q.value


def block_error_log2(n_e: int, q: int, delta: float) -> float:
    """log2 of Theorem 3.3's bound for one block."""
    return load().ext_block_error_log2(n_e, q, float(delta))


def stream_error_log2(n_e: int, q1: int, delta_steps: int, sample_bits: int, delta: float,
                      k: int) -> tuple[float, float]:
    """(log2 of Theorem 3.6's sum over k blocks, log2 of its closed bound)."""
    lib = load()
    s, c = ctypes.c_double(), ctypes.c_double()
    _check(lib.ext_stream_error_log2(n_e, q1, delta_steps, sample_bits, float(delta), k,
                                     ctypes.byref(s), ctypes.byref(c)), "ext_stream_error_log2")
    return s.value, c.value


def output_bits(q1: int, delta_steps: int, sample_bits: int, k: int) -> int:
    """m_k of Theorem 3.6."""
    lib = load()
    m = ctypes.c_uint64()
    _check(lib.ext_output_bits(q1, delta_steps, sample_bits, k, ctypes.byref(m)), "ext_output_bits")
    return m.value


class Growing:
    """One ext_growing: Algorithm 2's growing blocks (q_l = q1 + l * delta_steps * b)."""

    def __init__(self, n_e: int, q1: int, delta_steps: int, *, sample_bits: int = 8,
                 device_memory: bool = True, stream=None, device: int = -1,
                 device_bytes_cap: int = 0):
        self.lib = load()
        p = make_params(self.lib, device_memory=device_memory, stream=stream,
                        sample_bits=sample_bits, device=device, device_bytes_cap=device_bytes_cap)
        self.handle = ctypes.c_void_p()
        _check(self.lib.ext_growing_create(n_e, q1, delta_steps, ctypes.byref(p),
                                           ctypes.byref(self.handle)), "ext_growing_create")

    def blocks(self, n_bytes: int) -> tuple[int, int, int]:
        """(whole blocks in n_bytes per source, their input bytes, output bytes)."""
        k, i, o = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
        _check(self.lib.ext_growing_blocks(self.handle, n_bytes, ctypes.byref(k), ctypes.byref(i),
                                           ctypes.byref(o)), "ext_growing_blocks")
        return k.value, i.value, o.value

    def extract(self, x, y, n_bytes: int, out, out_cap: int, max_blocks: int = 2 ** 64 - 1) -> int:
        k = ctypes.c_uint64()
        _check(self.lib.ext_growing_extract(self.handle, _ptr(x), _ptr(y), n_bytes, max_blocks,
                                            _ptr(out), out_cap, ctypes.byref(k)),
               "ext_growing_extract")
        return k.value

    def extract_noalloc(self, x, y, n_bytes: int, out, out_cap: int,
                        max_blocks: int = 2 ** 64 - 1) -> int:
        """ext_growing_extract_noalloc: as extract (device memory only), with
        the launch tables in the library's static device scratch."""
        k = ctypes.c_uint64()
        _check(self.lib.ext_growing_extract_noalloc(self.handle, _ptr(x), _ptr(y), n_bytes,
                                                    max_blocks, _ptr(out), out_cap,
                                                    ctypes.byref(k)),
               "ext_growing_extract_noalloc")
        return k.value

    def open_stream(self) -> "GrowingStream":
        """Algorithm 2's online form on this handle (ext_growing_open)."""
        return GrowingStream(self)

    def close(self):
        if self.handle:
            self.lib.ext_growing_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class GrowingStream:
    """One ext_growing_stream: Algorithm 2 on unbounded sources fed in chunks."""

    def __init__(self, g: Growing):
        self.lib = g.lib
        self.g = g
        self.handle = ctypes.c_void_p()
        _check(self.lib.ext_growing_open(g.handle, ctypes.byref(self.handle)), "ext_growing_open")

    def submit(self, x, x_len: int, y, y_len: int) -> int:
        """EXT_OK or EXT_EAGAIN (nothing consumed); raises on other errors."""
        n = ctypes.c_uint64()
        rc = self.lib.ext_growing_submit(self.handle, _ptr(x) if x_len else None, x_len,
                                         _ptr(y) if y_len else None, y_len, ctypes.byref(n))
        if rc == EXT_EAGAIN:
            return rc
        _check(rc, "ext_growing_submit")
        return rc

    def poll(self, out, out_cap: int, wait: bool = False):
        """(bytes written, blocks returned so far)."""
        n = ctypes.c_size_t()
        done = ctypes.c_uint64()
        f = self.lib.ext_growing_drain if wait else self.lib.ext_growing_poll
        _check(f(self.handle, _ptr(out) if out_cap else None, out_cap, ctypes.byref(n),
                 ctypes.byref(done)), "ext_growing_poll")
        return n.value, done.value

    def state(self) -> tuple[int, int, int]:
        """(next block l, its degree q_l, bytes per source taken so far)."""
        a, b, c = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
        _check(self.lib.ext_growing_state(self.handle, ctypes.byref(a), ctypes.byref(b),
                                          ctypes.byref(c)), "ext_growing_state")
        return a.value, b.value, c.value

    def close(self) -> int:
        """Dropped bits of the incomplete block."""
        d = ctypes.c_uint64()
        if self.handle:
            _check(self.lib.ext_growing_close(self.handle, ctypes.byref(d)), "ext_growing_close")
            self.handle = ctypes.c_void_p()
        return d.value


def probe_valu_rate(device: int = -1) -> float:
    """The device's measured v_bitop3_b32 issue rate, lane-ops per second."""
    lib = load()
    r = ctypes.c_double()
    _check(lib.ext_probe_valu_rate(device, ctypes.byref(r)), "ext_probe_valu_rate")
    return r.value
