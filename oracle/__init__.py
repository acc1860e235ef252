"""CPU oracle for the block-wise inner-product extractor.

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the benchmark's
CPU-baseline leg are its only callers.  The product (the HIP library and its
Python binding) never imports this package, and this package imports nothing
from the product.

What it computes follows the paper (Li & Zhou, "Real-Time Seedless
Post-Processing for Quantum Random Number Generators"):

* Def. 3.2 -- the inner-product extractor over F_{2^q}, sum_i x_i * y_i;
* Algorithm 1 -- consecutive equal blocks of q*n_e bits per source, one q-bit
  output per block pair, outputs concatenated in block order.

The arithmetic lives in ``oracle.c`` (bit by bit, one bit per byte).  The
modulus P of each degree q follows a fixed convention (lowest weight, then
lexicographically smallest exponents), found by ``orc_find_modulus`` and
stored in ``moduli.txt`` by ``gen_moduli.py``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_TABLE = os.path.join(_HERE, "moduli.txt")



def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so with gcc (plain -O2, no vector
    intrinsics).  Returns the library path."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=c99", "-Wall", "-shared", "-fPIC", "-o", tmp, _SRC]
        )
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class OracleLib:
    """The compiled oracle.  ``OracleLib(path)`` loads another build of the
    same source (the mutation tests load deliberately broken copies)."""

    def __init__(self, path: str):
        lib = ctypes.CDLL(path)
        u8p = ctypes.POINTER(ctypes.c_uint8)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        lib.orc_ext_blocks.argtypes = [u8p, u8p, ctypes.c_uint64, ctypes.c_uint64,
                                       ctypes.c_uint32, u32p, ctypes.c_uint32, u8p]
        lib.orc_ext_blocks.restype = ctypes.c_int
        lib.orc_ext_sampled.argtypes = [u8p, u8p, u64p, ctypes.c_uint64, ctypes.c_uint64,
                                        ctypes.c_uint32, u32p, ctypes.c_uint32, u8p]
        lib.orc_ext_sampled.restype = ctypes.c_int
        lib.orc_is_irreducible.argtypes = [ctypes.c_uint32, u32p, ctypes.c_uint32]
        lib.orc_is_irreducible.restype = ctypes.c_int
        lib.orc_find_modulus.argtypes = [ctypes.c_uint32, u32p]
        lib.orc_find_modulus.restype = ctypes.c_int
        self.lib = lib
        self.path = path


def compile_variant(src_text: str, out_path: str) -> str:
    """Compile oracle source text (e.g. a mutated copy) to out_path."""
    c_path = out_path + ".c"
    with open(c_path, "w") as f:
        f.write(src_text)
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-w", "-shared", "-fPIC", "-o", out_path, c_path])
    return out_path


def source_text() -> str:
    with open(_SRC) as f:
        return f.read()


_default = None


def _load(lib: "OracleLib | None" = None):
    global _default
    if lib is not None:
        return lib.lib
    if _default is None:
        _default = OracleLib(build())
    return _default.lib


def _u8(a):
    a = np.ascontiguousarray(np.frombuffer(a, dtype=np.uint8) if isinstance(a, (bytes, bytearray)) else a,
                             dtype=np.uint8)
    return a


def _ptr(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def _exps_array(q: int, exps) -> np.ndarray:
    if exps is None:
        exps = modulus(q)
    e = np.asarray(sorted(set(int(v) for v in exps), reverse=True), dtype=np.uint32)
    if len(e) != len(exps) or e[0] != q or e[-1] != 0:
        raise ValueError("modulus exponents must be distinct and include q and 0: %r" % (exps,))
    return e


# ---------------------------------------------------------------------------
# modulus convention
# ---------------------------------------------------------------------------
_table_cache: dict[int, tuple] | None = None


def _read_table() -> dict[int, tuple]:
    global _table_cache
    if _table_cache is None:
        t = {}
        if os.path.exists(_TABLE):
            with open(_TABLE) as f:
                for line in f:
                    line = line.split("#", 1)[0].strip()
                    if not line:
                        continue
                    vals = tuple(int(v) for v in line.split())
                    t[vals[0]] = vals
        _table_cache = t
    return _table_cache


def find_modulus(q: int, lib: "OracleLib | None" = None) -> tuple:
    """Search for the conventional modulus of degree q (slow for large q)."""
    clib = _load(lib)
    out = np.zeros(5, dtype=np.uint32)
    n = clib.orc_find_modulus(q, _ptr(out, ctypes.c_uint32))
    if n <= 0:
        raise ValueError("no modulus found for q=%d (code %d)" % (q, n))
    return tuple(int(v) for v in out[:n])


def modulus(q: int) -> tuple:
    """Exponents of P (decreasing, q first, 0 last) for degree q: from the
    stored table when present, else searched now."""
    t = _read_table()
    if q in t:
        return t[q]
    return find_modulus(q)


def is_irreducible(q: int, exps, lib: "OracleLib | None" = None) -> bool:
    e = _exps_array(q, exps)
    r = _load(lib).orc_is_irreducible(q, _ptr(e, ctypes.c_uint32), len(e))
    if r < 0:
        raise ValueError("bad modulus %r (code %d)" % (exps, r))
    return bool(r)


# ---------------------------------------------------------------------------
# extractor
# ---------------------------------------------------------------------------
def ext_blocks(x, y, n_bits: int, q: int, exps=None, n_pairs: int | None = None,
               lib: "OracleLib | None" = None) -> np.ndarray:
    """Algorithm 1 over two raw byte streams: returns the concatenated outputs
    Z^(0) Z^(1) ... as bytes (q bits per block pair, LSB-first)."""
    x = _u8(x)
    y = _u8(y)
    if n_bits <= 0 or q <= 0 or n_bits % q:
        raise ValueError("n_bits must be a positive multiple of q")
    full = (8 * min(x.size, y.size)) // n_bits
    if n_pairs is None:
        n_pairs = full
    if n_pairs > full:
        raise ValueError("not enough input for %d block pairs" % n_pairs)
    e = _exps_array(q, exps)
    out = np.zeros((n_pairs * q + 7) // 8, dtype=np.uint8)
    if n_pairs == 0:
        return out
    rc = _load(lib).orc_ext_blocks(_ptr(x, ctypes.c_uint8), _ptr(y, ctypes.c_uint8), n_pairs, n_bits, q,
                                _ptr(e, ctypes.c_uint32), len(e), _ptr(out, ctypes.c_uint8))
    if rc != 0:
        raise RuntimeError("orc_ext_blocks failed: %d" % rc)
    return out


def ext_sampled(x, y, idx, n_bits: int, q: int, exps=None,
                lib: "OracleLib | None" = None) -> np.ndarray:
    """Outputs of the listed block pairs only, q bits each, densely packed
    (listed pair k at output bits [kq, (k+1)q))."""
    x = _u8(x)
    y = _u8(y)
    idx = np.ascontiguousarray(idx, dtype=np.uint64)
    full = (8 * min(x.size, y.size)) // n_bits
    if idx.size and int(idx.max()) >= full:
        raise ValueError("block index out of range")
    e = _exps_array(q, exps)
    out = np.zeros((idx.size * q + 7) // 8, dtype=np.uint8)
    if idx.size == 0:
        return out
    rc = _load(lib).orc_ext_sampled(_ptr(x, ctypes.c_uint8), _ptr(y, ctypes.c_uint8), _ptr(idx, ctypes.c_uint64),
                                 idx.size, n_bits, q, _ptr(e, ctypes.c_uint32), len(e),
                                 _ptr(out, ctypes.c_uint8))
    if rc != 0:
        raise RuntimeError("orc_ext_sampled failed: %d" % rc)
    return out


def field_mul(a: int, b: int, q: int, exps=None, lib: "OracleLib | None" = None) -> int:
    """One multiplication in F_{2^q}: the extractor with a single element
    (n_e = 1) is exactly the field product."""
    nb = (q + 7) // 8
    xa = np.frombuffer(int(a).to_bytes(nb, "little"), dtype=np.uint8)
    yb = np.frombuffer(int(b).to_bytes(nb, "little"), dtype=np.uint8)
    # pad to whole bytes: the block is q bits; ext_blocks reads bits [0, q)
    z = ext_blocks(xa, yb, q, q, exps, n_pairs=1, lib=lib)
    return int.from_bytes(z.tobytes(), "little") & ((1 << q) - 1)


def ext_ip_int(xs, ys, q: int, exps=None, lib: "OracleLib | None" = None) -> int:
    """Ext_IP over lists of field elements given as Python ints (element i =
    xs[i]); convenience for tests on tiny sizes."""
    n_e = len(xs)
    assert len(ys) == n_e
    xv = sum(int(v) << (i * q) for i, v in enumerate(xs))
    yv = sum(int(v) << (i * q) for i, v in enumerate(ys))
    nb = (n_e * q + 7) // 8
    xa = np.frombuffer(xv.to_bytes(nb, "little"), dtype=np.uint8)
    ya = np.frombuffer(yv.to_bytes(nb, "little"), dtype=np.uint8)
    z = ext_blocks(xa, ya, n_e * q, q, exps, n_pairs=1, lib=lib)
    return int.from_bytes(z.tobytes(), "little") & ((1 << q) - 1)
