"""The C-ABI library on the CPU: it loads, exports every function the
public header declares, and its host-side logic (modulus convention,
irreducibility test, argument checks) agrees with the oracle.  No GPU
compute is launched here."""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from paper_2402_14607_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qrng_ext.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ext_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = binding.load()
    names = declared_functions()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), "libqrngext.so does not export %s" % name
    assert set(names) == set(binding.EXPORTED)


def test_default_modulus_every_byte_multiple_degree():
    """Degrees 8, 16, ..., 1024 (the byte-granular fields of the paper's
    parameter rule with b = 8 or 16): the library's own search agrees with
    the oracle's table."""
    table = oracle._read_table()
    for m in range(8, 1025, 8):
        assert binding.default_modulus(m) == table[m], m


def test_default_modulus_matches_oracle_table():
    """Every degree the oracle's table holds that the library's built-in table
    holds too (the multiples of 8 up to 8192, among them Algorithm 2's
    degrees 80, 96, ..., 5184 at b = 16, and 16384), found by two independent
    searches; then the library's run-time search, for degrees outside its
    table, against the oracle's."""
    table = oracle._read_table()
    common = [m for m in table if (m % 8 == 0 and m <= 8192) or m == 16384]
    assert len(common) > 300 and max(m for m in common if m <= 8192) >= 5184
    for m in common:
        assert binding.default_modulus(m) == table[m], m
    for m in (3, 5, 17, 33, 41, 57, 63):
        assert binding.default_modulus(m) == table[m], m


def test_irreducibility_matches_oracle():
    rng = np.random.Generator(np.random.PCG64(11))
    for _ in range(60):
        m = int(rng.integers(8, 300))
        a, b, c = sorted(rng.choice(np.arange(1, m), 3, replace=False), reverse=True)
        taps = (int(a), int(b), int(c))
        assert binding.is_irreducible(m, taps) == oracle.is_irreducible(m, (m,) + taps + (0,))
    for m in range(2, 64):
        exps = oracle.modulus(m)
        assert binding.is_irreducible(m, exps[1:-1])


def test_strerror_and_bad_arguments():
    lib = binding.load()
    for code in range(-6, 1):
        assert lib.ext_strerror(code)
    assert binding.strerror(-4).startswith("device buffer full")
    with pytest.raises(binding.ExtError):
        binding.is_irreducible(8, (9,))
    # ext_create argument checks come before any device call
    p = binding.ExtParams()
    lib.ext_params_init(ctypes.byref(p))
    h = ctypes.c_void_p()
    assert lib.ext_create(1000, 256, ctypes.byref(p), ctypes.byref(h)) == binding.EXT_EINVAL
    assert lib.ext_create(0, 256, ctypes.byref(p), ctypes.byref(h)) == binding.EXT_EINVAL
    assert lib.ext_create(1024, 0, ctypes.byref(p), ctypes.byref(h)) == binding.EXT_EINVAL
    p.sample_bits = 16
    assert lib.ext_create(1000 * 24, 24, ctypes.byref(p), ctypes.byref(h)) == binding.EXT_EINVAL
    assert lib.ext_destroy(None) == 0
    assert lib.ext_submit(None, None, 0, None, 0, None) == binding.EXT_EINVAL


def test_word_only_forms_refuse_the_bitsliced_kernel():
    """The batched, served and growing forms run the word-level kernel: a
    request for the bit-sliced one is EXT_ENOTSUP, an unknown kernel value
    EXT_EINVAL, both answered before any device call."""
    import ctypes

    lib = binding.load()
    for kernel, want in ((binding.KERNEL_BITSLICE, binding.EXT_ENOTSUP), (3, binding.EXT_EINVAL)):
        p = binding.make_params(lib, kernel=kernel)
        h = ctypes.c_void_p()
        item = binding.BatchItem()
        item.n_bits, item.m_bits, item.n_pairs = 5680, 80, 1
        assert lib.ext_batch_create(ctypes.byref(item), 1, ctypes.byref(p), ctypes.byref(h)) == want
        cfg = binding.ServerConfig()
        lib.ext_server_config_init(ctypes.byref(cfg))
        assert lib.ext_server_create(ctypes.byref(cfg), ctypes.byref(p), ctypes.byref(h)) == want
        assert lib.ext_growing_create(71, 80, 1, ctypes.byref(p), ctypes.byref(h)) == want
        assert not h.value
