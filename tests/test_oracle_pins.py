"""The CPU oracle against its pins (no GPU), and the pins against planted
mistakes: each broken copy of the oracle must fail at least one pin."""
from __future__ import annotations

import hashlib
import os

import numpy as np
import pytest

import oracle
import oracle_pins as pins

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.parametrize("pin", pins.ALL_PINS, ids=lambda f: f.__name__)
def test_pin(pin):
    pin()


# (name, text in oracle.c, replacement): plausible mistakes -- a dropped term,
# a wrong index or sign, a transposed operand, a reversed bit order.
MUTATIONS = [
    ("drop_constant_term_of_P", "c[d - q + exps[e]] ^= 1;",
     "if (exps[e]) c[d - q + exps[e]] ^= 1;"),
    ("reduce_bottom_up", "for (int64_t d = 2 * (int64_t)q - 2; d >= (int64_t)q; d--) {\n        if (c[d])",
     "for (int64_t d = (int64_t)q; d <= 2 * (int64_t)q - 2; d++) {\n        if (c[d])"),
    ("reversed_y", "c[j + l] ^= (uint8_t)(xi[j] & yi[l]);",
     "c[j + l] ^= (uint8_t)(xi[j] & yi[q - 1 - l]);"),
    ("pair_x_i_with_y_next", "const uint8_t *yi = yb + (size_t)i * q;",
     "const uint8_t *yi = yb + (size_t)((i + 1) % n_e) * q;"),
    ("msb_first_bits", "return (buf[r >> 3] >> (r & 7)) & 1;",
     "return (buf[r >> 3] >> (7 - (r & 7))) & 1;"),
    ("skip_last_element", "for (uint32_t i = 0; i < n_e; i++) {\n        const uint8_t *xi",
     "for (uint32_t i = 0; i + 1 < n_e || i == 0; i++) {\n        const uint8_t *xi"),
    ("or_instead_of_and", "(uint8_t)(xi[j] & yi[l])", "(uint8_t)(xi[j] | yi[l])"),
    ("output_reversed", "put_bit(out, l * (uint64_t)q + j, z[j]);",
     "put_bit(out, l * (uint64_t)q + (q - 1 - j), z[j]);"),
    ("overlapping_blocks", "xb[r] = (uint8_t)get_bit(x, l * n_bits + r);",
     "xb[r] = (uint8_t)get_bit(x, l * q + r);"),
    ("drop_top_coefficient", "for (int64_t d = 2 * (int64_t)q - 2; d >= (int64_t)q; d--) {",
     "for (int64_t d = 2 * (int64_t)q - 3; d >= (int64_t)q; d--) {"),
    # the sampled path's own index arithmetic (its anchors occur only there)
    ("sampled_reads_kth_block", "uint64_t l = idx[k];", "uint64_t l = k;"),
    ("sampled_output_at_block_index", "put_bit(out, k * (uint64_t)q + j, z[j]);",
     "put_bit(out, l * (uint64_t)q + j, z[j]);"),
    ("sampled_list_reversed", "uint64_t l = idx[k];", "uint64_t l = idx[n_idx - 1 - k];"),
]


@pytest.mark.parametrize("name,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_pins_catch_planted_mistake(tmp_path, name, old, new):
    src = oracle.source_text()
    assert src.count(old) >= 1, "mutation anchor not found: %s" % name
    lib = oracle.OracleLib(oracle.compile_variant(src.replace(old, new, 1),
                                                  str(tmp_path / ("%s.so" % name))))
    caught = []
    for pin in pins.ALL_PINS:
        if pin is pins.pin_moduli:
            continue  # exercises the modulus helpers, not the extractor
        try:
            pin(lib)
        except (AssertionError, RuntimeError, ValueError) as e:
            caught.append((pin.__name__, str(e)[:80]))
    assert caught, "no pin detects the planted mistake %s" % name


def test_find_modulus_small_degrees_match_table():
    table = oracle._read_table()
    for q in list(range(2, 65)) + [80, 96, 128, 256, 512]:
        assert oracle.find_modulus(q) == table[q]


def test_tiny_workload_digest():
    """The oracle's output on the tiny workload is the one recorded by
    tests/golden/gen_golden.py (guards against silent changes)."""
    from paper_2402_14607_amd import inputs

    with open(os.path.join(HERE, "golden", "tiny_oracle.txt")) as f:
        rec = dict(line.split("=", 1) for line in f.read().split() if "=" in line)
    w = inputs.tiny()
    z = oracle.ext_blocks(w.x, w.y, w.n_bits, w.m_bits)
    assert z.size == int(rec["bytes"])
    assert hashlib.sha256(z.tobytes()).hexdigest() == rec["sha256"]
    assert hashlib.sha256(w.x.tobytes() + w.y.tobytes()).hexdigest() == rec["input_sha256"]


def test_oracle_rejects_bad_arguments():
    x = np.zeros(64, dtype=np.uint8)
    with pytest.raises(ValueError):
        oracle.ext_blocks(x, x, 100, 64)          # n not a multiple of q
    with pytest.raises(ValueError):
        oracle.ext_blocks(x, x, 256, 64, exps=(64, 4, 3, 1))   # no constant term
    with pytest.raises(ValueError):
        oracle.ext_blocks(x, x, 256, 64, n_pairs=3)            # not enough input
    assert oracle.ext_blocks(x[:8], x[:8], 256, 64).size == 0  # fewer bytes than a block
