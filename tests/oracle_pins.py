"""Pins of the CPU oracle: checks that tie it to facts outside itself.

Each ``pin_*`` takes an optional oracle build (``lib``) and raises
AssertionError when the oracle disagrees with the fact it is pinned to.  The
test-suite runs them on the real oracle (all must pass) and on deliberately
broken copies (each copy must fail at least one pin).

What each pin rests on:
  pin_fips197        worked examples of GF(2^8) products printed in FIPS-197
  pin_identity       closed forms of Def. 3.2: 1 is the field identity, so
                     Ext(x, e_k) = x_k, and Ext(0, y) = 0
  pin_matrix         Ext(x, y) = M_y x with the columns y_i t^j mod P built by
                     repeated multiplication by t (shift, conditional XOR of P):
                     a different route from the oracle's convolution + reduction
  pin_no_reduction   for operands of degree < q/2 no reduction happens and the
                     result is the carry-less product (shift-XOR on Python ints)
  pin_bilinear       GF(2)-bilinearity in x and in y, symmetry Ext(x,y)=Ext(y,x)
  pin_field          field axioms of F_{2^q}: associativity, distributivity,
                     Frobenius a^(2^q) = a, inverses a^(2^q - 2) a = 1
  pin_hadamard       Prop. A.2 (Appendix A): bit 0 of a * Ext(x, y) is a
                     Hadamard function for every nonzero a (exhaustive, tiny q)
  pin_balanced       for fixed x != 0, y -> Ext(x, y) takes every value equally
                     often (the linear map y -> sum x_i y_i is onto)
  pin_partition      Algorithm 1: consecutive blocks, outputs concatenated in
                     block order, trailing partial block unused, Nb/n_e output bits
  pin_moduli         the stored moduli are irreducible (Rabin), Rabin agrees with
                     brute-force trial division on small degrees, and the stored
                     modulus is the convention's choice (exhaustive for small q)
  pin_sampled        the sampled path (block pairs listed by index, outputs packed
                     densely in list order) returns, for every listed index, the
                     bits the whole-stream path (pinned above) computes for that
                     block pair: unsorted lists, repeats, the first and last pair,
                     fields whose degree is not a multiple of 8
"""
from __future__ import annotations

import os

import numpy as np

import oracle

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


# ---------------------------------------------------------------------------
# independent helpers (Python ints; bit j = coefficient of t^j)
# ---------------------------------------------------------------------------
def poly_int(exps) -> int:
    return sum(1 << e for e in exps)


def xtime(a: int, q: int, p: int) -> int:
    """a * t mod P by shift and conditional subtraction of P."""
    a <<= 1
    if (a >> q) & 1:
        a ^= p
    return a


def clmul_int(a: int, b: int) -> int:
    r = 0
    while b:
        if b & 1:
            r ^= a
        a <<= 1
        b >>= 1
    return r


def poly_mod_int(a: int, f: int) -> int:
    df = f.bit_length() - 1
    while a and a.bit_length() - 1 >= df:
        a ^= f << (a.bit_length() - 1 - df)
    return a


def irreducible_bruteforce(f: int) -> bool:
    """Trial division by every polynomial of degree 1 .. deg(f)/2."""
    d = f.bit_length() - 1
    for g in range(2, 1 << (d // 2 + 1)):
        if poly_mod_int(f, g) == 0:
            return False
    return True


def read_golden(name: str):
    rows, mod = [], None
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            if line.startswith("modulus"):
                mod = tuple(int(v) for v in line.split()[1:])
            else:
                rows.append(line.split())
    return mod, rows


def pack_blocks(elems, q: int) -> bytes:
    """Blocks given as lists of q-bit field elements -> byte stream, each
    block n_e*q bits, element i at block bits [iq, (i+1)q), blocks back to
    back (bit-level, LSB first)."""
    bits = []
    for blk in elems:
        for v in blk:
            bits.extend(((v >> j) & 1) for j in range(q))
    arr = np.asarray(bits, dtype=np.uint8)
    return np.packbits(arr, bitorder="little").tobytes()


def unpack_outputs(buf, q: int, count: int):
    bits = np.unpackbits(np.frombuffer(bytes(buf), dtype=np.uint8), bitorder="little")
    out = []
    for k in range(count):
        v = 0
        seg = bits[k * q:(k + 1) * q]
        for j in np.nonzero(seg)[0]:
            v |= 1 << int(j)
        out.append(v)
    return out


def ext_many(xblocks, yblocks, q: int, exps, lib=None):
    """Ext over many block pairs in one oracle call."""
    n_e = len(xblocks[0])
    xs = pack_blocks(xblocks, q)
    ys = pack_blocks(yblocks, q)
    z = oracle.ext_blocks(xs, ys, n_e * q, q, exps, n_pairs=len(xblocks), lib=lib)
    return unpack_outputs(z, q, len(xblocks))


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def rand_elem(rng, q: int) -> int:
    return int.from_bytes(rng.bytes((q + 7) // 8), "little") & ((1 << q) - 1)


# ---------------------------------------------------------------------------
# pins
# ---------------------------------------------------------------------------
def pin_fips197(lib=None):
    mod, rows = read_golden("fips197_gf256.txt")
    for a, b, c in rows:
        got = oracle.field_mul(int(a, 16), int(b, 16), 8, mod, lib=lib)
        assert got == int(c, 16), "{%s}.{%s} = %02x, FIPS-197 prints {%s}" % (a, b, got, c)


def pin_identity(lib=None):
    rng = _rng(101)
    for q, n_e in ((64, 4), (256, 4), (96, 3)):
        exps = oracle.modulus(q)
        xs = [[rand_elem(rng, q) for _ in range(n_e)] for _ in range(n_e + 1)]
        ys = []
        for k in range(n_e):
            e = [0] * n_e
            e[k] = 1
            ys.append(e)
        ys.append([0] * n_e)
        got = ext_many(xs, ys, q, exps, lib)
        for k in range(n_e):
            assert got[k] == xs[k][k], "Ext(x, e_%d) != x_%d at q=%d" % (k, k, q)
        assert got[n_e] == 0, "Ext(x, 0) != 0 at q=%d" % q
        # and Ext(0, y) = 0 with y arbitrary
        z = ext_many([[0] * n_e], [[rand_elem(rng, q) for _ in range(n_e)]], q, exps, lib)
        assert z[0] == 0


def pin_matrix(lib=None):
    rng = _rng(102)
    for q in (8, 16, 32, 64):
        exps = oracle.modulus(q)
        p = poly_int(exps)
        for n_e in (1, 2, 4):
            y = [rand_elem(rng, q) for _ in range(n_e)]
            # columns y_i t^j mod P by repeated xtime
            cols = []
            for i in range(n_e):
                c = y[i]
                row = []
                for j in range(q):
                    row.append(c)
                    c = xtime(c, q, p)
                cols.append(row)
            if q * n_e <= 16:
                xs = [[(v >> (i * q)) & ((1 << q) - 1) for i in range(n_e)]
                      for v in range(1 << (q * n_e))]
            else:
                xs = [[rand_elem(rng, q) for _ in range(n_e)] for _ in range(64)]
            got = ext_many(xs, [y] * len(xs), q, exps, lib)
            for x, g in zip(xs, got):
                want = 0
                for i in range(n_e):
                    for j in range(q):
                        if (x[i] >> j) & 1:
                            want ^= cols[i][j]
                assert g == want, "Ext != M_y x at q=%d n_e=%d" % (q, n_e)


def pin_no_reduction(lib=None):
    rng = _rng(103)
    for q in (64, 256):
        exps = oracle.modulus(q)
        xs, ys = [], []
        for _ in range(16):
            xs.append([rand_elem(rng, q // 2)])
            ys.append([rand_elem(rng, q // 2 - 1)])
        got = ext_many(xs, ys, q, exps, lib)
        for x, y, g in zip(xs, ys, got):
            assert g == clmul_int(x[0], y[0]), "unreduced product wrong at q=%d" % q


def pin_bilinear(lib=None):
    rng = _rng(104)
    for q, n_e, reps in ((256, 4, 6), (2048, 1, 2), (96, 5, 6)):
        exps = oracle.modulus(q)
        for _ in range(reps):
            x, x2, y, y2 = ([rand_elem(rng, q) for _ in range(n_e)] for _ in range(4))
            xx = [a ^ b for a, b in zip(x, x2)]
            yy = [a ^ b for a, b in zip(y, y2)]
            a, b, c, d, e, f, g = ext_many([x, x2, xx, x, x, y, y],
                                           [y, y, y, y2, yy, x, y], q, exps, lib)
            assert c == a ^ b, "not linear in x (q=%d)" % q
            assert e == a ^ d, "not linear in y (q=%d)" % q
            assert f == a, "not symmetric (q=%d)" % q
            assert g == ext_many([y], [y], q, exps, lib)[0]


def _fmul_many(pairs, q, exps, lib):
    return ext_many([[a] for a, _ in pairs], [[b] for _, b in pairs], q, exps, lib)


def pin_field(lib=None):
    rng = _rng(105)
    for q in (8, 64, 256):
        exps = oracle.modulus(q)
        a, b, c = (rand_elem(rng, q) | 1 for _ in range(3))
        ab, bc = _fmul_many([(a, b), (b, c)], q, exps, lib)
        ab_c, a_bc = _fmul_many([(ab, c), (a, bc)], q, exps, lib)
        assert ab_c == a_bc, "not associative (q=%d)" % q
        l1, r1, r2 = _fmul_many([(a, b ^ c), (a, b), (a, c)], q, exps, lib)
        assert l1 == r1 ^ r2, "not distributive (q=%d)" % q
        # Frobenius: q squarings return a
        v = a
        for _ in range(q):
            v = _fmul_many([(v, v)], q, exps, lib)[0]
        assert v == a, "a^(2^q) != a (q=%d)" % q
    # inverse by Fermat in F_{2^64}: a^(2^64 - 2) * a = 1
    q = 64
    exps = oracle.modulus(q)
    a = rand_elem(rng, q) | 1
    e = (1 << q) - 2
    r, base = 1, a
    while e:
        if e & 1:
            r = _fmul_many([(r, base)], q, exps, lib)[0]
        base = _fmul_many([(base, base)], q, exps, lib)[0]
        e >>= 1
    assert _fmul_many([(r, a)], q, exps, lib)[0] == 1, "no inverse (q=64)"


def _ext_table(q, n_e, exps, lib):
    """T[x][y] = Ext(x, y) for every x, y in {0,1}^(q n_e)."""
    nb = q * n_e
    vals = list(range(1 << nb))
    xs = [[(v >> (i * q)) & ((1 << q) - 1) for i in range(n_e)] for v in vals for _ in vals]
    ys = [[(w >> (i * q)) & ((1 << q) - 1) for i in range(n_e)] for _ in vals for w in vals]
    flat = ext_many(xs, ys, q, exps, lib)
    return np.asarray(flat, dtype=np.int64).reshape(len(vals), len(vals))


def pin_hadamard(lib=None):
    for q, n_e in ((2, 2), (3, 2), (4, 2)):
        exps = oracle.modulus(q)
        T = _ext_table(q, n_e, exps, lib)
        size = T.shape[0]
        for a in range(1, 1 << q):
            mul = _fmul_many([(a, z) for z in range(1 << q)], q, exps, lib)
            bit0 = np.asarray([m & 1 for m in mul])
            F = 1 - 2 * bit0[T]  # (-1)^f_a(x, y)
            G = F @ F.T
            assert np.array_equal(G, size * np.eye(size, dtype=G.dtype)), \
                "bit 0 of a*Ext is not Hadamard (q=%d, a=%d)" % (q, a)


def pin_balanced(lib=None):
    q, n_e = 4, 2
    T = _ext_table(q, n_e, oracle.modulus(q), lib)
    for x in range(1, T.shape[0]):
        counts = np.bincount(T[x], minlength=1 << q)
        assert np.all(counts == (1 << (q * (n_e - 1)))), "not balanced for x=%d" % x


def pin_partition(lib=None):
    rng = _rng(106)
    q, n_e = 64, 4
    nbits = q * n_e
    blocks = 5
    exps = oracle.modulus(q)
    x = rng.integers(0, 256, blocks * nbits // 8 + 17, dtype=np.uint8)
    y = rng.integers(0, 256, blocks * nbits // 8 + 3, dtype=np.uint8)
    whole = oracle.ext_blocks(x, y, nbits, q, exps, lib=lib)
    assert whole.size * 8 == blocks * q, "output length is not (#blocks) q"
    assert whole.size * 8 == (min(x.size, y.size) * 8 // nbits) * nbits // n_e
    parts = []
    for k in range(blocks):
        xs = x[k * nbits // 8:(k + 1) * nbits // 8]
        ys = y[k * nbits // 8:(k + 1) * nbits // 8]
        parts.append(oracle.ext_blocks(xs, ys, nbits, q, exps, lib=lib))
    assert np.array_equal(whole, np.concatenate(parts)), "blocks not consecutive / in order"
    # the same blocks with their pairs in swapped roles give the same bytes
    # (Ext is symmetric), and a different block order gives different bytes
    swapped = oracle.ext_blocks(y[:blocks * nbits // 8], x[:blocks * nbits // 8], nbits, q, exps,
                                lib=lib)
    assert np.array_equal(whole, swapped)


def pin_moduli(lib=None):
    table = oracle._read_table()
    assert table, "oracle/moduli.txt is empty"
    for q, exps in table.items():
        if q <= 4096:
            assert oracle.is_irreducible(q, exps, lib=lib), "stored modulus of q=%d reducible" % q
    mod, _ = read_golden("gcm_modulus.txt")
    assert oracle.is_irreducible(128, mod, lib=lib)
    assert table[128] == mod
    mod, _ = read_golden("fips197_gf256.txt")
    assert oracle.is_irreducible(8, mod, lib=lib)
    # Rabin's test against trial division on every trinomial and pentanomial
    # of degree 2..12
    for q in range(2, 13):
        for a in range(1, q):
            for taps in ([a],) + tuple([a, b, c] for b in range(2, a) for c in range(1, b)):
                exps = [q] + list(taps) + [0]
                want = irreducible_bruteforce(poly_int(exps))
                got = oracle.is_irreducible(q, exps, lib=lib)
                assert got == want, "Rabin disagrees with trial division on %r" % exps
    # the stored modulus is the convention's choice, by exhaustive search
    for q in range(2, 17):
        best = None
        for a in range(1, q):
            if irreducible_bruteforce(poly_int([q, a, 0])):
                best = (q, a, 0)
                break
        if best is None:
            for a in range(3, q):
                for b in range(2, a):
                    for c in range(1, b):
                        if best is None and irreducible_bruteforce(poly_int([q, a, b, c, 0])):
                            best = (q, a, b, c, 0)
        assert table[q] == best, "stored modulus for q=%d is %r, convention gives %r" % (
            q, table[q], best)


def pin_sampled(lib=None):
    rng = _rng(107)
    for q, n_e in ((64, 4), (80, 3), (24, 5), (256, 2), (12, 2)):
        nbits = q * n_e
        blocks = 9
        exps = oracle.modulus(q)
        nbytes = (blocks * nbits + 7) // 8
        x = rng.integers(0, 256, nbytes + 3, dtype=np.uint8)
        y = rng.integers(0, 256, nbytes, dtype=np.uint8)
        whole = np.unpackbits(oracle.ext_blocks(x, y, nbits, q, exps, lib=lib),
                              bitorder="little")
        assert whole.size >= blocks * q
        # as many listed pairs as blocks: unsorted, with repeats, first and
        # last included; then a random order of every block
        lists = [np.asarray([8, 0, 3, 3, 7, 1, 8, 2, 5], dtype=np.uint64),
                 rng.permutation(blocks).astype(np.uint64)]
        for idx in lists:
            got = np.unpackbits(oracle.ext_sampled(x, y, idx, nbits, q, exps, lib=lib),
                                bitorder="little")
            assert got.size == (idx.size * q + 7) // 8 * 8
            for k, l in enumerate(idx.tolist()):
                assert np.array_equal(got[k * q:(k + 1) * q], whole[l * q:(l + 1) * q]), \
                    "sampled pair %d (block %d) differs from the whole-stream output, q=%d" % (
                        k, l, q)
            assert not got[idx.size * q:].any(), "bits after the last listed pair are set"


ALL_PINS = [pin_fips197, pin_identity, pin_matrix, pin_no_reduction, pin_bilinear, pin_field,
            pin_hadamard, pin_balanced, pin_partition, pin_moduli, pin_sampled]
