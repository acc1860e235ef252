"""Write oracle/moduli.txt: the conventional modulus of each degree used by
the tests, found by the oracle's own search (orc_find_modulus).

Usage:  python -m oracle.gen_moduli [--jobs N] [q ...]

Each line holds the exponents of P in decreasing order (q first, 0 last).
Calls only code under oracle/.
"""
from __future__ import annotations

import os
import sys
import time

import oracle

DEFAULT_DEGREES = sorted(set(
    list(range(2, 65))
    + list(range(8, 1025, 8))
    # Algorithm 2 at b = 16, Delta = 1 from q_1 = 80: the first 320 blocks
    + list(range(80, 5200, 16))
    + [1536, 2048, 3072, 4096, 8192, 16384]
))


def _search(q):
    t0 = time.time()
    return q, oracle.find_modulus(q), time.time() - t0


def main(argv):
    jobs = 1
    if argv[:1] == ["--jobs"]:
        jobs, argv = int(argv[1]), argv[2:]
    degrees = [int(a) for a in argv] if argv else DEFAULT_DEGREES
    table = dict(oracle._read_table())
    todo = [q for q in degrees if q not in table]
    # the largest degrees first, so that the pool ends with short searches
    todo.sort(reverse=True)
    if jobs > 1:
        import multiprocessing as mp

        with mp.Pool(jobs) as pool:
            for q, exps, dt in pool.imap_unordered(_search, todo):
                table[q] = exps
                print("q=%d %r  %.1fs" % (q, exps, dt), flush=True)
                _write(table)
    else:
        for q in todo:
            q, table[q], dt = _search(q)
            print("q=%d %r  %.1fs" % (q, table[q], dt), flush=True)
            _write(table)
    _write(table)


def _write(table):
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "moduli.txt")
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        f.write("# exponents of the conventional modulus P of degree q (q first, 0 last):\n")
        f.write("# lowest weight, then lexicographically smallest; written by oracle/gen_moduli.py\n")
        for q in sorted(table):
            f.write(" ".join(str(v) for v in table[q]) + "\n")
    os.replace(tmp, path)


if __name__ == "__main__":
    main(sys.argv[1:])
