"""Write tests/golden/tiny_oracle.txt: digest of the CPU oracle's output on
the tiny workload (n = 1024, m = 256, 1024 pairs, seeds 1 and 2).

Calls only the oracle and the seeded input generator.
Usage:  python tests/golden/gen_golden.py
"""
import hashlib
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2402_14607_amd import inputs  # noqa: E402


def main():
    w = inputs.tiny()
    z = oracle.ext_blocks(w.x, w.y, w.n_bits, w.m_bits)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tiny_oracle.txt")
    with open(path, "w") as f:
        f.write("# oracle output on the tiny workload (n=1024, m=256, 1024 pairs, seeds 1, 2)\n")
        f.write("bytes=%d\n" % z.size)
        f.write("sha256=%s\n" % hashlib.sha256(z.tobytes()).hexdigest())
        f.write("input_sha256=%s\n" % hashlib.sha256(w.x.tobytes() + w.y.tobytes()).hexdigest())
        f.write("first32=%s\n" % z[:32].tobytes().hex())
    print(open(path).read())


if __name__ == "__main__":
    main()
