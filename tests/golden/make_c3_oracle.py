"""Write the exact (FP64 transfer-matrix, oracle O3) log Z of the first N
syndromes of the d = 17, p = 0.12, seed-3000 workload to c3_oracle_logz.txt.

Calls only the oracle and the seeded input generator:

    python tests/golden/make_c3_oracle.py [N] [threads]
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth  # noqa: E402

D, P, SEED = 17, 0.12, 3000


def main():
    n = int(sys.argv[1]) if len(sys.argv) > 1 else 1024
    threads = int(sys.argv[2]) if len(sys.argv) > 2 else (os.cpu_count() or 1)
    rates = synth.depolarizing(D, P)
    syn = synth.sample(D, rates, n, SEED)["syndromes"]
    logz = oracle.transfer(D, rates, syn, threads=threads)
    path = os.path.join(HERE, "c3_oracle_logz.txt")
    with open(path, "w") as f:
        f.write("# exact log Z_l (l = I, X, Y, Z) of syndromes 0..%d of: rotated surface code d=17, "
                "depolarizing p=0.12, synth.sample seed 3000; oracle O3 (FP64 transfer matrix)\n" % (n - 1))
        for row in logz:
            f.write(" ".join("%.17g" % v for v in row) + "\n")
    print("wrote", path, logz.shape)


if __name__ == "__main__":
    main()
