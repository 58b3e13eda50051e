"""Write the exact (FP64 transfer-matrix, oracle O3) log Z of the first N
syndromes of the d = 17, p = 0.12, seed-3000 workload to c3_oracle_logz.txt.

Calls only the oracle and the seeded input generator:

    python tests/golden/make_c3_oracle.py [N] [threads]

Rows already in the file are kept (the oracle is deterministic: a few of them
are recomputed first and must come out bit-identical), so raising N only adds
the missing syndromes.
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth  # noqa: E402

D, P, SEED = 17, 0.12, 3000
PATH = os.path.join(HERE, "c3_oracle_logz.txt")


def main():
    n = int(sys.argv[1]) if len(sys.argv) > 1 else 1024
    threads = int(sys.argv[2]) if len(sys.argv) > 2 else (os.cpu_count() or 1)
    rates = synth.depolarizing(D, P)
    syn = synth.sample(D, rates, n, SEED)["syndromes"]
    have = np.zeros((0, 4))
    if os.path.exists(PATH):
        have = np.loadtxt(PATH).reshape(-1, 4)[:n]
        if len(have):
            probe = [0, len(have) - 1]
            again = oracle.transfer(D, rates, syn[probe], threads=threads)
            if not np.array_equal(again, have[probe]):
                raise SystemExit("stored rows do not reproduce; regenerate from scratch")
    new = oracle.transfer(D, rates, syn[len(have):], threads=threads) if n > len(have) else np.zeros((0, 4))
    logz = np.concatenate([have, new])
    with open(PATH, "w") as f:
        f.write("# exact log Z_l (l = I, X, Y, Z) of syndromes 0..%d of: rotated surface code d=17, "
                "depolarizing p=0.12, synth.sample seed 3000; oracle O3 (FP64 transfer matrix)\n" % (n - 1))
        for row in logz:
            f.write(" ".join("%.17g" % v for v in row) + "\n")
    print("wrote", PATH, logz.shape)


if __name__ == "__main__":
    main()
