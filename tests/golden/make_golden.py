"""Writes the stored expected values under tests/golden/ that come from the
oracle: the brute-force Graver basis (both signs) of the tiny m=2, n=8
instances in the box [-6, 6]^8.  Calls only the oracle and the seeded input
generators.  Run from the repository root:  python tests/golden/make_golden.py
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle.conformal import graver_basis_in_box  # noqa: E402
from paper_2412_13576_amd import workloads as W  # noqa: E402


def main():
    path = os.path.join(HERE, "tiny_graver_box6.txt")
    with open(path, "w") as fh:
        fh.write("# Brute-force Graver basis G(A) within [-6,6]^8 of the tiny m=2, n=8\n")
        fh.write("# instances (workloads.tiny_instance(seed)), written by make_golden.py\n")
        fh.write("# from oracle.conformal.graver_basis_in_box.  One element per line.\n")
        for seed in range(1000, 1005):
            inst = W.tiny_instance(seed)
            G = graver_basis_in_box(inst.A, 6)
            fh.write(f"seed {seed} count {len(G)}\n")
            for g in G:
                fh.write(" ".join(str(x) for x in g) + "\n")
    print("wrote", path)


if __name__ == "__main__":
    main()
