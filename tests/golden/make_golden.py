"""Writes the stored expected values under tests/golden/ using only the oracle package.

Run from the repository root: python tests/golden/make_golden.py
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import exact_sc  # noqa: E402

# Fig. 1: 4 vertices, 5 edges, A and D of degree 2, B and C of degree 3 (K4 minus A-D).
# A=0, B=1, C=2, D=3.
TOY_EDGES = [(0, 1), (0, 2), (1, 2), (1, 3), (2, 3)]


def main():
    sc, total = exact_sc.sc_enumerate(TOY_EDGES, 4)
    with open(os.path.join(HERE, "fig1_toy.txt"), "w") as f:
        f.write("# Sample graph of Fig. 1 (Sec. 2): A,D degree 2; B,C degree 3; ids A=0 B=1 C=2 D=3.\n")
        f.write("# The caption states SC = 1/2 for every edge; enumerating the spanning trees\n")
        f.write("# (written by make_golden.py with oracle.exact_sc.sc_enumerate) gives the values below.\n")
        f.write(f"# spanning_trees {total}\n")
        f.write("# u v sc_numerator sc_denominator\n")
        for (u, v), s in zip(TOY_EDGES, sc):
            f.write(f"{u} {v} {s.numerator} {s.denominator}\n")


if __name__ == "__main__":
    main()
