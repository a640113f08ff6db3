"""Writes poisson3d_64_hss_ranks.txt with the oracle only: per HSS front of
the 64^3 Poisson workload (leaf 64, eps 1e-6, d0 = dd = 128, p = 10, seed 0):
front id, max row rank, max column rank, final d, growth rounds.
Takes about ten minutes on 8 cores."""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import mf  # noqa: E402
from paper_1502_07405_amd import problems as P  # noqa: E402


def main():
    A, o, b = P.workload(**P.WORKLOADS["poisson3d_64"])
    fac = mf.factor(A, o, mf.Options(min_sep_hss=512, leaf_size=64, rel_tol=1e-6, d0=128, dd=128, p=10))
    with open(os.path.join(HERE, "poisson3d_64_hss_ranks.txt"), "w") as f:
        f.write("# written by tests/golden/make_poisson3d_64.py (oracle only)\n")
        f.write("# front max_row_rank max_col_rank final_d growth_rounds\n")
        for r in mf.hss_ranks(fac):
            f.write(" ".join(str(int(v)) for v in r) + "\n")


if __name__ == "__main__":
    main()
