"""Writes the 64^3 Poisson goldens with the oracle only (leaf 64, eps 1e-6,
d0 = dd = 128, p = 10, seed 0):

- poisson3d_64_hss_ranks.txt: per HSS front, front id, max row rank, max
  column rank, final d, growth rounds;
- poisson3d_64_vectors.npz: ``minv_v`` = M^{-1} v for v drawn from
  default_rng(7) (standard normal, length N), one application of the
  oracle's factors; ``x`` = the solution of A x = b for the workload's b
  (default_rng(1)), iterative refinement with those factors to a relative
  residual of 1e-12; ``relres`` its final residual, ``its`` its steps;
- poisson3d_64_work.json: the algorithmic work of that factorization per
  stage (flops, HBM bytes) and the HBM bytes of one M^{-1} application and
  of one sparse product, counted by oracle.work.

Run:  python tests/golden/make_poisson3d_64.py [--vectors-only]
Takes about ten minutes on 8 cores."""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import krylov, mf, work  # noqa: E402
from paper_1502_07405_amd import problems as P  # noqa: E402


def main():
    A, o, b = P.workload(**P.WORKLOADS["poisson3d_64"])
    fac = mf.factor(A, o, mf.Options(min_sep_hss=512, leaf_size=64, rel_tol=1e-6, d0=128, dd=128, p=10))
    if "--vectors-only" not in sys.argv:
        with open(os.path.join(HERE, "poisson3d_64_hss_ranks.txt"), "w") as f:
            f.write("# written by tests/golden/make_poisson3d_64.py (oracle only)\n")
            f.write("# front max_row_rank max_col_rank final_d growth_rounds\n")
            for r in mf.hss_ranks(fac):
                f.write(" ".join(str(int(v)) for v in r) + "\n")
    v = np.random.default_rng(7).standard_normal(A.n)
    minv_v = mf.apply_inverse(fac, v)
    S = A.to_scipy()
    x, its, hist = krylov.refine(lambda z: S @ z, lambda r: mf.apply_inverse(fac, r), b, 1e-12, max_it=50)
    np.savez_compressed(os.path.join(HERE, "poisson3d_64_vectors.npz"), minv_v=minv_v, x=x,
                        relres=np.float64(hist[-1]), its=np.int64(its))
    print(f"refinement: {its} steps, relres {hist[-1]:.3e}")
    out = {"factorization": work.factorization_work(fac), "apply_bytes": work.apply_bytes(fac),
           "spmv_bytes": work.spmv_bytes(A), "refinement_steps": int(its)}
    with open(os.path.join(HERE, "poisson3d_64_work.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
