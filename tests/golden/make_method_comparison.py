"""Times the three CPU references of the method and stores their errors (calls only synth and
oracle; test infrastructure).

  O1  exact D: dense diagonalisation, the occupied eigenprojector (the paper's exact reference
      is a tightly thresholded expansion, Results, Fig. 2 text; for a gapped H they agree)
  O2  whole-matrix thresholded SP2: the same trace-driven sequence on the full matrix, every
      entry below tau zeroed after each update (the sparse-algebra comparison of Fig. 3)
  O3  the graph-partitioned SP2 (Eq. 6; the parity reference of the GPU library)

For each workload the script records the wall time of each on this host, the SP2 steps, and the
errors of O2 and O3 against O1 with the measures of Fig. 2: max-abs, Frobenius norm per site and
band-energy error per site (E_band = Tr[D H]).  O2 at tau = 1e-12 is also run at N = 1024 as the
paper's exact reference and must agree with O1.

Usage: python tests/golden/make_method_comparison.py [n1024] [n18000]
writes tests/golden/method_comparison.json (entries are merged by workload).
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from synth import make_model, ell_sha256  # noqa: E402
from oracle.bounds import ell_to_dense  # noqa: E402
from oracle.exact import density_exact  # noqa: E402
from oracle.metrics import column_ell_to_dense, errors  # noqa: E402
from oracle.sp2 import density_partitioned, sp2_dense, x0_dense, default_idem_tol  # noqa: E402

OUT = os.path.join(HERE, "method_comparison.json")
CORE = {"n1024": 16, "n18000": 32}


def compare(name, tau=1e-5):
    from threadpoolctl import threadpool_info
    m = make_model(name)
    N, n_occ, n_sites = m["N"], m["n_occ"], m["N"] // 2
    H = ell_to_dense(m["H_col"], m["H_val"])
    rec = {"model": name, "N": N, "n_occ": n_occ, "tau": tau, "core_size": CORE[name],
           "H_sha256": ell_sha256(m["H_col"], m["H_val"]),
           "blas_threads": max([t.get("num_threads", 1) for t in threadpool_info()] or [1])}
    t = time.time()
    De, w, gap = density_exact(H, n_occ)
    rec["O1"] = {"seconds": time.time() - t, "gap": gap,
                 "idem": float(np.abs(De @ De - De).max()) if N <= 4096 else None}
    t = time.time()
    X0 = x0_dense(m["H_col"], m["H_val"])
    # thresholding holds |Tr X - Tr X^2| at a floor above the idempotency tolerance: the
    # expansion ends when it stops decreasing
    x, info = sp2_dense(X0, n_occ, default_idem_tol(N), tau=tau, stall_stop=True)
    rec["O2"] = {"seconds": time.time() - t, "iters": info["iters"],
                 "converged": info["converged"], "stalled": info["stalled"],
                 "vs_O1": errors(x, De, H, n_sites)}
    del x
    t = time.time()
    D_col, D_val, info = density_partitioned(m["H_col"], m["H_val"], n_occ, tau, CORE[name],
                                             low_memory=N > 4096)
    rec["O3"] = {"seconds": time.time() - t, "iters": info["iters"],
                 "converged": info["converged"], "branch": "".join(map(str, info["branch"])),
                 "vs_O1": errors(column_ell_to_dense(D_col, D_val), De, H, n_sites)}
    if N <= 4096:
        t = time.time()
        x, info = sp2_dense(X0, n_occ, default_idem_tol(N), tau=1e-12)
        rec["O2_tau_1e-12"] = {"seconds": time.time() - t, "iters": info["iters"],
                               "vs_O1": errors(x, De, H, n_sites)}
    return rec


def main(names):
    out = json.load(open(OUT)) if os.path.exists(OUT) else {}
    for name in names:
        rec = compare(name)
        out[name] = rec
        print(json.dumps(rec), flush=True)
        json.dump(out, open(OUT, "w"), indent=1)


if __name__ == "__main__":
    main(sys.argv[1:] or ["n1024"])
