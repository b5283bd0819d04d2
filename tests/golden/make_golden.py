"""Writes the stored expected values under tests/golden/ (calls only synth and oracle).

Usage: python tests/golden/make_golden.py [hashes] [n1024] [n18000] [n100000] [n1024_ml]
                                          [n18000_ml] [n100000_ml] [n18000_levels]
(the _ml variants use the multilevel cores instead of blocks of the vertex order)
Every value written here comes from the CPU oracle in oracle/ run on the seeded
inputs from synth/; nothing comes from the GPU library.
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from synth import make_model, ell_sha256  # noqa: E402
from oracle.sp2 import density_partitioned  # noqa: E402
from oracle.exact import frontier_levels  # noqa: E402
from oracle.bounds import ell_to_dense  # noqa: E402


def write_hashes():
    out = {}
    for name in ("tiny48", "small256", "n1024", "n4096", "n18000"):
        m = make_model(name)
        out[name] = ell_sha256(m["H_col"], m["H_val"])
    json.dump(out, open(os.path.join(HERE, "model_hashes.json"), "w"), indent=1)


def write_partitioned(name, tau, core_size, n_samples=4096, seed=123, low_memory=False,
                      method="block"):
    rec = partitioned_record(name, tau, core_size, n_samples, seed, low_memory, method)
    tag = "partitioned" if method == "block" else method
    json.dump(rec, open(os.path.join(HERE, f"{name}_fp64_{tag}.json"), "w"))
    return rec


def partitioned_record(name, tau, core_size, n_samples=4096, seed=123, low_memory=False,
                       method="block"):
    """The stored record of one partitioned FP64 oracle run (graph, partition, SP2 sequence,
    traces, D hashes and sampled entries)."""
    m = make_model(name)
    t = time.time()
    D_col, D_val, info = density_partitioned(m["H_col"], m["H_val"], m["n_occ"], tau, core_size,
                                             method=method, low_memory=low_memory)
    N = m["N"]
    rng = np.random.default_rng(seed)
    rows = rng.integers(0, N, n_samples)
    nnz_row = (D_col >= 0).sum(1)
    slots = (rng.random(n_samples) * nnz_row[rows]).astype(np.int64)
    rec = {
        "model": name, "tau": tau, "core_size": core_size, "partition": method, "N": N,
        "n_occ": m["n_occ"],
        "H_sha256": ell_sha256(m["H_col"], m["H_val"]),
        "emin": info["emin"].hex(), "emax": info["emax"].hex(),
        "graph_sha256": ell_sha256(info["row_ptr"], info["col"]),
        "graph_nnz": int(len(info["col"])),
        "partition_sha256": ell_sha256(info["core_ptr"], info["sub_ptr"], info["sub_idx"]),
        "n_sub": int(len(info["sub_ptr"]) - 1),
        "max_sub": int(np.diff(info["sub_ptr"]).max()),
        "iters": info["iters"], "converged": bool(info["converged"]),
        "branch": "".join(str(b) for b in info["branch"]),
        "traces": [[a.hex(), b.hex()] for a, b in info["traces"]],
        "min_margin": info["min_margin"],
        "trace_D": info["trace"],
        "D_col_sha256": ell_sha256(D_col),
        "D_frobenius": float(np.linalg.norm(D_val)),
        "samples": [[int(r), int(s), float(D_val[r, s]).hex()] for r, s in zip(rows, slots)],
        "oracle_seconds": time.time() - t,
    }
    if method != "block":
        # the communities themselves (the CPU baseline samples them)
        rec["core_ptr"] = [int(x) for x in info["core_ptr"]]
        rec["core_vtx"] = [int(x) for x in info["core_vertices"]]
    return rec


def write_levels(name):
    """HOMO and LUMO of the model by dense diagonalisation."""
    m = make_model(name)
    t = time.time()
    eh, el = frontier_levels(ell_to_dense(m["H_col"], m["H_val"]), m["n_occ"])
    rec = {"model": name, "H_sha256": ell_sha256(m["H_col"], m["H_val"]), "n_occ": m["n_occ"],
           "e_homo": eh.hex(), "e_lumo": el.hex(), "oracle_seconds": time.time() - t}
    json.dump(rec, open(os.path.join(HERE, f"{name}_levels.json"), "w"), indent=1)


if __name__ == "__main__":
    what = sys.argv[1:] or ["hashes", "n1024"]
    if "hashes" in what:
        write_hashes()
    if "n1024" in what:
        write_partitioned("n1024", 1e-5, 16)
    if "n18000" in what:
        write_partitioned("n18000", 1e-5, 32)
    if "n100000" in what:
        write_partitioned("n100000", 1e-5, 32, low_memory=True)
    if "n1024_ml" in what:
        write_partitioned("n1024", 1e-5, 16, method="multilevel")
    if "n18000_levels" in what:
        write_levels("n18000")
    if "n100000_ml" in what:
        write_partitioned("n100000", 1e-5, 32, method="multilevel", low_memory=True)
    if "n18000_ml" in what:
        write_partitioned("n18000", 1e-5, 32, method="multilevel", low_memory=True)
