"""Throughput of the graph-partitioned SP2 density matrix on one MI355X.

One step = the whole hot path on one synthetic system already resident in HBM: spectral
bounds, X2 graph, cores with halos, gather, batched SP2 squarings with the FP64 trace/branch
decision, FP64 refinement (mixed precision), scatter into column-ELL D.  Prints one JSON line:
the headline precision (default: two fp16 planes, three products), the other split method and
the FP64 path beside it, the roofline of the squaring kernel and the CPU oracle on a sample.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision fp16x3|bf16x6|fp32|fp64]
                  [--workload n18000|n100000|n1024] [--no-cpu-baseline]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "orbitals/s of D at ≤1e-6 err vs FP64 oracle; mixed vs FP64 GPU; X² MFMA util"
# dense matrix-core peaks of the precision the dominant squaring kernel runs in (TFLOP/s)
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16": 2500.0, "bf16x3": 2500.0, "bf16x6": 2500.0,
               "fp16x3": 2500.0}
# plane products per algorithmic multiply-add of the split squares
PLANE_PRODUCTS = {"bf16": 1, "bf16x3": 3, "bf16x6": 6, "fp16x3": 3}
# default cores per workload: the faster of the two partitions as measured on one MI355X
# (multilevel communities pay for their partitioner at N = 18000 and N = 100000, not at
# N = 1024, where it would take a large share of a 10 ms step)
WORKLOADS = {"n18000": dict(tau=1e-5, core=32, partition="multilevel"),
             "n1024": dict(tau=1e-5, core=16, partition="block"),
             "n100000": dict(tau=1e-5, core=32, partition="multilevel")}


def kernel_source_hash() -> str:
    import hashlib
    path = os.path.join(ROOT, "paper_1603_00937_amd", "csrc", "sp2.hip")
    return hashlib.sha256(open(path, "rb").read()).hexdigest()


def measured_traffic(workload, kernel, partition):
    """HBM bytes per launch of the squaring kernel from the committed rocprofv3 counter runs
    (FETCH_SIZE + WRITE_SIZE scaled by a plain copy of known size), or None when no record
    exists for this workload, partition and kernel or the kernel source changed since it was
    taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    for rec in json.load(open(path)):
        if (rec["workload"] == workload and rec["kernel"] == kernel
                and rec.get("partition") == partition
                and rec["sp2_source_sha256"] == kernel_source_hash()):
            return rec["bytes_per_launch"]
    return None


def square_kernel_name(precision, stats):
    """The rocprof name of the loop's squaring kernel for this run."""
    if precision.startswith("bf16") or precision == "fp16x3":
        planes = {"bf16": 1, "bf16x3": 2, "bf16x6": 3, "fp16x3": 2}[precision]
        edge = 64 if stats["n_tile64"] == stats["n_sub"] else 128
        if precision == "fp16x3" and 2 * stats.get("n_split_il", 0) > stats["n_sub"]:
            return f"k_symm_mm_split_il<{edge}>"
        return f"k_symm_mm_split<{planes}, {'true' if precision == 'fp16x3' else 'false'}, {edge}>"
    t = "double" if precision == "fp64" else "float"
    if stats.get("n_stage3", 0) == stats["n_sub"]:
        return f"k_symm_mm<{t}, 0, 64, 3, 0>"
    if stats.get("n_regstage", 0) == stats["n_sub"]:
        return f"k_symm_mm<{t}, 0, 64, 2, 1>"
    edge = 64 if stats["n_tile64"] == stats["n_sub"] else 128
    return f"k_symm_mm<{t}, 0, {edge}, 2, 0>"


def _working(vals, frac=0.05):
    """The dispatches that did the work: the device-driven loop enqueues steps past the stop
    whose launches return at once; they read as near-zero durations or counter values."""
    top = max(vals) if vals else 0.0
    return [v for v in vals if v >= frac * top]


def _largest_grid_counter(db, prefix, counter):
    """(kernel, average value) of ``counter`` over the largest-grid working dispatches of the
    most often dispatched kernel whose short name starts with one of ``prefix`` (the SP2 loop's
    squaring kernel, not the autotuner's one-off variants; None: a device copy)."""
    import sqlite3
    c = sqlite3.connect(db)
    rows = c.execute("select kernel_name, grid_size, counter_name, value from counters_collection"
                     ).fetchall()
    per = {}
    for name, grid, cname, val in rows:
        short = name.replace("gbi::(anonymous namespace)::", "").replace("void ", "", 1)
        short = short.split("(")[0]
        if cname != counter:
            continue
        if prefix is None:
            if "copy" not in short.lower():
                continue
        elif not short.startswith(tuple(prefix)):
            continue
        per.setdefault(short, {}).setdefault(grid, []).append(float(val))
    name = max(per, key=lambda k: sum(len(v) for v in per[k].values()))
    w = _working(per[name][max(per[name])])
    return name, sum(w) / len(w)


def traffic_from_pmc(pmc_dir, workload="n18000"):
    """Per-launch HBM bytes of the squaring kernels from FETCH_SIZE / WRITE_SIZE passes (KiB
    per dispatch, largest-grid dispatches), each scaled by what the same counter reads for a
    device copy of 4 GiB (the --copy-calibration run).  Prints the records for traffic.json."""
    nbytes = 4 << 30
    _, cf = _largest_grid_counter(os.path.join(pmc_dir, "copy_fetch", "run_results.db"), None,
                                  "FETCH_SIZE")
    _, cw = _largest_grid_counter(os.path.join(pmc_dir, "copy_write", "run_results.db"), None,
                                  "WRITE_SIZE")
    sf, sw = nbytes / (cf * 1024.0), nbytes / (cw * 1024.0)
    recs = []
    for tag in sorted(os.listdir(pmc_dir)):
        if not tag.endswith("_fetch") or tag.startswith("copy"):
            continue
        run = tag[:-len("_fetch")]
        f = os.path.join(pmc_dir, tag, "run_results.db")
        w = os.path.join(pmc_dir, run + "_write", "run_results.db")
        if not (os.path.exists(f) and os.path.exists(w)):
            continue
        prefix = ("k_symm_mm_split",) if run.startswith(("bf16", "fp16")) else (
            ("k_symm_mm<double, 0,",) if run.startswith("fp64") else ("k_symm_mm<float, 0,",))
        kf, fv = _largest_grid_counter(f, prefix, "FETCH_SIZE")
        kw, wv = _largest_grid_counter(w, prefix, "WRITE_SIZE")
        assert kf == kw, (kf, kw)
        fb, wb = fv * 1024.0 * sf, wv * 1024.0 * sw
        # run names: <precision>_<partition> (the counter passes' directories)
        part = "multilevel" if "_multilevel" in run else "block"
        recs.append({"workload": workload, "kernel": kf, "run": run, "partition": part,
                     "sp2_source_sha256": kernel_source_hash(), "fetch_bytes": fb,
                     "write_bytes": wb, "bytes_per_launch": fb + wb,
                     "copy_scale_fetch": sf, "copy_scale_write": sw})
    print(json.dumps(recs, indent=1))


def run_step(gb, Hc, Hv, n_occ, tau, core, D, args, times=None):
    import torch
    t0 = time.perf_counter()
    g = gb.build_graph(Hc, Hv, tau)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    p = gb.partition(g, core, method=args.partition)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    if times is not None:
        times["graph"] += (t1 - t0) * 1e3
        times["part"] += (t2 - t1) * 1e3
    return gb.density(Hc, Hv, n_occ, tau, partition=p, core_size=core, precision=args.precision,
                      D=D, launch_mode=args.launch_mode, tile_policy=args.tile_policy,
                      tile_order=args.tile_order, refine=args.refine,
                      n_fp64_first=args.n_fp64_first)


def rocpd_summary(path):
    """Per-kernel summary of a rocprofv3 database (--kernel-trace): calls, total and average
    duration; for each kernel also its largest-grid working launches (the SP2 loop's batched
    launches, not the autotuner's single-bucket ones nor the device-driven loop's launches past
    the stop, which return at once)."""
    import sqlite3
    c = sqlite3.connect(path)
    rows = c.execute("select name, duration, grid_x from kernels").fetchall()
    agg = {}
    for name, dur, grid in rows:
        short = name.replace("gbi::(anonymous namespace)::", "").replace("void ", "", 1)
        short = short.split("(")[0]
        a = agg.setdefault(short, [0, 0.0, {}])
        a[0] += 1
        a[1] += dur
        a[2].setdefault(grid, []).append(float(dur))
    total = sum(v[1] for v in agg.values())
    print("| kernel | calls | total ms | avg ms | % | largest-grid working launches: calls, "
          "avg ms (launches past the stop) |")
    print("|---|---|---|---|---|---|")
    for k, (n, t, grids) in sorted(agg.items(), key=lambda kv: -kv[1][1]):
        gmax = max(grids)
        w = _working(grids[gmax])
        print(f"| {k} | {n} | {t / 1e6:.3f} | {t / n / 1e6:.4f} | {100 * t / total:.1f} | "
              f"{len(w)}, {sum(w) / len(w) / 1e6:.4f} (grid {gmax // 256} WGs; "
              f"{len(grids[gmax]) - len(w)}) |")


def rocpd_counters(path):
    """Per-kernel hardware counter values of a rocprofv3 --pmc database: for each kernel and
    counter, dispatches, average and total value, and the average over the largest-grid
    working dispatches (the SP2 loop's batched launches)."""
    import sqlite3
    c = sqlite3.connect(path)
    rows = c.execute("select kernel_name, grid_size, counter_name, value from counters_collection"
                     ).fetchall()
    agg = {}
    for name, grid, cname, val in rows:
        short = name.replace("gbi::(anonymous namespace)::", "").replace("void ", "", 1)
        short = short.split("(")[0]
        agg.setdefault((short, cname), {}).setdefault(grid, []).append(float(val))
    print("| kernel | counter | dispatches | average | total | largest-grid working average "
          "(dispatches) |")
    print("|---|---|---|---|---|---|")
    for (k, cname), d in sorted(agg.items(), key=lambda kv: -sum(sum(g) for g in kv[1].values())):
        n = sum(len(g) for g in d.values())
        t = sum(sum(g) for g in d.values())
        w = _working(d[max(d)])
        print(f"| {k} | {cname} | {n} | {t / n:.6g} | {t:.6g} | {sum(w) / len(w):.6g} "
              f"({len(w)}) |")


def md_run(args):
    """Adaptive-graph displacement loop (the MD use of the paper's Eq. 8 estimate): each step
    displaces every site by N(0, sigma^2) per coordinate, rebuilds H on the host, derives the
    graph from the previous D and the new H (|D| >= 1e-4 united with the X2 graph), partitions,
    computes D and the gradient of Tr[D V].  Prints one JSON line with per-step statistics."""
    import torch
    import paper_1603_00937_amd as gb
    from synth import make_model, operator_v_pairs, displace_sites, rebuild_hamiltonian
    cfg = WORKLOADS[args.workload]
    m = make_model(args.workload)
    rng = np.random.default_rng(52)
    dev = torch.device("cuda:0")
    up = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
    Hc, Hv = up(m["H_col"]), up(m["H_val"])
    p = gb.partition(gb.build_graph(Hc, Hv, cfg["tau"]), cfg["core"], method=args.partition)
    D_col, D_val, st = gb.density(Hc, Hv, m["n_occ"], cfg["tau"], partition=p)
    steps = []
    pos = m["pos"]
    prev_branch = st["branch"] + [0, 1]
    for t in range(args.md_steps):
        pos = displace_sites(pos, m["L"], 0.02, rng)
        m = rebuild_hamiltonian(m, pos)
        Hc, Hv = up(m["H_col"]), up(m["H_val"])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g = gb.build_graph(Hc, Hv, cfg["tau"], mode="dprev", aux=(D_col, D_val), tau_aux=1e-4)
        torch.cuda.synchronize()
        tp = time.perf_counter()
        # cores from the new graph each step, or (--md-carry-cores) the previous step's multilevel
        # communities carried over with their halos on the new graph (on-the-fly update)
        if args.partition == "multilevel" and args.md_carry_cores:
            p = gb.partition_update(g, p)
        else:
            p = gb.partition(g, cfg["core"], method=args.partition)
        torch.cuda.synchronize()
        part_ms = (time.perf_counter() - tp) * 1e3
        # pre-determined sequence (MD section), no trace rule during the expansion: "replay"
        # repeats the previous step's branches plus one X^2 / 2X - X^2 pair as a margin; "gap"
        # builds the sequence from the HOMO/LUMO bracket estimated from the previous step's
        # traces (bounds narrowed by 5 % of their width).  Either falls back to the trace-driven
        # rule if the replay ends short of the stop test.
        seq = None
        if args.md_sequence == "replay":
            seq = prev_branch
        elif args.md_sequence == "gap":
            try:
                est = gb.sp2_estimate_gap(**gb.gap_inputs(st, m["n_occ"]))
                hb, lb = est["homo_bound"], est["lumo_bound"]
                lo, hi = gb.spectral_bounds(Hc, Hv)
                # both frontier images within 1 % of the stop tolerance of 0 or 1
                delta = 1e-12 * m["N"] / 1024.0
                seq = gb.sp2_sequence(lo, hi, hb + 0.05 * (lb - hb), lb - 0.05 * (lb - hb), delta)
            except gb.GbError:
                seq = None
        replayed = seq is not None
        D_col, D_val, st = gb.density(Hc, Hv, m["n_occ"], cfg["tau"], partition=p,
                                      core_size=cfg["core"], keep_tape=True, branch_in=seq)
        fallback = False
        if replayed and not st["converged"]:
            st.pop("tape")
            D_col, D_val, st = gb.density(Hc, Hv, m["n_occ"], cfg["tau"], partition=p,
                                          core_size=cfg["core"], keep_tape=True)
            fallback = True
        prev_branch = (st["branch"][:st["iters"]] if args.md_sequence != "replay" or fallback
                       else prev_branch[:-2]) + [0, 1]
        # dL/dD for L = Tr[D V] on D's pattern (V on H's pattern), then the adjoint
        tape = st.pop("tape")
        # V on this step's pattern (the ELL width of H changes as sites move; a pair keeps its
        # value from step to step)
        Vd = up(operator_v_pairs(m["H_col"], 51))
        if Vd.shape != Hc.shape:
            raise RuntimeError("V must have H's ELL shape")
        # V[i, r] for the entries r of column i of D that lie on row i of H (searchsorted in
        # the ascending ELL row; padding -1 mapped past every column)
        big = np.iinfo(np.int32).max
        Hs = torch.where(Hc >= 0, Hc, torch.full_like(Hc, big)).long().contiguous()
        rows = D_col.long().contiguous()
        slot = torch.searchsorted(Hs, rows).clamp(max=Hs.shape[1] - 1)
        hit = (torch.gather(Hs, 1, slot) == rows) & (rows >= 0)
        GD = torch.where(hit, torch.gather(Vd, 1, slot), torch.zeros_like(D_val))
        L = float((GD * D_val).sum())
        G_H = tape.vjp(GD.contiguous())
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        sizes = np.diff(p.arrays()[1].cpu().numpy())
        steps.append({"step": t + 1, "ms": dt * 1e3, "part_ms": part_ms,
                      "sum_n3": float((sizes.astype(np.float64) ** 3).sum()),
                      "iters": st["iters"],
                      "converged": st["converged"], "replayed": replayed,
                      "fallback": fallback, "seq_len": len(seq) if replayed else None,
                      "graph_nnz": g.nnz,
                      "sub_min": int(sizes.min()), "sub_mean": float(sizes.mean()),
                      "sub_max": int(sizes.max()), "trace_DV": L,
                      "grad_norm": float(G_H.norm())})
        print(json.dumps(steps[-1]), file=sys.stderr, flush=True)
    print(json.dumps({"md_steps": steps, "workload": args.workload}), flush=True)


def foe_run(args):
    """Finite-temperature Chebyshev expansion (the Fermi function of Eq. 7) on the workload's
    partition: one JSON line with orbitals/s of the whole path and the roofline of the batched
    product (one launch per Chebyshev term)."""
    import torch
    import paper_1603_00937_amd as gb
    from synth import make_model
    cfg = WORKLOADS[args.workload]
    m = make_model(args.workload)
    N = m["N"]
    dev = torch.device("cuda:0")
    Hc = torch.from_numpy(m["H_col"]).to(dev)
    Hv = torch.from_numpy(m["H_val"]).to(dev)
    mu = None if args.mu is None else float(args.mu)

    def step():
        g = gb.build_graph(Hc, Hv, cfg["tau"])
        p = gb.partition(g, cfg["core"])
        return gb.foe_density(Hc, Hv, m["n_occ"], cfg["tau"], args.beta, args.order, mu=mu,
                              partition=p)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    prod_ms, prod_n = 0.0, 0
    for _ in range(args.steps):
        _, _, st = step()
        prod_ms += st["ms_product"]
        prod_n += st["n_product"]
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    avg = prod_ms / prod_n / 1e3 if prod_n else None
    ach = st["product_flops"] / avg / 1e12 if avg else None
    print(json.dumps({
        "metric": "orbitals/s of the finite-temperature D (Chebyshev Fermi expansion)",
        "value": N / dt, "unit": "orbitals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{args.workload}: N={N}, tau={cfg['tau']}, cores of {cfg['core']}",
                   "beta": args.beta, "order": args.order,
                   "mu": "solved for n_occ" if mu is None else mu, "passes": st["passes"],
                   "n_sub": st["n_sub"], "max_sub": st["max_sub"]},
        "roofline": {"bound": "mfma", "achieved": ach, "peak": PEAK_TFLOPS["fp64"],
                     "unit": "TFLOP/s", "frac": ach / PEAK_TFLOPS["fp64"] if ach else None,
                     "traffic": None, "kernel": "k_symm_mm MODE 3 (Ht T_n) + k_cheb_combine",
                     "flops_per_launch_alg": st["product_flops"],
                     "avg_launch_ms": avg * 1e3 if avg else None},
        "result": {"mu": st["mu"], "trace": st["trace"], "coef_tail": st["coef_tail"]},
        "stage_ms": {k[3:]: st[k] for k in st if k.startswith("ms_")},
    }), flush=True)


def copy_calibration(nbytes=4 << 30, reps=5):
    """A plain device copy of known size (the scale for rocprof FETCH_SIZE / WRITE_SIZE)."""
    import torch
    x = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    y = torch.empty_like(x)
    for _ in range(reps):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "reps": reps}))


def host_cpu():
    """CPU model and the number of cores this process may use (the oracle's host)."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return model, len(os.sched_getaffinity(0))


def cpu_baseline(model, workload, golden, n_sub_sample):
    """The CPU oracle on a bounded sample: graph rows of the sampled cores, their halos,
    gather and the full SP2 sequence (the oracle's own branch sequence, replayed, since
    the branch needs every subgraph's trace) for n_sub_sample subgraphs.  Returns the record
    and the oracle's D columns of the sampled cores (for the element-wise comparison)."""
    from threadpoolctl import threadpool_info
    from oracle.subgraphs import core_columns
    cfg = WORKLOADS[workload]
    N = model["N"]
    core = cfg["core"]
    if golden and "core_ptr" in golden:
        # the oracle's own communities, stored with its run
        cptr = np.asarray(golden["core_ptr"])
        cvtx = np.asarray(golden["core_vtx"], dtype=np.int32)
        kind = golden.get("partition", "stored") + " cores"
    else:
        cptr = np.minimum(np.arange(0, N + core, core), N)
        cvtx = np.arange(N, dtype=np.int32)
        kind = "block cores"
    n_cores = len(cptr) - 1
    rng = np.random.default_rng(0)
    picks = np.sort(rng.choice(n_cores, size=min(n_sub_sample, n_cores), replace=False))
    branch = [int(c) for c in golden["branch"]]
    cores = [cvtx[cptr[c]:cptr[c + 1]] for c in picks]
    t0 = time.time()
    cols = core_columns(model["H_col"], model["H_val"], model["n_occ"], cfg["tau"], cores, branch)
    dt = time.time() - t0
    threads = max([t.get("num_threads", 1) for t in threadpool_info()] or [1])
    cpu_model, n_cpu = host_cpu()
    k = sum(len(c) for c in cores)
    rec = {"value": float(k / dt), "unit": "orbitals/s", "cores": int(threads),
           "kind": "oracle", "cpu_model": cpu_model, "host_cpus": n_cpu,
           "sample": f"{len(picks)} of {n_cores} subgraphs of {workload}, {kind} (graph rows, "
                     f"halo, gather, the {len(branch)} SP2 steps of the oracle's sequence), "
                     f"{dt:.1f} s on {threads} BLAS threads"}
    return rec, list(zip(cores, cols))


def d_errors(dc, dv, ref_cols):
    """Max-abs and Frobenius error of D (column-ELL host arrays) against the oracle on whole
    sampled subgraphs (every entry of their core columns); the pattern must match."""
    worst, sq, n_ent, pattern_ok = 0.0, 0.0, 0, True
    for verts, (rows, vals) in ref_cols:
        n = len(rows)
        pattern_ok &= bool(np.array_equal(dc[verts, :n], np.broadcast_to(rows, (len(verts), n))))
        d = dv[verts, :n] - vals
        worst = max(worst, float(np.abs(d).max()))
        sq += float((d * d).sum())
        n_ent += d.size
    return {"max_abs": worst, "frobenius": float(np.sqrt(sq)), "entries": n_ent,
            "subgraphs": len(ref_cols), "pattern_equal": pattern_ok}


def idempotency(dc, dv, col_sets):
    """|D^2 - D| on the given columns of the assembled D (column-ELL host arrays): column j of
    D^2 is the sum over the rows r of column j of D[r, j] * column r of D.  Returns max-abs and
    Frobenius norm over those columns."""
    worst, sq = 0.0, 0.0
    for cols in col_sets:
        rows_j = [dc[j][dc[j] >= 0] for j in cols]
        R = np.unique(np.concatenate(rows_j))                # rows of the chosen columns
        cr = [dc[r][dc[r] >= 0] for r in R]
        U = np.unique(np.concatenate(cr + [R]))              # rows of D^2 on those columns
        M = np.zeros((len(U), len(R)))
        for a, r in enumerate(R):
            M[np.searchsorted(U, cr[a]), a] = dv[r][:len(cr[a])]
        B = np.zeros((len(R), len(cols)))
        Dj = np.zeros((len(U), len(cols)))
        for b, (j, rj) in enumerate(zip(cols, rows_j)):
            B[np.searchsorted(R, rj), b] = dv[j][:len(rj)]
            Dj[np.searchsorted(U, rj), b] = dv[j][:len(rj)]
        E = M @ B - Dj
        worst = max(worst, float(np.abs(E).max()))
        sq += float((E * E).sum())
    return {"max_abs": worst, "frobenius": float(np.sqrt(sq)),
            "columns": int(sum(len(c) for c in col_sets))}


def sym_square_flops(sizes, planes):
    """Algorithmic flops of one symmetric squaring launch: the n(n+1)/2 upper entries of each
    block's X^2, 2n flops each, times the bf16 plane products of the split method."""
    n = np.asarray(sizes, dtype=np.float64)
    return float((n * n * (n + 1.0)).sum()) * planes


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", default="fp16x3",
                    choices=["fp64", "fp32", "bf16", "bf16x3", "bf16x6", "fp16x3"])
    ap.add_argument("--launch-mode", default="device",
                    choices=["device", "per_subgraph", "graph", "host"])
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--traffic-from-pmc", default=None,
                    help="per-launch HBM bytes from a directory of rocprofv3 --pmc runs")
    ap.add_argument("--tile-policy", default="auto",
                    choices=["auto", "128", "64", "64s3", "64r", "128i", "64i"])
    ap.add_argument("--tile-order", default="xcd", choices=["xcd", "plain"])
    ap.add_argument("--refine", default="mcweeny", choices=["mcweeny", "sp2", "mcweeny_blocks"])
    ap.add_argument("--n-fp64-first", type=int, default=0)
    ap.add_argument("--partition", default=None, choices=["block", "multilevel"],
                    help="cores: multilevel communities of at most the core size, or blocks of "
                         "the (spatially sorted) vertex order (default: per workload)")
    ap.add_argument("--rocpd-summary", default=None, help="summarise a rocprofv3 database")
    ap.add_argument("--rocpd-counters", default=None,
                    help="summarise the counters of a rocprofv3 --pmc database")
    ap.add_argument("--md-sequence", default="trace", choices=["trace", "replay", "gap"],
                    help="MD: choose each branch from the traces, replay the previous step's "
                         "sequence, or build it from the gap estimated from its traces")
    ap.add_argument("--md-carry-cores", action="store_true",
                    help="MD with multilevel communities: carry the previous step's cores")
    ap.add_argument("--md-steps", type=int, default=0,
                    help="run the adaptive-graph displacement loop instead of the benchmark")
    ap.add_argument("--workload", default="n18000", choices=list(WORKLOADS))
    ap.add_argument("--foe", action="store_true",
                    help="time the finite-temperature Chebyshev expansion instead of SP2")
    ap.add_argument("--beta", type=float, default=5.0, help="FOE inverse temperature (1/eV)")
    ap.add_argument("--order", type=int, default=300, help="FOE Chebyshev order")
    ap.add_argument("--mu", default=None, help="FOE chemical potential (default: solved)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-compare", action="store_true",
                    help="skip the FP64 GPU measurement reported beside a mixed-precision run")
    ap.add_argument("--cpu-sample", type=int, default=96)
    args = ap.parse_args()
    if args.partition is None:
        args.partition = WORKLOADS[args.workload]["partition"]
    if args.rocpd_summary:
        rocpd_summary(args.rocpd_summary)
        return
    if args.rocpd_counters:
        rocpd_counters(args.rocpd_counters)
        return
    if args.copy_calibration:
        copy_calibration()
        return
    if args.traffic_from_pmc:
        traffic_from_pmc(args.traffic_from_pmc, args.workload)
        return
    if args.md_steps:
        md_run(args)
        return
    if args.foe:
        foe_run(args)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(subgraphs would shard across GPUs with one 16-byte trace all-reduce per "
              "SP2 iteration; see DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1603_00937_amd as gb
    from synth import make_model, ell_sha256

    cfg = WORKLOADS[args.workload]
    model = make_model(args.workload)
    N = model["N"]
    tag = "partitioned" if args.partition == "block" else args.partition
    gpath = os.path.join(ROOT, "tests", "golden", f"{args.workload}_fp64_{tag}.json")
    golden = json.load(open(gpath)) if os.path.exists(gpath) else None
    if golden and golden["H_sha256"] != ell_sha256(model["H_col"], model["H_val"]):
        golden = None
    dev = torch.device("cuda:0")
    Hc = torch.from_numpy(model["H_col"]).to(dev)
    Hv = torch.from_numpy(model["H_val"]).to(dev)
    g = gb.build_graph(Hc, Hv, cfg["tau"])
    p = gb.partition(g, cfg["core"], method=args.partition)
    sizes = np.diff(p.arrays()[1].cpu().numpy())
    core_sizes = np.diff(p.arrays()[0].cpu().numpy())
    D = (torch.empty((N, p.max_sub), dtype=torch.int32, device=dev),
         torch.empty((N, p.max_sub), dtype=torch.float64, device=dev))
    del g, p

    out = measure(gb, torch, args, args.precision, model, cfg, Hc, Hv, D, golden, sizes)
    out["stage_hbm_gbps"] = stage_hbm(out["stage_ms"], sizes, core_sizes, model,
                                      args.precision)
    dcm, dvm = D[0].cpu().numpy(), D[1].cpu().numpy()
    low = args.precision != "fp64"
    dcf = dvf = None
    if low and not args.no_fp64_compare:
        ref = measure(gb, torch, args, "fp64", model, cfg, Hc, Hv, D, golden, sizes)
        dcf, dvf = D[0].cpu().numpy(), D[1].cpu().numpy()
        out["fp64_gpu"] = {k: ref[k] for k in ("value", "ms_per_step", "roofline", "accuracy")}
        out["speedup_vs_fp64_gpu"] = out["value"] / ref["value"]
    # the other split method beside the headline run: three bf16 planes (six products) beside
    # two fp16 planes (three products), and the reverse
    ext = None
    alt = {"fp16x3": "bf16x6", "bf16x6": "fp16x3"}.get(args.precision)
    if alt and not args.no_fp64_compare:
        ext = measure(gb, torch, args, alt, model, cfg, Hc, Hv, D, golden, sizes)
        dce, dve = D[0].cpu().numpy(), D[1].cpu().numpy()
        out[alt + "_gpu"] = {k: ext[k] for k in ("value", "ms_per_step", "dtype", "roofline",
                                                  "accuracy")}
        out[alt + "_gpu"]["speedup_vs_fp64_gpu"] = ext["value"] / out["fp64_gpu"]["value"]
    ref_cols = None
    if golden and not args.no_cpu_baseline:
        out["cpu_baseline"], ref_cols = cpu_baseline(model, args.workload, golden,
                                                     args.cpu_sample)
    # accuracy (outside the timed region): every entry of the sampled subgraphs' core columns
    # against the oracle; the whole D against the FP64 GPU path of the same run; |D^2 - D| on
    # the core columns of 16 of the sampled subgraphs
    acc = out["accuracy"]
    n_sites = N // 2
    if golden:
        acc["D_pattern_bit_exact"] = ell_sha256(dcm) == golden["D_col_sha256"]
    if ref_cols is not None:
        e = d_errors(dcm, dvm, ref_cols)
        acc["vs_oracle_subgraphs"] = e
        idem_cols = [v for v, _ in ref_cols[:16]]
        acc["idempotency_D"] = idempotency(dcm, dvm, idem_cols)
        if dcf is not None:
            out["fp64_gpu"]["accuracy"]["vs_oracle_subgraphs"] = d_errors(dcf, dvf, ref_cols)
            out["fp64_gpu"]["accuracy"]["idempotency_D"] = idempotency(dcf, dvf, idem_cols)
    if ext is not None:
        ea = out[alt + "_gpu"]["accuracy"]
        if ref_cols is not None:
            ea["vs_oracle_subgraphs"] = d_errors(dce, dve, ref_cols)
        d = dve - dvf
        ea["vs_fp64_gpu_whole_D"] = {"pattern_equal": bool(np.array_equal(dce, dcf)),
                                     "max_abs": float(np.abs(d).max()),
                                     "frobenius": float(np.linalg.norm(d))}
        del dce, dve
    if dcf is not None:
        same = bool(np.array_equal(dcm, dcf))
        d = dvm - dvf
        acc["vs_fp64_gpu_whole_D"] = {
            "pattern_equal": same, "max_abs": float(np.abs(d).max()),
            "frobenius": float(np.linalg.norm(d)),
            "frobenius_per_site": float(np.linalg.norm(d)) / n_sites,
            "entries": int((dcm >= 0).sum())}
    worst = [acc.get("vs_oracle_subgraphs", {}).get("max_abs")]
    if "vs_fp64_gpu_whole_D" in acc and "fp64_gpu" in out:
        fe = out["fp64_gpu"]["accuracy"].get("vs_oracle_subgraphs", {}).get("max_abs", 0.0)
        worst.append(acc["vs_fp64_gpu_whole_D"]["max_abs"] + fe)
    known = [w for w in worst if w is not None]
    acc["meets_1e-6"] = (max(known) <= 1e-6) if known else None
    print(json.dumps(_finite(out)), flush=True)


def _finite(x):
    """JSON has no NaN / Inf: such values (an unmeasured quantity) become null."""
    if isinstance(x, dict):
        return {k: _finite(v) for k, v in x.items()}
    if isinstance(x, list):
        return [_finite(v) for v in x]
    if isinstance(x, float) and not np.isfinite(x):
        return None
    return x


def stage_hbm(ms, sizes, core_sizes, model, precision):
    """Algorithmic HBM rates of the gather and the scatter (GB/s, from the stage times): the
    gather reads H's ELL (4 + 8 bytes per slot) and writes every padded block (4 bytes per
    element for the low-precision loops, 8 for FP64); the scatter reads the core columns (8
    bytes per entry) and writes D's column-ELL (4 + 8 bytes per entry)."""
    npad = (np.asarray(sizes, dtype=np.int64) + 63) // 64 * 64
    elem = 8 if precision == "fp64" else 4
    h_bytes = model["H_col"].size * 12
    gather = float((npad * npad).sum() * elem + h_bytes)
    scatter = float((np.asarray(core_sizes, dtype=np.int64) * sizes).sum() * (8 + 12))
    out = {"gather_bytes": gather, "scatter_bytes": scatter}
    if ms.get("gather", 0) > 0:
        out["gather"] = gather / (ms["gather"] * 1e-3) / 1e9
    if ms.get("scatter", 0) > 0:
        out["scatter"] = scatter / (ms["scatter"] * 1e-3) / 1e9
    return out


def measure(gb, torch, args, precision, model, cfg, Hc, Hv, D, golden, sizes):
    """Warm-up, then K timed steps of the whole path in ``precision``; one result record."""
    N, n_occ = model["N"], model["n_occ"]
    a = argparse.Namespace(**vars(args))
    a.precision = precision
    for _ in range(args.warmup):
        run_step(gb, Hc, Hv, n_occ, cfg["tau"], cfg["core"], D, a)
    torch.cuda.synchronize()
    low = precision != "fp64"
    key = "square_lo" if low else "square"
    sq_ms, sq_n, stats = 0.0, 0, None
    host_ms = {"graph": 0.0, "part": 0.0}
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, _, stats = run_step(gb, Hc, Hv, n_occ, cfg["tau"], cfg["core"], D, a, host_ms)
        sq_ms += stats["ms"][key]
        sq_n += stats["n_" + key]
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    # graph and partition are separate calls before gb_density: their wall time per step
    stats["ms"]["graph"] = host_ms["graph"] / args.steps
    stats["ms"]["part"] = host_ms["part"] / args.steps
    planes = PLANE_PRODUCTS.get(precision, 1)
    # algorithmic work of one squaring launch: the symmetric square (upper triangle) of every
    # block, times the plane products of the split method; executed: what the matrix cores
    # run (blocks padded to 64, whole diagonal tiles); dense-equivalent: sum 2 n^3
    flops_alg = sym_square_flops(sizes, planes)
    flops_exec = stats["square_flops_exec"] * planes
    flops_dense = stats["square_flops"]
    peak = PEAK_TFLOPS[precision]
    # per-launch HIP events around every square (host and device-driven loops; the hipGraph
    # replay has none)
    avg_launch_s = (sq_ms / sq_n / 1e3) if (sq_n and sq_ms > 0) else None
    achieved = flops_alg / avg_launch_s / 1e12 if avg_launch_s else None
    # the matrix-core rate this device sustains on register operands in the kernel's input
    # type (the library's own MFMA chains): what the executed rate is read against
    mfma_kind = {"fp64": "fp64", "fp32": "fp32", "fp16x3": "fp16"}.get(precision, "bf16")
    sustained, clock_mhz = gb.peak_rate(mfma_kind, with_clock=True)
    exec_rate = flops_exec / avg_launch_s / 1e12 if avg_launch_s else None
    return {
        "metric": METRIC, "value": N / dt, "unit": "orbitals/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32+f64", "fp16x3": "f16+f64"}.get(precision,
                                                                               "bf16+f64"),
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: seeded 3D tight-binding model, N={N} orbitals, "
                               f"n_occ={n_occ}, tau={cfg['tau']}, cores of {cfg['core']}"
                               + ("" if args.partition == "block" else
                                  f" (at most; {args.partition} communities)"),
                   "partition": args.partition,
                   "precision": precision, "launch_mode": args.launch_mode,
                   "tile_policy": args.tile_policy, "tile_order": args.tile_order,
                   "refine": args.refine, "n_fp64_first": args.n_fp64_first,
                   "n_tile64": stats["n_tile64"], "n_split_il": stats["n_split_il"],
                   "n_sub": stats["n_sub"],
                   "max_sub": stats["max_sub"], "sp2_iters": stats["iters"],
                   "refine_steps": stats["n_refine_done"]},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak if achieved else None,
                     "traffic": measured_traffic(args.workload, square_kernel_name(precision, stats),
                                                 args.partition),
                     "kernel": square_kernel_name(precision, stats),
                     "flops_per_launch_alg": flops_alg, "flops_per_launch_exec": flops_exec,
                     "flops_per_launch_dense_2n3": flops_dense,
                     "exec_frac": exec_rate / peak if exec_rate else None,
                     "sustained_mfma_peak": sustained, "sustained_mfma_kind": mfma_kind,
                     "sustained_mfma_clock_mhz": clock_mhz,
                     "exec_frac_of_sustained": exec_rate / sustained if exec_rate else None,
                     "avg_launch_ms": avg_launch_s * 1e3 if avg_launch_s else None,
                     "launches": sq_n},
        "accuracy": {"converged": stats["converged"], "trace_D": stats["trace"],
                     "branch": "".join(map(str, stats["branch"])),
                     "branch_matches_oracle": (golden is not None and
                                               "".join(map(str, stats["branch"])) == golden["branch"]),
                     "n_near_tie": stats["n_near_tie"]},
        "stage_ms": stats["ms"],
    }


if __name__ == "__main__":
    main()
