"""Benchmark of the MBE(3)-OSV-MP2 per-cluster hot path on one MI355X.

One step = the whole path on one batch of synthetic input already resident in
HBM: cluster selection and plan, S/F and K orbital-pair blocks, pair-domain
preparation, couplings, the residual solve of every 1b/2b/3b cluster, the MBE
energy and the densities dE/dC, dE/dF_occ, dE/deps_vir.

metric: pair-blocks/s (one pair-block = one unordered LMO pair of one cluster),
for the mixed-precision path; the plain FP64 GPU path is timed beside it and the
speedup and energy difference are reported.

usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload 4]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"fp64_mfma_tflops": 78.6, "fp64_vector_tflops": 78.6, "hbm_gbs": 8000.0}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", type=int, default=None,
                    help="synthetic workload (default 4; 3 with --osvgen, the largest that carries B)")
    ap.add_argument("--precision", choices=["mixed", "fp64", "both"], default="both")
    ap.add_argument("--cpu-sample", type=int, default=6000,
                    help="clusters of the workload timed on the CPU oracle (0 = skip)")
    ap.add_argument("--tau-R", type=float, default=1e-10)
    ap.add_argument("--weak-l2b", type=float, default=None,
                    help="instead of the step: build the workload with the overlap selection "
                         "at this l_2b and time the weak-pair (one-block) energies")
    ap.add_argument("--weak-l3b", type=float, default=0.2)
    ap.add_argument("--response", action="store_true",
                    help="instead of the step: after one solve of the workload, time the OSV "
                         "response intermediates N_ij (eq:nij, MBE-combined) of every ordered pair")
    ap.add_argument("--correction", action="store_true",
                    help="instead of the step: after one solve of the workload, time the one-step "
                         "high-order correction")
    ap.add_argument("--osvgen", action="store_true",
                    help="instead of the step: time the OSV generation from the fitted integrals B")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="before the steps, copy a buffer of this many MiB once (device to "
                         "device) so that a counter run can calibrate its byte counters")
    return ap.parse_args()


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_k_solve_mbe3-lattice-nocc400.md")
SOLVE_SOURCES = ["paper_2106_06149_amd/csrc/k_solve.hip", "paper_2106_06149_amd/csrc/osv_internal.h"]
TRAFFIC_NIJ_FILE = os.path.join(ROOT, "profiles", "traffic_k_nij_mbe3-lattice-nocc400.md")
NIJ_SOURCES = ["paper_2106_06149_amd/csrc/k_nij.hip", "paper_2106_06149_amd/csrc/tiles.h",
               "paper_2106_06149_amd/csrc/osv_internal.h"]


def source_hash(files):
    import hashlib
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def solve_source_hash():
    return source_hash(SOLVE_SOURCES)


def nij_source_hash():
    return source_hash(NIJ_SOURCES)


def measured_traffic(workload, path=TRAFFIC_FILE, hash_fn=None):
    """HBM bytes of one stage (the solve's k_solve launches, or the k_nij launch)
    from the committed counter summary, or None when there is none for this
    workload or the kernel has changed since the counters were taken (the summary
    records a hash of its sources)."""
    try:
        with open(path) as fh:
            lines = fh.read().splitlines()
    except OSError:
        return None
    kv = {}
    for ln in lines:
        if ln.startswith("- ") and ":" in ln:
            k, v = ln[2:].split(":", 1)
            kv[k.strip()] = v.strip().strip("`")
    want = (hash_fn or solve_source_hash)()
    if kv.get("source_hash") != want or kv.get("workload") != str(workload):
        return None
    try:
        return float(kv["traffic_bytes_per_stage"])
    except (KeyError, ValueError):
        return None


_CPU_SYS = None


def _cpu_clusters(chunk):
    """Worker of the CPU baseline: each cluster's own pair blocks, solve, energy and
    densities with the oracle (one BLAS thread per worker)."""
    from oracle import osv_oracle as O
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except Exception:
        pass
    npb = 0
    pb = O.PairBlocks(_CPU_SYS)
    for X in chunk:
        cl = O.Cluster(pb, X)
        cl.solve(1e-10, 100)
        cl.energy()
        cl.densities()
        npb += len(X) * (len(X) + 1) // 2
        pb._S.clear(); pb._F.clear(); pb._K.clear()   # no reuse of pair blocks across clusters
    return npb


def _cpu_response(chunk):
    """Worker of the response CPU baseline: per cluster the oracle's solve (not
    timed), then its N_ij contributions (timed).  Returns (contributions, seconds)."""
    from oracle import osv_oracle as O
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except Exception:
        pass
    units, secs = 0, 0.0
    pb = O.PairBlocks(_CPU_SYS)
    for X in chunk:
        T = O.Cluster(pb, X).solve(1e-10, 100)
        t0 = time.perf_counter()
        O.osv_response(_CPU_SYS, dict(clusters=[X], coef=[1.0], T=[T]))
        secs += time.perf_counter() - t0
        units += len(X) * len(X)
        pb._S.clear(); pb._F.clear(); pb._K.clear()
    return units, secs


def cpu_response_baseline(s, n_sample, seed=7, workers=None):
    """The FP64 CPU oracle's N_ij (osv_response) on a seeded sample of the
    workload's clusters with nonzero c_X, over forked workers (one BLAS thread
    each); only the N_ij evaluation is timed.  Returns contributions/s (one
    contribution = one ordered pair of one cluster) on the host cores."""
    import multiprocessing as mp
    import numpy as np
    from oracle import osv_oracle as O
    global _CPU_SYS
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    nw = max(1, min(16, avail)) if workers is None else workers
    clusters, coef, _ = O.select_clusters(s.centroid, s.sel_mode, s.cut2, s.cut3)
    live = [X for X, c in zip(clusters, coef) if c != 0.0]
    rng = np.random.default_rng(seed)
    idx = rng.choice(len(live), size=min(n_sample, len(live)), replace=False)
    sample = [live[n] for n in idx]
    chunks = [sample[w::nw] for w in range(nw)]
    _CPU_SYS = s
    if nw == 1:
        res = [_cpu_response(sample)]
    else:
        with mp.get_context("fork").Pool(nw) as pool:
            res = pool.map(_cpu_response, chunks, chunksize=1)
    _CPU_SYS = None
    units = sum(u for u, _ in res)
    rate = sum(u / t for u, t in res if t > 0)
    tsum = sum(t for _, t in res)
    return {"value": rate, "unit": "contributions/s", "cores": nw, "kind": "oracle",
            "sample": f"{len(idx)} seeded clusters with nonzero c_X ({units} ordered-pair "
                      f"contributions) of the same workload, the oracle's N_ij of each cluster "
                      f"(its solve not timed), over {nw} worker processes with one BLAS thread "
                      f"each; {tsum:.1f} s of N_ij work in all",
            "cpu_model": cpu_model(), "cpu_count": os.cpu_count()}


def cpu_osvgen_baseline(s):
    """The FP64 CPU oracle's OSV generation (generate_osvs) on the whole workload,
    timed once in this process (before the GPU is touched), with the BLAS threads it
    has.  Returns LMOs/s."""
    from oracle import osv_oracle as O
    threads = None
    try:
        from threadpoolctl import threadpool_info
        threads = max((d.get("num_threads") or 0) for d in threadpool_info()) or None
    except Exception:
        pass
    t0 = time.perf_counter()
    O.generate_osvs(s.B, s.eps_vir, s.F_occ, 1e-4, 50)
    dt = time.perf_counter() - t0
    return {"value": s.nocc / dt, "unit": "LMOs/s", "cores": threads or 1, "kind": "oracle",
            "sample": f"the whole workload ({s.nocc} LMOs), one call, {dt:.1f} s",
            "cpu_model": cpu_model(), "cpu_count": os.cpu_count()}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(s, n_sample, seed=7, workers=None):
    """The FP64 CPU oracle, as it stands, on a seeded sample of the workload's
    clusters (each cluster's full path: its pair blocks, solve, energy and
    densities), spread over forked worker processes (one per host core available
    to this process, at most 16), each with one BLAS thread.  Must run before the
    process touches the GPU.  Returns pair-blocks/s on the host cores."""
    import multiprocessing as mp
    import numpy as np
    from oracle import osv_oracle as O
    global _CPU_SYS
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    nw = max(1, min(16, avail)) if workers is None else workers
    clusters, coef, order = O.select_clusters(s.centroid, s.sel_mode, s.cut2, s.cut3)
    rng = np.random.default_rng(seed)
    # sample in proportion to the workload's mix of 1b/2b/3b clusters
    idx = rng.choice(len(clusters), size=min(n_sample, len(clusters)), replace=False)
    sample = [clusters[n] for n in idx]
    chunks = [sample[w::nw] for w in range(nw)]
    _CPU_SYS = s
    t0 = time.perf_counter()
    if nw == 1:
        npb = _cpu_clusters(sample)
    else:
        with mp.get_context("fork").Pool(nw) as pool:
            npb = sum(pool.map(_cpu_clusters, chunks, chunksize=1))
    dt = time.perf_counter() - t0
    _CPU_SYS = None
    return {"value": npb / dt, "unit": "pair-blocks/s", "cores": nw, "kind": "oracle",
            "sample": f"{len(idx)} seeded clusters ({npb} pair-blocks) of the same workload, "
                      f"each with its own pair blocks, solve, energy and densities, over {nw} "
                      f"worker processes with one BLAS thread each; {dt:.1f} s",
            "cpu_model": cpu_model(), "cpu_count": os.cpu_count()}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              f"(asked for --gpus {args.gpus}).", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    from paper_2106_06149_amd import synth

    if args.workload is None:
        args.workload = 3 if args.osvgen else 4
    s = synth.workload(args.workload)
    spec = synth.WORKLOADS[args.workload]
    # the host baseline forks its workers before this process initialises the GPU
    cpu_rec = None
    if args.osvgen:
        if getattr(s, "B", None) is None:
            print(f"bench.py --osvgen: workload {args.workload} carries no B", file=sys.stderr)
            sys.exit(2)
        if args.cpu_sample > 0:
            cpu_rec = cpu_osvgen_baseline(s)
            print(f"[bench] cpu baseline (OSV generation): {cpu_rec['value']:.2f} LMOs/s on "
                  f"{cpu_rec['cores']} BLAS threads", file=sys.stderr, flush=True)
    elif args.response:
        if args.cpu_sample > 0:
            cpu_rec = cpu_response_baseline(s, min(args.cpu_sample, 240))
            print(f"[bench] cpu baseline (N_ij): {cpu_rec['value']:.1f} contributions/s on "
                  f"{cpu_rec['cores']} workers", file=sys.stderr, flush=True)
    elif args.cpu_sample > 0 and args.weak_l2b is None and not args.correction:
        cpu_rec = cpu_baseline(s, args.cpu_sample)
        print(f"[bench] cpu baseline: {cpu_rec['value']:.1f} pair-blocks/s on {cpu_rec['cores']} "
              f"workers ({cpu_rec['cpu_model']})", file=sys.stderr, flush=True)
    import torch
    from paper_2106_06149_amd.api import OSVContext, Selection, get_tuning

    dev = torch.device("cuda:0")
    Qt = torch.from_numpy(np.ascontiguousarray(s.Q.T)).to(dev)
    C = torch.from_numpy(s.C).to(dev)
    eps = torch.from_numpy(s.eps_vir).to(dev)
    F = torch.from_numpy(s.F_occ).to(dev)
    sel = Selection(s.sel_mode, s.cut2, s.cut3)
    torch.cuda.synchronize()
    if args.copy_probe_mib > 0:
        n = args.copy_probe_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)                 # reads and writes n * 8 bytes
        torch.cuda.synchronize()
        print(f"[bench] copy probe: {n * 8} bytes read, {n * 8} bytes written", file=sys.stderr)
        del src, dst

    if args.weak_l2b is not None:
        # weak 2b clusters (one-block scheme): the build with the overlap selection
        # is not timed; the timed call forms every weak pair's energy from the K
        # blocks, W slots and eigenvalues the build left on the device
        from paper_2106_06149_amd import _lib as L
        wsel = Selection(L.OSV_SEL_OVERLAP, l2b=args.weak_l2b, l3b=args.weak_l3b)
        oc = OSVContext(Qt, C, eps, F, s.r, s.centroid, wsel, 1)
        for _ in range(max(1, args.warmup)):
            Ew, pairs, _ = oc.weak_pairs()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            Ew, pairs, _ = oc.weak_pairs()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        n2b = oc.counts["n2b"]
        oc.close()
        print(json.dumps({"metric": "weak 2b pairs/s (one-block energies)", "value": len(pairs) / dt,
                          "unit": "pairs/s", "n_gpus": 1, "steps": args.steps,
                          "ms_per_call": dt * 1e3, "higher_is_better": True, "dtype": "f64",
                          "data": "synthetic",
                          "config": {"workload": spec["name"], "l2b": args.weak_l2b,
                                     "l3b": args.weak_l3b, "n_weak": int(len(pairs)),
                                     "n_strong_2b": int(n2b), "precision": "mixed"},
                          "E_weak": Ew}))
        return

    if args.osvgen:
        from paper_2106_06149_amd.api import generate_osvs, generation_stats
        B = torch.from_numpy(np.ascontiguousarray(s.B)).to(dev)
        for _ in range(max(1, args.warmup)):
            generate_osvs(B, eps, F, 1e-4, 50)
        torch.cuda.synchronize()
        st = []
        t0 = time.perf_counter()
        for _ in range(args.steps):
            r, _, _, _ = generate_osvs(B, eps, F, 1e-4, 50)
            st.append(generation_stats())
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        ms = {k: float(np.mean([x[k][0] for x in st])) for k in st[0]}
        fl = {k: st[0][k][1] for k in st[0]}
        rec = {"metric": "LMOs/s (OSV generation from B, eq:svd)", "value": s.nocc / dt, "unit": "LMOs/s",
               "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_call": dt * 1e3,
               "higher_is_better": True, "dtype": "f64", "data": "synthetic",
               "config": {"workload": spec["name"], "nocc": s.nocc, "nvir": s.nvir, "naux": s.naux,
                          "l_osv": 1e-4, "r_max": 50, "osvs_kept": int(r.sum())},
               "stages_ms": {k: round(v, 3) for k, v in ms.items()},
               "stage_tflops": {k: round(fl[k] / (ms[k] * 1e-3) / 1e12, 3) for k in ms if ms[k] > 0},
               # the dominant kernel: the per-LMO Householder reduction (FP64 vector ALU)
               "roofline": {"kernel": "k_osv_tridiag", "bound": "alu",
                            "achieved": fl["tridiag"] / (ms["tridiag"] * 1e-3) / 1e12,
                            "peak": PEAK["fp64_vector_tflops"], "unit": "TFLOP/s",
                            "frac": fl["tridiag"] / (ms["tridiag"] * 1e-3) / 1e12 / PEAK["fp64_vector_tflops"],
                            "traffic": None}}
        if cpu_rec is not None:
            rec["cpu_baseline"] = cpu_rec
        print(json.dumps(rec), flush=True)
        return

    if args.correction:
        # the one-step correction after one converged solve (not timed)
        prec = 0 if args.precision == "fp64" else 1
        oc = OSVContext(Qt, C, eps, F, s.r, s.centroid, sel, prec)
        oc.solve(tau_R=args.tau_R)
        for _ in range(max(1, args.warmup)):
            oc.high_order_correction()
        torch.cuda.synchronize()
        st = []
        t0 = time.perf_counter()
        for _ in range(args.steps):
            dE, Ec, mx, _ = oc.high_order_correction()
            st.append(oc.correction_stats())
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        nd = oc.counts["n_domains"]
        oc.close()
        cms = float(np.mean([x["collective"][0] for x in st]))
        sms = float(np.mean([x["step"][0] for x in st]))
        cby, sfl = st[0]["collective"][1], st[0]["step"][1]
        rec = {"metric": "pair domains/s (one-step high-order correction)", "value": nd / dt,
               "unit": "domains/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
               "ms_per_call": dt * 1e3, "higher_is_better": True, "dtype": "f64", "data": "synthetic",
               "config": {"workload": spec["name"], "nocc": s.nocc, "pair_domains": int(nd),
                          "precision": "mixed" if prec == 1 else "fp64", "tau_R": args.tau_R},
               "stages_ms": {"collective": round(cms, 3), "step": round(sms, 3)},
               "roofline": {"kernel": "k_collective_step", "bound": "mfma",
                            "achieved": sfl / (sms * 1e-3) / 1e12, "peak": PEAK["fp64_mfma_tflops"],
                            "unit": "TFLOP/s", "frac": sfl / (sms * 1e-3) / 1e12 / PEAK["fp64_mfma_tflops"],
                            "flops": sfl, "traffic": None},
               "roofline_collective": {"kernel": "k_collective", "bound": "hbm",
                                       "achieved": cby / (cms * 1e-3) / 1e9, "peak": PEAK["hbm_gbs"],
                                       "unit": "GB/s", "frac": cby / (cms * 1e-3) / 1e9 / PEAK["hbm_gbs"],
                                       "bytes": cby, "traffic": None},
               "dE": dE, "E_coll": Ec, "max_dR": mx}
        print(json.dumps(rec), flush=True)
        return

    if args.response:
        # N_ij after one converged solve (not timed); the timed calls evaluate every
        # ordered pair's MBE-combined N_ij from the amplitudes left on the device
        from paper_2106_06149_amd.api import plan_clusters
        prec = 0 if args.precision == "fp64" else 1
        oc = OSVContext(Qt, C, eps, F, s.r, s.centroid, sel, prec)
        oc.solve(tau_R=args.tau_R)
        out = None
        for _ in range(max(1, args.warmup)):
            out, pairs, offs, _ = oc.response(out)
        torch.cuda.synchronize()
        ms = []
        t0 = time.perf_counter()
        for _ in range(args.steps):
            out, pairs, offs, (ms_k, fl) = oc.response(out)
            ms.append(ms_k)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        oc.close()
        _, lmos, coef = plan_clusters(s.centroid, sel)
        size = (lmos >= 0).sum(axis=1)
        units = int(np.sum((size ** 2)[coef != 0.0]))
        kms = float(np.mean(ms))
        achieved = fl / (kms * 1e-3) / 1e12
        rec = {"metric": "N_ij cluster ordered-pair contributions/s (eq:nij, MBE-combined)",
               "value": units / dt, "unit": "contributions/s", "n_gpus": 1, "steps": args.steps,
               "warmup": args.warmup, "ms_per_call": dt * 1e3, "higher_is_better": True,
               "dtype": "f64", "data": "synthetic",
               "config": {"workload": spec["name"], "nocc": s.nocc, "ordered_pairs": int(len(pairs)),
                          "contributions": units, "output_doubles": int(out.numel()),
                          "precision": "mixed" if prec == 1 else "fp64", "tau_R": args.tau_R},
               "roofline": {"kernel": "k_nij", "bound": "mfma", "achieved": achieved,
                            "peak": PEAK["fp64_mfma_tflops"], "unit": "TFLOP/s",
                            "frac": achieved / PEAK["fp64_mfma_tflops"], "kernel_ms": kms,
                            "flops": fl,
                            "traffic": measured_traffic(args.workload, TRAFFIC_NIJ_FILE, nij_source_hash)}}
        if cpu_rec is not None:
            rec["cpu_baseline"] = cpu_rec
        print(json.dumps(rec), flush=True)
        return

    def step(prec):
        oc = OSVContext(Qt, C, eps, F, s.r, s.centroid, sel, prec)
        info = oc.solve(tau_R=args.tau_R)
        E, orders, _ = oc.energy()
        oc.densities(dC=True, dF=True, deps=True)
        counts = dict(oc.counts, sweeps=info["sweeps"])
        out = (E, orders, oc.stage_times(), oc.stage_flops(), counts)
        oc.close()
        return out

    precs = {"mixed": [1], "fp64": [0], "both": [1, 0]}[args.precision]
    res = {}
    for prec in precs:
        for _ in range(args.warmup):
            step(prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        stages = []
        for _ in range(args.steps):
            E, orders, st, fl, counts = step(prec)
            stages.append(st)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        print(f"[bench] precision={'mixed' if prec else 'fp64'} ms/step={dt*1e3:.1f} E={E:.10f} "
              f"stages={ {k: round(v, 1) for k, v in st.items()} }", file=sys.stderr, flush=True)
        res[prec] = dict(dt=dt, E=E, orders=orders, stages=stages, flops=fl, counts=counts)

    main_prec = precs[0]
    r = res[main_prec]
    npb = r["counts"]["n_pair_blocks"]
    value = npb / r["dt"]
    # dominant kernel: the persistent residual solve (FP64 MFMA)
    solve_ms = float(np.mean([st["solve"] for st in r["stages"]]))
    solve_flops = r["flops"]["solve"]
    achieved = solve_flops / (solve_ms * 1e-3) / 1e12
    out = {
        "metric": "pair-blocks/s for MBE(3) residual+densities",
        "value": value,
        "unit": "pair-blocks/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["dt"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+int8-digit-K" if main_prec == 1 else "f64",
        "data": "synthetic",
        "config": {"workload": spec["name"], "nocc": s.nocc, "nvir": s.nvir, "naux": s.naux,
                   "r_range": list(spec["r"]) if isinstance(spec["r"], tuple) else spec["r"],
                   "cut2": s.cut2, "cut3": s.cut3, "clusters": r["counts"]["n_clusters"],
                   "pair_blocks": npb, "precision": "mixed" if main_prec == 1 else "fp64"},
        "roofline": {"kernel": "k_solve", "bound": "mfma", "achieved": achieved,
                     "peak": PEAK["fp64_mfma_tflops"], "unit": "TFLOP/s",
                     "frac": achieved / PEAK["fp64_mfma_tflops"],
                     "traffic": measured_traffic(args.workload)},
        "stages_ms": {k: round(float(np.mean([st[k] for st in r["stages"]])), 2) for k in r["stages"][0]},
        # algorithmic TFLOP/s per stage (kept ranks, selected blocks only) over its device time
        "stage_tflops": {k: round(r["flops"][k] / (1e-3 * float(np.mean([st[k] for st in r["stages"]]))) / 1e12, 2)
                         for k in r["flops"] if r["flops"][k] > 0 and k != "host_plan"},
        # launch variants in use (the autotuner's table, include/osv.h)
        "tuning": get_tuning(),
        "E": r["E"],
        # the path without the build stages (S/F, K, domain preparation, couplings)
        "pair_blocks_per_s_solve_energy_densities": npb / (1e-3 * sum(
            float(np.mean([st[k] for st in r["stages"]]))
            for k in ("solve", "energy", "adjoint", "backtransform"))),
        # sweeps = the largest number any cluster took (every cluster runs to its own bar)
        "pair_block_sweeps_per_s": npb * r["counts"]["sweeps"] / (solve_ms * 1e-3),
    }
    if 0 in res and 1 in res:
        out["fp64_value"] = npb / res[0]["dt"]
        out["speedup_vs_fp64"] = res[0]["dt"] / res[1]["dt"]
        out["mixed_minus_fp64_Eh"] = res[1]["E"] - res[0]["E"]
    if cpu_rec is not None:
        out["cpu_baseline"] = cpu_rec
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
