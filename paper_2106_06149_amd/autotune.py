"""Autotuner of the library's launch variants (the tuning table of include/osv.h).

On one GPU it times the whole path (build, solve, energy, densities) on a
synthetic workload for every allowed value of each tuning key, one key at a time
with the others at their best values so far (coordinate descent, two passes), and
keeps the value whose stage time (the stages that key affects) is smallest.  Every
variant must give the same energy as the default shapes (to 1e-10 relative), or it
is not chosen.  The result goes to a "key value" file that the library reads when
a process first builds a context (osv_tuning.txt beside the library by default),
with the measured times as comments.

usage: python -m paper_2106_06149_amd.autotune [--workload 4] [--steps 2] [--out PATH]
"""
import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_OUT = os.path.join(HERE, "osv_tuning.txt")

# the stages (osv_stage_times names) whose device time each key changes
STAGES = {
    "gemm_ks": ("sf", "k", "backtransform"),   # FP64 products (mixed mode: digit products)
    "prep_nt_small": ("prep",),
    "prep_nt_mid": ("prep",),
    "prep_nt_big": ("prep",),
    "cpl_split": ("couplings",),
    "solve_split": ("solve",),
}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", type=int, default=4)
    ap.add_argument("--precision", type=int, default=None, help="0 FP64, 1 mixed (default: the workload's)")
    ap.add_argument("--steps", type=int, default=2, help="timed steps per variant (median)")
    ap.add_argument("--passes", type=int, default=2)
    ap.add_argument("--out", default=DEFAULT_OUT)
    args = ap.parse_args(argv)

    import numpy as np
    import torch
    from . import _lib as L, synth
    from .api import OSVContext, Selection, get_tuning, set_tuning

    os.environ.setdefault("OSV_TUNING_FILE", "")   # start from the compiled-in defaults
    dev = torch.device("cuda:0")
    s = synth.workload(args.workload)
    prec = s.precision if args.precision is None else args.precision
    Qt = torch.from_numpy(np.ascontiguousarray(s.Q.T)).to(dev)
    C = torch.from_numpy(s.C).to(dev)
    eps = torch.from_numpy(s.eps_vir).to(dev)
    F = torch.from_numpy(s.F_occ).to(dev)
    sel = Selection(s.sel_mode, s.cut2, s.cut3)

    def step():
        oc = OSVContext(Qt, C, eps, F, s.r, s.centroid, sel, prec)
        oc.solve(tau_R=1e-10)
        E, _, _ = oc.energy()
        oc.densities()
        st = oc.stage_times()
        oc.close()
        return E, st

    def measure():
        step()                                          # warm-up (block cache, code objects)
        Es, sts = [], []
        for _ in range(args.steps):
            E, st = step()
            Es.append(E)
            sts.append(st)
        med = {k: float(np.median([st[k] for st in sts])) for k in sts[0]}
        return Es[-1], med

    best = get_tuning()
    E_ref, st_ref = measure()
    print(f"[autotune] workload {s.name}, precision {prec}, defaults {best}: E = {E_ref:.12f}",
          file=sys.stderr, flush=True)
    log = []
    for ps in range(args.passes):
        for key, vals in L.TUNING_KEYS.items():
            times = {}
            for v in vals:
                set_tuning(**dict(best, **{key: v}))
                E, st = measure()
                t = sum(st[k] for k in STAGES[key])
                ok = abs(E - E_ref) <= 1e-10 * abs(E_ref)
                times[v] = (t, ok)
                log.append((ps, key, v, t, ok))
                print(f"[autotune] pass {ps} {key}={v}: {'+'.join(STAGES[key])} {t:.2f} ms"
                      f"{'' if ok else ' (energy differs: not chosen)'}", file=sys.stderr, flush=True)
            good = {v: t for v, (t, ok) in times.items() if ok}
            best[key] = min(good, key=good.get) if good else best[key]
            set_tuning(**best)
    name = torch.cuda.get_device_name(0)
    with open(args.out, "w") as fh:
        fh.write(f"# launch tuning of libosvmbe, written by paper_2106_06149_amd.autotune\n")
        fh.write(f"# device: {name}; workload {s.name} (precision {prec}), "
                 f"{args.steps} timed steps per variant, {args.passes} passes\n")
        fh.write("# measured (pass, key, value, ms of the stages the key affects, energy ok):\n")
        for ps, key, v, t, ok in log:
            fh.write(f"#   {ps} {key} {v} {t:.2f} {int(ok)}\n")
        for k, v in best.items():
            fh.write(f"{k} {v}\n")
    print(json.dumps({"tuning": best, "out": args.out}), flush=True)


if __name__ == "__main__":
    main()
