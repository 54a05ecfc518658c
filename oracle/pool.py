"""Cluster-parallel driver of the FP64 oracle.

TEST INFRASTRUCTURE ONLY (like osv_oracle): tests and the CPU-baseline leg of the
benchmark use it to run the oracle's independent cluster problems in worker
processes.  It adds no arithmetic of its own beyond summing the per-cluster
results with their MBE coefficients (eq:mbe1, eq:mbe2), in a fixed order: the
clusters are cut into contiguous chunks, each chunk is summed in cluster order,
and the chunk sums are added in chunk order.
"""
from __future__ import annotations

import multiprocessing as mp
import os

import numpy as np

from . import osv_oracle as O

_SYS = None


def _init(sysm):
    global _SYS
    _SYS = sysm
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)     # one BLAS thread per worker process
    except Exception:
        pass


def _run_chunk(args):
    """Solve a contiguous chunk of clusters; return their energies and the
    coefficient-weighted density sums of the chunk."""
    clusters, coef, tau_R, tau_S, max_sweeps, densities, dvir, k_exact = args
    s = _SYS
    pb = O.PairBlocks(s, k_exact=k_exact)
    off = s.off
    E = np.zeros(len(clusters))
    sweeps = np.zeros(len(clusters), dtype=np.int64)
    maxres = 0.0
    conv = True
    dC = np.zeros((s.nosv, s.naux)) if densities else None
    dF = np.zeros((s.nocc, s.nocc)) if densities else None
    de = np.zeros(s.nvir) if densities else None
    Dv = np.zeros((s.nvir, s.nvir)) if (densities and dvir) else None
    for n, X in enumerate(clusters):
        cl = O.Cluster(pb, X, tau_S)
        cl.solve(tau_R, max_sweeps)
        E[n] = cl.energy()
        sweeps[n] = cl.sweeps
        maxres = max(maxres, cl.max_residual)
        conv = conv and cl.converged
        if densities and coef[n] != 0.0:
            d = cl.densities(dvir=dvir)
            if not k_exact:
                for p, g in d[0].items():
                    dC[off[p]:off[p + 1]] += coef[n] * g
            dF += coef[n] * d[1]
            de += coef[n] * d[2]
            if dvir:
                Dv += coef[n] * d[3]
    return E, sweeps, maxres, conv, dC, dF, de, Dv


def default_workers() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def solve(sysm, nproc: int = None, tau_R: float = 1e-10, tau_S: float = 1e-8,
          max_sweeps: int = 100, densities: bool = True, dvir: bool = False,
          clusters=None, coef=None, order=None, chunks_per_worker: int = 4, k_exact: bool = False):
    """Same result as osv_oracle.solve for the workload's selection (or the given
    cluster list), with the clusters spread over nproc worker processes (spawned,
    each holding one copy of the system)."""
    nproc = nproc or default_workers()
    if clusters is None:
        clusters, coef, order = O.select_clusters(sysm.centroid, sysm.sel_mode, sysm.cut2, sysm.cut3)
    n = len(clusters)
    nch = max(1, min(n, nproc * chunks_per_worker))
    bounds = np.linspace(0, n, nch + 1).astype(int)
    tasks = [(clusters[bounds[c]:bounds[c + 1]], coef[bounds[c]:bounds[c + 1]], tau_R, tau_S,
              max_sweeps, densities, dvir, k_exact) for c in range(nch)]
    ctx = mp.get_context("spawn")
    with ctx.Pool(nproc, initializer=_init, initargs=(sysm,)) as pool:
        parts = pool.map(_run_chunk, tasks, chunksize=1)
    E_cl = np.concatenate([p[0] for p in parts])
    out = dict(E=float(np.dot(coef, E_cl)), E_cluster=E_cl,
               E_orders=O.mbe_orders(clusters, order, E_cl), clusters=clusters, coef=coef,
               order=order, sweeps=np.concatenate([p[1] for p in parts]),
               max_residual=max(p[2] for p in parts), converged=all(p[3] for p in parts),
               workers=nproc)
    if densities:
        dC, dF, de = parts[0][4].copy(), parts[0][5].copy(), parts[0][6].copy()
        Dv = parts[0][7].copy() if dvir else None
        for p in parts[1:]:
            dC += p[4]
            dF += p[5]
            de += p[6]
            if dvir:
                Dv += p[7]
        out.update(dE_dC=None if k_exact else dC, dE_dF=dF, dE_deps=de)
        if dvir:
            out["Dvir"] = Dv
    return out
