"""Seeded synthetic OSV-MP2 systems.

This module only draws inputs: LMO centroids, occupied Fock matrix, virtual
orbital energies, OSV matrices Q_i and the OSV-projected fitted integrals
C_i = Q_i^T B_i (the one-index OSV transformation of eq:osv applied to the
fitted 3-index integrals; in the C-direct workloads C_i is drawn itself).
It contains none of the residual, energy, MBE or density arithmetic, and is
the only code that both the GPU path and the CPU oracle read.

Workload recipes stand in for the paper's molecules (polyglycine chains are
modelled by LMO centroids on a line, water clusters by a jittered 3D lattice;
Section "Scaling and Parallel Performance" and the large-system timing table).

Draw order (numpy PCG64, seed = 2106061490 + workload index):
  1. lattice jitter (3D geometries only)
  2. r_i (when drawn from a range)
  3. eps_occ, 4. eps_vir, 5. virtual centres, 6. aux centres (C-direct only)
  7. one Gaussian nvir x r_i matrix per LMO (in LMO order), for Q_i
  8. B (nocc x nvir x naux) or C (sum r x naux) directly.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional, Tuple

import numpy as np

SEED_BASE = 2106061490

# Cluster selection modes (shared vocabulary of the C ABI).
SEL_DISTANCE = 0
SEL_OVERLAP = 1
SEL_FULL = 2


@dataclasses.dataclass
class System:
    """Inputs of one OSV-MP2 problem (all float64 unless stated)."""

    nocc: int
    nvir: int
    naux: int
    r: np.ndarray            # int32 [nocc], OSVs per LMO
    centroid: np.ndarray     # [nocc, 3] bohr
    F_occ: np.ndarray        # [nocc, nocc] symmetric, diagonal = eps_occ
    eps_vir: np.ndarray      # [nvir]
    Q: np.ndarray            # [nvir, sum r] Fortran order (column-major); block i at off[i]
    C: np.ndarray            # [sum r, naux] C order (row = one OSV); float64 or float32
    B: Optional[np.ndarray]  # [nocc, nvir, naux] fitted integrals (B-based workloads) or None
    name: str = "custom"
    # selection parameters of the workload
    sel_mode: int = SEL_DISTANCE
    cut2: float = 15.0
    cut3: float = 8.0
    precision: int = 0       # 0 = FP64, 1 = MIXED

    @property
    def off(self) -> np.ndarray:
        o = np.zeros(self.nocc + 1, dtype=np.int64)
        o[1:] = np.cumsum(self.r)
        return o

    @property
    def nosv(self) -> int:
        return int(np.sum(self.r))

    def Qi(self, i: int) -> np.ndarray:
        o = self.off
        return self.Q[:, o[i]:o[i + 1]]

    def Ci(self, i: int) -> np.ndarray:
        o = self.off
        return self.C[o[i]:o[i + 1], :]


def _line_centroids(nocc: int, spacing: float) -> np.ndarray:
    c = np.zeros((nocc, 3))
    c[:, 0] = spacing * np.arange(nocc)
    return c


def _lattice_centroids(rng: np.random.Generator, nocc: int, spacing: float,
                       jitter: float) -> np.ndarray:
    n = int(math.ceil(round(nocc ** (1.0 / 3.0), 9)))
    while n ** 3 < nocc:
        n += 1
    sites = []
    for iz in range(n):
        for iy in range(n):
            for ix in range(n):
                sites.append((ix, iy, iz))
    sites = np.array(sites[:nocc], dtype=np.float64) * spacing
    sites += rng.uniform(-jitter, jitter, size=sites.shape)
    return sites


def _householder_qr_q(a: np.ndarray) -> np.ndarray:
    """Orthonormal Q of a Householder QR with the sign fixed so diag(R) > 0."""
    q, rr = np.linalg.qr(a, mode="reduced")
    s = np.sign(np.diag(rr))
    s[s == 0] = 1.0
    return q * s[None, :]


def make_system(nocc: int, nvir: int, naux: int, r, *, seed: int,
                geometry: str = "line", spacing: float = 2.0, jitter: float = 0.3,
                c_direct: bool = False, c_dtype=np.float64,
                f_offdiag: float = 0.02, f_decay: float = 3.0,
                q_decay: float = 3.0, b_decay: float = 4.0, b_scale: float = 0.1,
                eps_occ_range=(-1.2, -0.4), eps_vir_range=(0.3, 4.0),
                name: str = "custom", sel_mode: int = SEL_DISTANCE,
                cut2: float = 15.0, cut3: float = 8.0, precision: int = 0,
                keep_B: bool = True, geometry_only: bool = False):
    """Draw one system.  `r` is an int (all LMOs), a (lo, hi) inclusive range,
    or an explicit sequence.  r_i = nvir gives square orthogonal Q_i (the
    all-OSV limit)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if geometry == "line":
        cen = _line_centroids(nocc, spacing)
    elif geometry == "lattice":
        cen = _lattice_centroids(rng, nocc, spacing, jitter)
    else:
        raise ValueError(geometry)

    if isinstance(r, (int, np.integer)):
        rr = np.full(nocc, int(r), dtype=np.int32)
    elif isinstance(r, tuple) and len(r) == 2:
        rr = rng.integers(r[0], r[1] + 1, size=nocc).astype(np.int32)
    else:
        rr = np.asarray(r, dtype=np.int32).copy()
        assert rr.shape == (nocc,)
    if np.any(rr < 1) or np.any(rr > nvir):
        raise ValueError("r_i must lie in [1, nvir]")
    if geometry_only:
        # centroids and r_i are the first draws, so they equal the full draw's
        return cen, rr

    eps_occ = rng.uniform(eps_occ_range[0], eps_occ_range[1], size=nocc)
    eps_vir = rng.uniform(eps_vir_range[0], eps_vir_range[1], size=nvir)

    if geometry == "line":
        vcen = np.zeros((nvir, 3))
        vcen[:, 0] = rng.uniform(0.0, spacing * nocc, size=nvir)
    else:
        lo = cen.min(axis=0) - 1.25
        hi = cen.max(axis=0) + 1.25
        vcen = rng.uniform(lo, hi, size=(nvir, 3))
    acen = None
    if c_direct:
        if geometry == "line":
            acen = np.zeros((naux, 3))
            acen[:, 0] = rng.uniform(0.0, spacing * nocc, size=naux)
        else:
            lo = cen.min(axis=0) - 1.25
            hi = cen.max(axis=0) + 1.25
            acen = rng.uniform(lo, hi, size=(naux, 3))

    dist_ij = np.linalg.norm(cen[:, None, :] - cen[None, :, :], axis=-1)
    F_occ = f_offdiag * np.exp(-dist_ij / f_decay)
    np.fill_diagonal(F_occ, eps_occ)

    nosv = int(rr.sum())
    off = np.zeros(nocc + 1, dtype=np.int64)
    off[1:] = np.cumsum(rr)
    Q = np.zeros((nvir, nosv), dtype=np.float64, order="F")
    for i in range(nocc):
        g = rng.standard_normal((nvir, int(rr[i])))
        w = np.exp(-np.linalg.norm(vcen - cen[i], axis=1) / q_decay)
        Q[:, off[i]:off[i + 1]] = _householder_qr_q(g * w[:, None])

    B = None
    if c_direct:
        C = np.empty((nosv, naux), dtype=c_dtype)
        for i in range(nocc):
            dec = np.exp(-np.linalg.norm(acen - cen[i], axis=1) / b_decay)
            g = rng.standard_normal((int(rr[i]), naux))
            C[off[i]:off[i + 1], :] = (b_scale * g * dec[None, :]).astype(c_dtype)
    else:
        B = np.empty((nocc, nvir, naux))
        for i in range(nocc):
            dec = np.exp(-np.linalg.norm(vcen - cen[i], axis=1) / b_decay)
            B[i] = b_scale * rng.standard_normal((nvir, naux)) * dec[:, None]
        C = np.empty((nosv, naux), dtype=np.float64)
        for i in range(nocc):
            # one-index OSV transformation of the fitted integrals (eq:osv)
            C[off[i]:off[i + 1], :] = Q[:, off[i]:off[i + 1]].T @ B[i]
        C = C.astype(c_dtype)
        if not keep_B:
            B = None
    return System(nocc=nocc, nvir=nvir, naux=naux, r=rr, centroid=cen, F_occ=F_occ,
                  eps_vir=eps_vir, Q=Q, C=np.ascontiguousarray(C), B=B, name=name,
                  sel_mode=sel_mode, cut2=cut2, cut3=cut3, precision=precision)


# Five workloads.  Index k uses seed SEED_BASE + k.
WORKLOADS = {
    0: dict(name="full-osv-mp2-line-nocc6", nocc=6, nvir=60, naux=150, r=8,
            geometry="line", c_direct=False, sel_mode=SEL_FULL, precision=0),
    1: dict(name="mbe3-line-nocc32", nocc=32, nvir=320, naux=800, r=12,
            geometry="line", c_direct=False, sel_mode=SEL_DISTANCE, cut2=15.0, cut3=8.0,
            precision=0),
    2: dict(name="mbe3-lattice-nocc128-mixed", nocc=128, nvir=1280, naux=3200, r=(10, 40),
            geometry="lattice", spacing=2.5, c_direct=True, c_dtype=np.float32,
            sel_mode=SEL_DISTANCE, cut2=15.0, cut3=8.0, precision=1),
    3: dict(name="mbe3-line-nocc64-gradient", nocc=64, nvir=640, naux=1600, r=(10, 20),
            geometry="line", c_direct=False, sel_mode=SEL_DISTANCE, cut2=15.0, cut3=8.0,
            precision=0),
    4: dict(name="mbe3-lattice-nocc400-large", nocc=400, nvir=4000, naux=10000, r=(15, 50),
            geometry="lattice", spacing=2.5, c_direct=True, c_dtype=np.float32,
            sel_mode=SEL_DISTANCE, cut2=15.0, cut3=7.0, precision=1),
}


def workload(k: int, **overrides) -> System:
    """Draw workload k (0..4) with its fixed seed; keyword overrides allowed
    (a smaller copy keeps the recipe but changes sizes).  With
    geometry_only=True only (centroids, r) are returned."""
    spec = dict(WORKLOADS[k])
    spec.update(overrides)
    nocc = spec.pop("nocc")
    nvir = spec.pop("nvir")
    naux = spec.pop("naux")
    r = spec.pop("r")
    seed = spec.pop("seed", SEED_BASE + k)
    return make_system(nocc, nvir, naux, r, seed=seed, **spec)
