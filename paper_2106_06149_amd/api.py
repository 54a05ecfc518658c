"""Python face of libosvmbe: device tensors in, results out.  PyTorch provides
device memory and the HIP stream; every computation runs in the library."""
from __future__ import annotations

import ctypes
from typing import Optional

import numpy as np
import torch

from . import _lib as L


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Selection:
    def __init__(self, mode=L.OSV_SEL_DISTANCE, cut2=15.0, cut3=8.0, l2b=1e-2, l3b=0.2,
                 tau_S=1e-8):
        self.mode, self.cut2, self.cut3, self.l2b, self.l3b, self.tau_S = mode, cut2, cut3, l2b, l3b, tau_S

    def c(self):
        return L.OsvSelect(self.mode, self.cut2, self.cut3, self.l2b, self.l3b, self.tau_S)


def release_cached_memory(device: int = -1):
    """Free the device blocks that the library keeps for reuse by later contexts
    (device -1: every device).  Blocks of live contexts are not touched."""
    L.check(L.load().osv_release_cached_memory(device))


def cached_bytes(device: int = -1) -> int:
    """Bytes of device memory held in the library's block cache."""
    return int(L.load().osv_cached_bytes(device))


def get_tuning() -> dict:
    """The library's launch tuning table (see include/osv.h)."""
    lib = L.load()
    out = {}
    for k in L.TUNING_KEYS:
        v = ctypes.c_int32()
        L.check(lib.osv_get_tuning(k.encode(), ctypes.byref(v)))
        out[k] = v.value
    return out


def set_tuning(**kv):
    lib = L.load()
    for k, v in kv.items():
        L.check(lib.osv_set_tuning(k.encode(), int(v)))


def load_tuning(path: str):
    L.check(L.load().osv_load_tuning(path.encode()))


def plan_clusters(centroid: np.ndarray, sel: Selection):
    """Host-only cluster selection (no GPU): counts, LMO triples (-1 padded), c_X."""
    lib = L.load()
    cen = np.ascontiguousarray(centroid, dtype=np.float64)
    nocc = cen.shape[0]
    counts = L.OsvCounts()
    s = sel.c()
    L.check(lib.osv_plan_clusters(nocc, cen.ctypes.data_as(ctypes.c_void_p), ctypes.byref(s),
                                  ctypes.byref(counts), None, None, 0))
    n = counts.n_clusters
    lmos = np.empty((n, 3), dtype=np.int32)
    coef = np.empty(n, dtype=np.float64)
    L.check(lib.osv_plan_clusters(nocc, cen.ctypes.data_as(ctypes.c_void_p), ctypes.byref(s),
                                  ctypes.byref(counts), lmos.ctypes.data_as(ctypes.c_void_p),
                                  coef.ctypes.data_as(ctypes.c_void_p), n))
    return counts.as_dict(), lmos, coef


def generate_osvs(B: torch.Tensor, eps_vir: torch.Tensor, F_occ: torch.Tensor,
                  l_osv: float = 1e-4, r_max: int = 50):
    """OSVs from the fitted integrals B (nocc x nvir x naux, FP64, on the device):
    returns (r [nocc] int32 numpy array, Qt [sum r, nvir] (Q in the layout
    OSVContext takes), C [sum r, naux], omega [nocc, r_max])."""
    for name, t in (("B", B), ("eps_vir", eps_vir), ("F_occ", F_occ)):
        if not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous float64 device tensor")
    if B.dim() != 3 or eps_vir.shape != (B.shape[1],) or F_occ.shape != (B.shape[0], B.shape[0]):
        raise ValueError("B must be nocc x nvir x naux with eps_vir [nvir] and F_occ nocc x nocc")
    nocc, nvir, naux = (int(x) for x in B.shape)
    lib = L.load()
    r = np.zeros(nocc, dtype=np.int32)
    f64 = dict(dtype=torch.float64, device=B.device)
    Qt = torch.empty(nocc * r_max, nvir, **f64)
    C = torch.empty(nocc * r_max, naux, **f64)
    om = torch.empty(nocc, r_max, **f64)
    with torch.cuda.device(B.device):
        L.check(lib.osv_generate_osvs(nocc, nvir, naux, _ptr(B), _ptr(eps_vir), _ptr(F_occ), l_osv, r_max,
                                      _stream(B.device), r.ctypes.data_as(ctypes.c_void_p), _ptr(om),
                                      _ptr(Qt), _ptr(C)))
    n = int(r.sum())
    return r, Qt[:n], C[:n], om


def generation_stats() -> dict:
    """Device times (ms) and algorithmic flops of the last generate_osvs call of
    this thread, per stage: products, tridiag, vectors, c."""
    out = np.zeros(8)
    L.check(L.load().osv_generation_stats(out.ctypes.data_as(ctypes.c_void_p)))
    return {k: (float(out[2 * i]), float(out[2 * i + 1]))
            for i, k in enumerate(("products", "tridiag", "vectors", "c"))}


def validate_inputs(Q: torch.Tensor, C: torch.Tensor, eps_vir: torch.Tensor,
                    F_occ: torch.Tensor, r) -> None:
    """Checks the tensors handed to the library against osv_system: the library
    keeps their addresses and reads Q, eps_vir and F_occ as FP64 and C as FP64 or
    FP32, dense row-major at the shapes the OSV counts r imply, so a wrong dtype,
    shape or a strided view would make it read past or around the data.  Raises
    ValueError; needs no GPU (the device type is checked by the caller)."""
    r = np.asarray(r)
    if r.ndim != 1 or r.size < 1 or np.any(r < 1):
        raise ValueError("r must be a non-empty 1-D array of OSV counts >= 1")
    nocc, nosv = int(r.size), int(r.sum())
    for name, t in (("Q", Q), ("eps_vir", eps_vir), ("F_occ", F_occ)):
        if t.dtype != torch.float64:
            raise ValueError(f"{name} must be float64 (got {t.dtype})")
    if C.dtype not in (torch.float32, torch.float64):
        raise ValueError(f"C must be float32 or float64 (got {C.dtype})")
    if eps_vir.dim() != 1:
        raise ValueError("eps_vir must be 1-D [nvir]")
    nvir = int(eps_vir.shape[0])
    if tuple(Q.shape) != (nosv, nvir):
        raise ValueError(f"Q must be given as Q^T, shape (sum r, nvir) = ({nosv}, {nvir}); "
                         f"got {tuple(Q.shape)}")
    if C.dim() != 2 or C.shape[0] != nosv or C.shape[1] < 1:
        raise ValueError(f"C must have shape (sum r, naux) with sum r = {nosv}; got {tuple(C.shape)}")
    if tuple(F_occ.shape) != (nocc, nocc):
        raise ValueError(f"F_occ must have shape ({nocc}, {nocc}); got {tuple(F_occ.shape)}")
    for name, t in (("Q", Q), ("C", C), ("eps_vir", eps_vir), ("F_occ", F_occ)):
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous (row-major); got strides {t.stride()}")
    devs = {t.device for t in (Q, C, eps_vir, F_occ)}
    if len(devs) != 1:
        raise ValueError(f"Q, C, eps_vir and F_occ must be on one device; got {sorted(map(str, devs))}")


class OSVContext:
    """One built problem.  The input tensors are borrowed by the library and kept
    alive here until close()."""

    def __init__(self, Q: torch.Tensor, C: torch.Tensor, eps_vir: torch.Tensor,
                 F_occ: torch.Tensor, r, centroid=None, sel: Selection = None,
                 precision: int = L.OSV_FP64, B: torch.Tensor = None):
        """With B (nocc x nvir x naux, FP64, on the device) the strong pairs' domain
        integrals are the cross-projected ones (osv_build_pairs_exact); C is then
        formed by the library and may be None."""
        self.lib = L.load()
        self.device = Q.device
        sel = sel or Selection()
        self.r = np.ascontiguousarray(np.asarray(r), dtype=np.int32)
        self.cen = None if centroid is None else np.ascontiguousarray(centroid, dtype=np.float64)
        self.handle = None
        if B is not None:
            if not B.is_cuda or B.dtype != torch.float64 or not B.is_contiguous() or B.dim() != 3 \
                    or B.shape[0] != len(self.r) or B.shape[1] != eps_vir.shape[0]:
                raise ValueError("B must be a contiguous float64 device tensor nocc x nvir x naux")
            if C is None:
                C = torch.empty(int(self.r.sum()), B.shape[2], dtype=torch.float64, device=B.device)
        self.B = B
        # Q is nvir x sum(r) column-major: we hold its transpose as a contiguous tensor
        self.Q, self.C, self.eps, self.F = Q, C, eps_vir, F_occ
        validate_inputs(Q, C, eps_vir, F_occ, self.r)
        for name, t in (("Q", Q), ("C", C), ("eps_vir", eps_vir), ("F_occ", F_occ)):
            if not t.is_cuda:
                raise ValueError(f"{name} must be a device tensor")
        nvir = eps_vir.shape[0]
        self.nocc, self.nvir, self.naux = len(self.r), nvir, C.shape[1]
        self.nosv = int(self.r.sum())
        sysc = L.OsvSystem(self.nocc, nvir, self.naux,
                           self.r.ctypes.data_as(ctypes.c_void_p), Q.data_ptr(), C.data_ptr(),
                           L.OSV_DT_F32 if C.dtype == torch.float32 else L.OSV_DT_F64,
                           eps_vir.data_ptr(), F_occ.data_ptr(),
                           None if self.cen is None else self.cen.ctypes.data_as(ctypes.c_void_p))
        self.sel = sel
        s = sel.c()
        h = ctypes.c_void_p()
        self.handle = None
        with torch.cuda.device(self.device):
            if B is not None:
                L.check(self.lib.osv_build_pairs_exact(ctypes.byref(sysc), _ptr(B), ctypes.byref(s), precision,
                                                       _stream(self.device), ctypes.byref(h)))
            else:
                L.check(self.lib.osv_build_pairs(ctypes.byref(sysc), ctypes.byref(s), precision,
                                                 _stream(self.device), ctypes.byref(h)))
        self.handle = h
        self.precision = precision
        c = L.OsvCounts()
        L.check(self.lib.osv_query(self.handle, ctypes.byref(c)), self.handle)
        self.counts = c.as_dict()

    @classmethod
    def from_system(cls, s, device="cuda", precision=None, sel: Selection = None, k_exact: bool = False):
        """Copy a synth.System to the device and build it (k_exact: cross-projected
        integrals from the system's B)."""
        dev = torch.device(device)
        if k_exact:
            B = torch.from_numpy(np.ascontiguousarray(s.B)).to(dev)
            Qt = torch.from_numpy(np.ascontiguousarray(s.Q.T)).to(dev)
            eps = torch.from_numpy(np.ascontiguousarray(s.eps_vir)).to(dev)
            F = torch.from_numpy(np.ascontiguousarray(s.F_occ)).to(dev)
            sel = sel or Selection(s.sel_mode, s.cut2, s.cut3)
            return cls(Qt, None, eps, F, s.r, s.centroid, sel, L.OSV_FP64, B=B)
        Qt = torch.from_numpy(np.ascontiguousarray(s.Q.T)).to(dev)   # sum(r) x nvir row-major = Q col-major
        C = torch.from_numpy(np.ascontiguousarray(s.C)).to(dev)
        eps = torch.from_numpy(np.ascontiguousarray(s.eps_vir)).to(dev)
        F = torch.from_numpy(np.ascontiguousarray(s.F_occ)).to(dev)
        prec = s.precision if precision is None else precision
        sel = sel or Selection(s.sel_mode, s.cut2, s.cut3)
        return cls(Qt, C, eps, F, s.r, s.centroid, sel, prec)

    def solve(self, tau_R=1e-10, max_sweeps=60, raise_on_error=True):
        info = L.OsvSolveInfo()
        with torch.cuda.device(self.device):
            st = self.lib.osv_solve_clusters(self.handle, tau_R, max_sweeps, _stream(self.device),
                                             ctypes.byref(info))
        if raise_on_error:
            L.check(st, self.handle)
        return dict(status=st, sweeps=info.sweeps, max_residual=info.max_residual,
                    converged=bool(info.converged), n_not_converged=info.n_not_converged)

    def energy(self, per_cluster=False):
        E = ctypes.c_double()
        orders = (ctypes.c_double * 3)()
        Ecl = None
        if per_cluster:
            Ecl = torch.empty(self.counts["n_clusters"], dtype=torch.float64, device=self.device)
        with torch.cuda.device(self.device):
            L.check(self.lib.osv_energy(self.handle, _stream(self.device), ctypes.byref(E), orders,
                                        _ptr(Ecl)), self.handle)
        return E.value, np.array(orders[:]), Ecl

    def weak_pairs(self):
        """Weak 2b clusters (overlap selection): (E_weak, pairs [n, 2] int32 array,
        per-pair energies as a device tensor), by the one-block scheme."""
        E = ctypes.c_double()
        n = ctypes.c_int64()
        with torch.cuda.device(self.device):
            if getattr(self, "_n_weak", None) is None:
                # the pair count first (the list is fixed by the build)
                L.check(self.lib.osv_weak_pairs(self.handle, _stream(self.device), ctypes.byref(E),
                                                ctypes.byref(n), None, None), self.handle)
                self._n_weak = n.value
            nw = self._n_weak
            pairs = np.zeros((nw, 2), dtype=np.int32)
            Ep = torch.empty(nw, dtype=torch.float64, device=self.device)
            if nw:
                L.check(self.lib.osv_weak_pairs(self.handle, _stream(self.device), ctypes.byref(E),
                                                ctypes.byref(n), _ptr(Ep),
                                                pairs.ctypes.data_as(ctypes.c_void_p)), self.handle)
        return E.value, pairs, Ep

    def high_order_correction(self):
        """One-step correction of the MBE(3) amplitudes: (dE, E_coll, max_dR,
        per-domain [n_domains, 3] array of dE_d, E_d, ||W^T dR W||_F)."""
        dE, Ec, mx = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        per = np.zeros((self.counts["n_domains"], 3))
        with torch.cuda.device(self.device):
            L.check(self.lib.osv_high_order_correction(self.handle, _stream(self.device), ctypes.byref(dE),
                                                       ctypes.byref(Ec), ctypes.byref(mx),
                                                       per.ctypes.data_as(ctypes.c_void_p)), self.handle)
        return dE.value, Ec.value, mx.value, per

    def correction_stats(self):
        """The last high_order_correction call: {"collective": (ms, bytes),
        "step": (ms, flops)}."""
        out = np.zeros(4)
        L.check(self.lib.osv_correction_stats(self.handle, out.ctypes.data_as(ctypes.c_void_p)), self.handle)
        return {"collective": (float(out[0]), float(out[1])), "step": (float(out[2]), float(out[3]))}

    def response_layout(self):
        """Ordered pairs (n_pairs x 2 int32 array) and the offset of each one's
        n x n block in the output of response()."""
        npair, nd = ctypes.c_int64(), ctypes.c_int64()
        L.check(self.lib.osv_response_layout(self.handle, ctypes.byref(npair), ctypes.byref(nd), None, None),
                self.handle)
        pairs = np.zeros((npair.value, 2), dtype=np.int32)
        offs = np.zeros(npair.value, dtype=np.int64)
        L.check(self.lib.osv_response_layout(self.handle, None, None, pairs.ctypes.data_as(ctypes.c_void_p),
                                             offs.ctypes.data_as(ctypes.c_void_p)), self.handle)
        return pairs, offs, nd.value

    def response(self, out=None):
        """OSV response intermediates N_ij (eq:nij, MBE-combined) of every ordered
        pair: (flat device tensor, pairs, offsets, (ms, flops))."""
        pairs, offs, nd = self.response_layout()
        if out is None:
            out = torch.empty(max(nd, 1), dtype=torch.float64, device=self.device)
        elif out.numel() < nd or out.dtype != torch.float64 or not out.is_contiguous():
            raise ValueError(f"response(): out needs {nd} contiguous float64 elements")
        mf = np.zeros(2)
        with torch.cuda.device(self.device):
            L.check(self.lib.osv_response(self.handle, _stream(self.device), _ptr(out),
                                          mf.ctypes.data_as(ctypes.c_void_p)), self.handle)
        return out, pairs, offs, (float(mf[0]), float(mf[1]))

    def weak_response(self):
        """Weak pairs' N^up_ij = T_(i,j) K_(j,i) (eq:nij2b, one-block scheme) as a
        dict {(i, j): r_i x r_i host array}, pairs in the order of weak_pairs()."""
        _, pairs, _ = self.weak_pairs()
        nd = ctypes.c_int64()
        L.check(self.lib.osv_weak_response(self.handle, None, ctypes.byref(nd), None), self.handle)
        out = torch.empty(max(nd.value, 1), dtype=torch.float64, device=self.device)
        with torch.cuda.device(self.device):
            L.check(self.lib.osv_weak_response(self.handle, _stream(self.device), None, _ptr(out)),
                    self.handle)
        h = out.cpu().numpy()
        res, o = {}, 0
        for i, j in pairs:
            ri = int(self.r[i])
            res[(int(i), int(j))] = h[o:o + ri * ri].reshape(ri, ri)
            o += ri * ri
        return res

    def response_blocks(self):
        """N_ij as a dict {(i, j): n x n host array}."""
        N, pairs, offs, _ = self.response()
        h = N.cpu().numpy()
        out = {}
        for (i, j), o in zip(pairs, offs):
            n = self.r[i] + (self.r[j] if i != j else 0)
            out[(int(i), int(j))] = h[o:o + n * n].reshape(n, n)
        return out

    def densities(self, dC=True, dF=True, deps=True, dvir=False):
        f64 = dict(dtype=torch.float64, device=self.device)
        out_C = torch.empty(self.nosv, self.naux, **f64) if dC else None
        out_F = torch.empty(self.nocc, self.nocc, **f64) if dF else None
        out_e = torch.empty(self.nvir, **f64) if deps else None
        out_D = torch.empty(self.nvir, self.nvir, **f64) if dvir else None
        with torch.cuda.device(self.device):
            L.check(self.lib.osv_densities(self.handle, _stream(self.device), _ptr(out_C),
                                           _ptr(out_F), _ptr(out_e), _ptr(out_D)), self.handle)
        return out_C, out_F, out_e, out_D

    STAGES = ["sf", "k", "prep", "couplings", "solve", "energy", "adjoint", "backtransform",
              "host_plan"]

    def stage_times(self):
        ms = (ctypes.c_double * 9)()
        L.check(self.lib.osv_stage_times(self.handle, ms), self.handle)
        return dict(zip(self.STAGES, ms[:]))

    def stage_flops(self):
        f = (ctypes.c_double * 9)()
        L.check(self.lib.osv_stage_flops(self.handle, f), self.handle)
        return dict(zip(self.STAGES, f[:]))

    def close(self):
        if self.handle is not None:
            self.lib.osv_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
