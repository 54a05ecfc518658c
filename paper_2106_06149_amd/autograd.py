"""torch.autograd.Function over the library: forward = build + solve + MBE
energy; backward = the hand-written adjoint (osv_densities).  By Hylleraas
stationarity the amplitudes contribute nothing, so the backward returns the
density contributions dE/dC_i, dE/dF_occ and dE/deps_vir directly."""
import torch

from . import _lib as L
from .api import OSVContext, Selection


class OSVEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, C, F_occ, eps_vir, Qt, r, centroid, sel: Selection, precision: int,
                tau_R: float = 1e-10):
        oc = OSVContext(Qt, C, eps_vir, F_occ, r, centroid, sel, precision)
        oc.solve(tau_R=tau_R)
        E, _, _ = oc.energy()
        ctx.oc = oc
        ctx.c_dtype = C.dtype
        # the library reads C (dE/dC = 2 G^K C) and the Fock inputs again in the
        # backward: saving them lets autograd's version counter reject in-place
        # changes made between forward and backward
        ctx.save_for_backward(C, F_occ, eps_vir)
        return torch.tensor(E, dtype=torch.float64, device=C.device)

    @staticmethod
    def backward(ctx, g):
        ctx.saved_tensors   # raises if C, F_occ or eps_vir changed in place
        oc = ctx.oc
        dC, dF, de, _ = oc.densities(dC=ctx.needs_input_grad[0], dF=ctx.needs_input_grad[1],
                                     deps=ctx.needs_input_grad[2])
        gC = None if dC is None else (g * dC).to(ctx.c_dtype)
        gF = None if dF is None else g * dF
        ge = None if de is None else g * de
        oc.close()
        return gC, gF, ge, None, None, None, None, None, None
