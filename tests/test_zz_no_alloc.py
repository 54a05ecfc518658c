"""The allocation-free weak-pair entry point osv_weak_pairs_noalloc, through the
C ABI, against osv_weak_pairs on the same contexts: two calls in a row, the second
on a context with fewer weak pairs (so the static device array still holds the
first call's longer tables), and the refusal beyond its size limit."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2106_06149_amd import _lib as L, synth
from paper_2106_06149_amd.api import OSVContext, Selection, _stream
from oracle import osv_oracle as O

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)


def weak_context(nocc, seed):
    s = synth.make_system(nocc, 60, 50, (4, 9), seed=seed, sel_mode=synth.SEL_OVERLAP)
    s2b = O.s2b_metric(s)
    off = np.sort(s2b[np.triu_indices(nocc, 1)])
    h = len(off) // 2
    l2b = float(0.5 * (off[h - 1] + off[h]))
    return OSVContext.from_system(s, device="cuda:0", sel=Selection(L.OSV_SEL_OVERLAP, l2b=l2b, l3b=0.9))


def call(oc, fn):
    """One count-only call, then one with the per-pair outputs."""
    E = ctypes.c_double()
    n = ctypes.c_int64()
    L.check(fn(oc.handle, _stream(oc.device), ctypes.byref(E), ctypes.byref(n), None, None), oc.handle)
    nw = n.value
    Ep = torch.full((nw,), float("nan"), dtype=torch.float64, device=oc.device)
    pairs = np.full((nw, 2), -1, dtype=np.int32)
    L.check(fn(oc.handle, _stream(oc.device), ctypes.byref(E), ctypes.byref(n),
               ctypes.c_void_p(Ep.data_ptr()), pairs.ctypes.data_as(ctypes.c_void_p)), oc.handle)
    torch.cuda.synchronize()
    return E.value, pairs, Ep.cpu().numpy()


def test_noalloc_weak_pairs_match_allocating_entry_point():
    lib = L.load()
    say("case allocation-free weak pairs: contexts nocc=12 and nocc=7")
    big, small = weak_context(12, 19), weak_context(7, 23)
    ref_big = call(big, lib.osv_weak_pairs)
    ref_small = call(small, lib.osv_weak_pairs)
    assert len(ref_small[1]) < len(ref_big[1]) and len(ref_small[1]) > 0
    got_big = call(big, lib.osv_weak_pairs_noalloc)
    got_small = call(small, lib.osv_weak_pairs_noalloc)      # second call, smaller input
    for ref, got in ((ref_big, got_big), (ref_small, got_small)):
        assert np.array_equal(got[1], ref[1])                # the same pair list
        assert np.array_equal(got[2], ref[2])                # the same kernel: bitwise energies
        scale = np.abs(ref[2]).sum()
        assert abs(got[0] - ref[0]) <= 1e-14 * scale, (got[0], ref[0])
    big.close()
    small.close()


def test_noalloc_weak_pairs_size_limit():
    """More weak pairs than the static array holds: OSV_E_ARG before any device
    work, with the count reported."""
    lib = L.load()
    nocc, nvir, naux = 1500, 4, 8
    say(f"case allocation-free weak pairs beyond the limit: nocc={nocc}")
    # one OSV per LMO, a random unit vector of 4 virtuals: almost every pair has
    # 1e-7 <= s2b <= 2 and is weak
    rng = np.random.default_rng(29)
    q = rng.standard_normal((nvir, nocc))
    q /= np.linalg.norm(q, axis=0)
    F = np.diag(rng.uniform(-1.2, -0.4, nocc))
    s = synth.System(nocc=nocc, nvir=nvir, naux=naux, r=np.ones(nocc, dtype=np.int32),
                     centroid=np.zeros((nocc, 3)), F_occ=F, eps_vir=rng.uniform(0.3, 4.0, nvir),
                     Q=np.asfortranarray(q), C=0.1 * rng.standard_normal((nocc, naux)), B=None,
                     sel_mode=synth.SEL_OVERLAP)
    ov = (q.T @ q) ** 2
    assert int((ov[np.triu_indices(nocc, 1)] >= O.WEAK_MIN).sum()) > L.OSV_NOALLOC_MAX_WEAK
    oc = OSVContext.from_system(s, device="cuda:0", sel=Selection(L.OSV_SEL_OVERLAP, l2b=2.0, l3b=2.0))
    E = ctypes.c_double()
    n = ctypes.c_int64()
    st = lib.osv_weak_pairs_noalloc(oc.handle, _stream(oc.device), ctypes.byref(E), ctypes.byref(n),
                                    None, None)
    assert n.value > L.OSV_NOALLOC_MAX_WEAK
    assert st == L.OSV_E_ARG
    assert b"allocation-free limit" in lib.osv_last_error(oc.handle)
    oc.close()
