"""The Python binding's checks of the tensors it hands to the library (no GPU):
the library keeps their addresses and reads them at fixed dtypes and shapes, so
each mismatch must raise before any device call."""
import numpy as np
import pytest
import torch

from paper_2106_06149_amd import api, synth


def tensors(s, c_dtype=torch.float64):
    Qt = torch.from_numpy(np.ascontiguousarray(s.Q.T))
    C = torch.from_numpy(np.ascontiguousarray(s.C)).to(c_dtype)
    eps = torch.from_numpy(s.eps_vir.copy())
    F = torch.from_numpy(s.F_occ.copy())
    return Qt, C, eps, F


@pytest.fixture(scope="module")
def sysm():
    return synth.make_system(4, 13, 9, [2, 3, 4, 3], seed=3)


def test_valid_inputs_pass(sysm):
    api.validate_inputs(*tensors(sysm), sysm.r)
    api.validate_inputs(*tensors(sysm, torch.float32), sysm.r)


@pytest.mark.parametrize("which", ["Q", "eps", "F"])
def test_wrong_dtype_rejected(sysm, which):
    Qt, C, eps, F = tensors(sysm)
    if which == "Q":
        Qt = Qt.float()
    elif which == "eps":
        eps = eps.float()
    else:
        F = F.float()
    with pytest.raises(ValueError, match="float64"):
        api.validate_inputs(Qt, C, eps, F, sysm.r)


def test_wrong_C_dtype_rejected(sysm):
    Qt, C, eps, F = tensors(sysm)
    with pytest.raises(ValueError, match="C must be float32 or float64"):
        api.validate_inputs(Qt, C.half(), eps, F, sysm.r)


def test_wrong_shapes_rejected(sysm):
    Qt, C, eps, F = tensors(sysm)
    with pytest.raises(ValueError, match="Q must be given as Q\\^T"):
        api.validate_inputs(Qt.T.contiguous(), C, eps, F, sysm.r)   # nvir x sum(r) instead
    with pytest.raises(ValueError, match="C must have shape"):
        api.validate_inputs(Qt, C[:-1].contiguous(), eps, F, sysm.r)
    with pytest.raises(ValueError, match="F_occ must have shape"):
        api.validate_inputs(Qt, C, eps, F[:3, :3].contiguous(), sysm.r)
    with pytest.raises(ValueError, match="eps_vir must be 1-D"):
        api.validate_inputs(Qt, C, eps[None, :], F, sysm.r)
    with pytest.raises(ValueError, match="r must be"):
        api.validate_inputs(Qt, C, eps, F, np.array([2, 0, 4, 3]))


def test_strided_views_rejected(sysm):
    Qt, C, eps, F = tensors(sysm)
    wide = torch.zeros(C.shape[0], 2 * C.shape[1], dtype=C.dtype)
    wide[:, ::2] = C
    with pytest.raises(ValueError, match="contiguous"):
        api.validate_inputs(Qt, wide[:, ::2], eps, F, sysm.r)
    with pytest.raises(ValueError, match="contiguous"):
        api.validate_inputs(Qt, C, eps, F.T, sysm.r)   # same shape, transposed strides


def test_mixed_devices_rejected(sysm):
    Qt, C, eps, F = tensors(sysm)
    with pytest.raises(ValueError, match="one device"):
        api.validate_inputs(Qt, C.to("meta"), eps, F, sysm.r)


def test_context_refuses_host_tensors_before_any_device_call(sysm):
    with pytest.raises(ValueError, match="device tensor"):
        api.OSVContext(*tensors(sysm), sysm.r, sysm.centroid)


def test_context_methods_present():
    """Every call of the boundary has its method on OSVContext (each wraps one
    C-ABI entry point; a method lost in an edit fails here, without a GPU)."""
    import inspect
    want = {"solve": "osv_solve_clusters", "energy": "osv_energy", "densities": "osv_densities",
            "weak_pairs": "osv_weak_pairs", "high_order_correction": "osv_high_order_correction",
            "response_layout": "osv_response_layout", "response": "osv_response",
            "weak_response": "osv_weak_response", "stage_times": "osv_stage_times",
            "correction_stats": "osv_correction_stats",
            "stage_flops": "osv_stage_flops"}
    for name, entry in want.items():
        fn = getattr(api.OSVContext, name, None)
        assert callable(fn), name
        assert entry in inspect.getsource(fn), (name, entry)
