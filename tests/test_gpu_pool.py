"""The library's device block cache: contexts built one after another reuse
blocks freed by earlier ones, and no kernel depends on what a block held before.

Each case runs the same system three times through the C ABI: first on fresh
blocks with the cache emptied, then twice with OSV_POOL_POISON=1 (every block
handed out filled with 0xFF bytes, NaN as FP64; the third run takes the blocks
the second one left).  Results must agree bit for bit with the first run."""
import numpy as np
import pytest

from paper_2106_06149_amd import synth
from paper_2106_06149_amd.api import OSVContext, cached_bytes, release_cached_memory

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)


def run(s, precision):
    oc = OSVContext.from_system(s, device="cuda:0", precision=precision)
    oc.solve(tau_R=1e-10)
    E, orders, Ecl = oc.energy(per_cluster=True)
    dC, dF, de, Dv = oc.densities(dvir=True)
    out = [np.array([E]), orders, Ecl.cpu().numpy(), dC.cpu().numpy(), dF.cpu().numpy(),
           de.cpu().numpy(), Dv.cpu().numpy()]
    oc.close()
    return out


@pytest.mark.parametrize("precision", [0, 1])
def test_reused_and_poisoned_blocks_bitwise(monkeypatch, precision):
    c_dtype = np.float32 if precision == 1 else np.float64
    s = synth.make_system(12, 90, 200, (5, 21), seed=31, cut2=6.5, cut3=4.5,
                          c_dtype=c_dtype, precision=precision)
    say(f"case block cache precision={precision} nocc=12 nvir=90 naux=200 r=5..21")
    release_cached_memory(-1)
    assert cached_bytes(-1) == 0
    ref = run(s, precision)
    assert cached_bytes(-1) > 0          # the context's blocks went back to the cache
    assert all(np.all(np.isfinite(x)) for x in ref)
    monkeypatch.setenv("OSV_POOL_POISON", "1")
    for rep in range(2):
        got = run(s, precision)
        for a, b in zip(got, ref):
            assert np.array_equal(a, b), rep
    monkeypatch.delenv("OSV_POOL_POISON")
    release_cached_memory(0)
    assert cached_bytes(0) == 0
