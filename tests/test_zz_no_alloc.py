"""The solve entry point that allocates nothing (basker_solve_noalloc), through the C
ABI, against basker_solve on the same factors: bitwise equal results on two calls in a
row, the second with a smaller system, no device memory taken by the handle, and a
clear refusal when a solve needs more than the static scratch."""
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def bk():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1601_05725_amd as bk
    bk.load()
    return bk


def test_noalloc_solve_equals_solve(bk, oracle_lib):
    import torch
    cases = [("mna12k-nd", synth.gen_mna(12000, seed=6), dict(nd_min_block=3000, nd_leaves=8), 3),
             ("mna2k", synth.gen_mna(2000, seed=9), {}, 1)]
    for label, a, opts, nrhs in cases:
        say("no-alloc solve %s n=%d nrhs=%d" % (label, a.n, nrhs))
        h = bk.Handle.symbolic(a, bk.default_options(**opts))
        h.factor(a.values)
        b = synth.rhs(a.n, nrhs, ident=77)
        Bt = torch.from_numpy(np.ascontiguousarray(b.T)).cuda()
        torch.cuda.synchronize()
        held = h.info()["device_bytes"]
        h.solve_noalloc(Bt)            # first solve on this handle: nothing allocated yet
        torch.cuda.synchronize()
        assert h.info()["device_bytes"] == held
        x = Bt.cpu().numpy().T.copy()
        ref = h.solve(b)               # the allocating entry point on the same factors
        np.testing.assert_array_equal(x, ref)
        assert oracle_lib.residual(a, x, b) <= 1e-12
        h.free()


def test_noalloc_solve_refuses_oversized(bk):
    import torch
    a = synth.gen_mna(12000, seed=6)
    h = bk.Handle.symbolic(a)
    h.factor(a.values)
    nrhs = (4 << 20) // (2 * a.n) + 1     # 2 n nrhs doubles exceed the 4 Mi-double scratch
    B = torch.zeros((nrhs, a.n), dtype=torch.float64, device="cuda")
    with pytest.raises(bk.BaskerError) as e:
        h.solve_noalloc(B)
    assert e.value.status == bk.ERR_WORKSPACE
    h.free()
