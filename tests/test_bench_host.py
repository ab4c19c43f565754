"""Host-side pieces of bench.py (no GPU): the FP64 operation count it reports is the
oracle's own count of the left-looking factorization, recomputed from the factors."""
import os
import sys

import pytest

import oracle
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


@pytest.mark.parametrize("case", ["mna", "btf"])
def test_factor_flops_match_the_oracle(case):
    import bench
    if case == "mna":
        a = synth.gen_mna(800, seed=4)
    else:
        a = synth.gen_batched_btf(nblocks=200, big=1500, seed=8).a
    f = oracle.factor(a, oracle.Ordering.natural(a.n), update_order=oracle.ORDER_ASCENDING)
    assert f.status == oracle.OK
    assert bench.factor_flops(f) == f.flops
