"""Mixed precision (binary32 M2L on radius-scaled expansions, everything else
binary64) against the binary64 oracle, through the C ABI.

The tolerance is not a parity bound but the accuracy target of the mode
(1e-6 relative): binary32 carries 24 bits, the translations of one batch are
summed in binary32 and the batches in binary64.  Measured on these workloads
the far field differs from the binary64 one by about 1e-7 normwise and by up
to 6e-7 relative to the largest value (order 1, field).
"""
import numpy as np
import pytest

from paper_2002_04894_amd import workloads as W
from test_gpu_parity import F, assert_close, dev, gpu_tree, make, say, torch  # noqa: F401 (fixtures)

pytestmark = pytest.mark.gpu

MIXED_TOL = 1e-6


def gpu_eval_prec(torch, F, tree, q, p, parts, precision):
    qd = dev(torch, q)
    outs = [torch.empty_like(qd) for _ in range(4)]
    F.fmm_evaluate_tree(tree, qd, p, *outs, parts=parts, precision=precision)
    torch.cuda.synchronize()
    return [o.cpu().numpy() for o in outs]


@pytest.mark.parametrize("p", list(range(16)))
def test_mixed_far_field_vs_oracle(torch, F, orc, p):
    say(f"[mixed] far field p={p}")
    x, y, z, q = make("gmix", 2_000, seed=4)
    ot = orc.Tree(x, y, z, 2, 0.6)
    gt = gpu_tree(torch, F, x, y, z, 2, 0.6)
    ref = ot.evaluate(q, p, parts=2)
    got = gpu_eval_prec(torch, F, gt, q, p, 2, F.FMM_PREC_MIXED)
    assert_close(got, ref, tol=MIXED_TOL, what=f"mixed far p={p}")
    gt.free()


def test_mixed_plummer_all_parts(torch, F, orc):
    say("[mixed] plummer 4000, 3 levels, p 8")
    x, y, z, q = make("plummer", 4_000, seed=5)
    ot = orc.Tree(x, y, z, 3, 0.5)
    gt = gpu_tree(torch, F, x, y, z, 3, 0.5)
    ref = ot.evaluate(q, 8)
    got = gpu_eval_prec(torch, F, gt, q, 8, 3, F.FMM_PREC_MIXED)
    assert_close(got, ref, tol=MIXED_TOL, what="mixed plummer")
    # the near field alone is binary64 in this mode: bit-identical
    near_m = gpu_eval_prec(torch, F, gt, q, 8, 1, F.FMM_PREC_MIXED)
    near_d = gpu_eval_prec(torch, F, gt, q, 8, 1, F.FMM_PREC_F64)
    for a, b in zip(near_m, near_d):
        assert np.array_equal(a, b)
    gt.free()


def test_mixed_above_order_15_is_binary64(torch, F):
    x, y, z, q = W.uniform_cube(1_500, seed=6)
    gt = gpu_tree(torch, F, x, y, z, 2, 0.5)
    a = gpu_eval_prec(torch, F, gt, q, 16, 3, F.FMM_PREC_MIXED)
    b = gpu_eval_prec(torch, F, gt, q, 16, 3, F.FMM_PREC_F64)
    for u, v in zip(a, b):
        assert np.array_equal(u, v)
    gt.free()


def test_unknown_precision_rejected(torch, F):
    x, y, z, q = W.uniform_cube(100, seed=1)
    gt = gpu_tree(torch, F, x, y, z, 1, 0.5)
    with pytest.raises(F.FMMError) as e:
        gpu_eval_prec(torch, F, gt, q, 3, 3, 2)
    assert e.value.code == F.FMM_EINVAL
    gt.free()
