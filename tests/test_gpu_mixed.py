"""Mixed precision (binary32 M2L on radius-scaled expansions, everything else
binary64) and the binary32 near field (FMM_PREC_F32: also P2P in binary32,
compensated sums) against the binary64 oracle, through the C ABI.

The tolerances are not parity bounds but the accuracy targets of the modes:
1e-6 relative for the binary32 M2L (binary32 carries 24 bits; the pair
results are summed in binary64); 1e-4 for the binary32 near field, whose
single terms carry binary32 rounding that the cancellation among near
contributions amplifies (measured below).  Measured on these workloads the
far field differs from the binary64 one by about 1e-7 normwise and by up to
6e-7 relative to the largest value (order 1, field).
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
        gpu_eval_prec(torch, F, gt, q, 3, 3, 7)
    assert e.value.code == F.FMM_EINVAL
    gt.free()


F32_TOL = 1e-4


def _normwise(got, ref):
    ephi = np.linalg.norm(got[0] - ref[0]) / np.linalg.norm(ref[0])
    eE = np.linalg.norm(np.concatenate(got[1:]) - np.concatenate(ref[1:])) / np.linalg.norm(np.concatenate(ref[1:]))
    return ephi, eE


@pytest.mark.parametrize("gen,n,L,theta,p", [
    ("uniform", 20_000, 3, 0.5, 10),
    ("gmix", 30_000, 3, 0.5, 8),
    ("plummer", 20_000, 3, 0.6, 6),
    ("sphere", 12_000, 3, 0.5, 5),
])
def test_f32_near_field_vs_oracle(torch, F, orc, gen, n, L, theta, p):
    """FMM_PREC_F32 (binary32 M2L and near field): the near field alone and the
    whole result against the binary64 oracle within F32_TOL normwise, with
    the error printed; the far field alone equals the mixed mode's bit for
    bit (the same binary32 M2L)."""
    if gen == "sphere":
        x, y, z, q = W.sphere_surface(n, seed=8)
    else:
        x, y, z, q = make(gen, n, seed=8)
    ot = orc.Tree(x, y, z, L, theta)
    gt = gpu_tree(torch, F, x, y, z, L, theta)
    leaves = np.arange(0, 8 ** L, 5)
    s0, perm = ot.start(L), ot.perm()
    pts = np.concatenate([perm[s0[b]:s0[b + 1]] for b in leaves])
    for parts, what in ((1, "near"), (3, "all")):
        ref = [a[pts] for a in ot.evaluate(q, p, parts=parts, leaves=leaves)]
        got = [a[pts] for a in gpu_eval_prec(torch, F, gt, q, p, parts, F.FMM_PREC_F32)]
        ephi, eE = _normwise(got, ref)
        say(f"[f32] {gen} n={n} {what}: phi {ephi:.2e} E {eE:.2e}")
        assert ephi <= F32_TOL and eE <= F32_TOL
    far32 = gpu_eval_prec(torch, F, gt, q, p, 2, F.FMM_PREC_F32)
    farm = gpu_eval_prec(torch, F, gt, q, p, 2, F.FMM_PREC_MIXED)
    for a, b in zip(far32, farm):
        assert np.array_equal(a, b)
    gt.free()


def test_f32_near_field_at_separate_targets_and_coincident_points(torch, F, orc):
    """The binary32 near field at separate targets (grouped by leaf), with
    targets placed on sources (skipped as coincident) and duplicates among
    the sources."""
    x, y, z, q = W.gaussian_mixture(8_000, seed=3)
    x[100:110] = x[0]
    y[100:110] = y[0]
    z[100:110] = z[0]
    tx, ty, tz, _ = W.gaussian_mixture(600, seed=4)
    tx[:50], ty[:50], tz[:50] = x[:50], y[:50], z[:50]
    ot = orc.Tree(x, y, z, 2, 0.5, targets=(tx, ty, tz))
    ref = ot.evaluate_targets(q, 7)
    X = [dev(torch, a) for a in (x, y, z)]
    T = [dev(torch, a) for a in (tx, ty, tz)]
    gt = F.fmm_build_ex(*X, 2, 0.5, targets=tuple(T))
    outs = [torch.empty(600, dtype=torch.float64, device="cuda") for _ in range(4)]
    F.fmm_evaluate_targets(gt, dev(torch, q), 7, *outs, precision=F.FMM_PREC_F32)
    torch.cuda.synchronize()
    got = [o.cpu().numpy() for o in outs]
    ephi, eE = _normwise(got, ref)
    say(f"[f32] targets: phi {ephi:.2e} E {eE:.2e}")
    assert ephi <= F32_TOL and eE <= F32_TOL
    assert all(np.all(np.isfinite(a)) for a in got)
    gt.free()
