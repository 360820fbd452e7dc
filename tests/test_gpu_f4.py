"""eta-blended splits (Section 2.1.2) and evaluation at separate targets
(the convergence test of Section 3.1) on the GPU, through the C ABI, against
the oracle: trees, lists and target leaves bit for bit, potentials and fields
within FP64_TOL (FMM_PREC_MIXED within 1e-6)."""
import numpy as np
import pytest

from paper_2002_04894_amd import workloads as W
from test_gpu_parity import (FP64_TOL, F, assert_close, assert_tree_equal, dev, make, say,  # noqa: F401
                             torch)

pytestmark = pytest.mark.gpu


def targets_for(x, y, z, m, seed):
    """Random targets over a box a little wider than the sources', three of
    them exactly on sources."""
    tx, ty, tz, _ = W.uniform_cube(m, seed=seed)
    lo = np.array([x.min(), y.min(), z.min()]); hi = np.array([x.max(), y.max(), z.max()])
    w = hi - lo
    tx, ty, tz = lo[0] - 0.1 * w[0] + 1.2 * w[0] * tx, lo[1] - 0.1 * w[1] + 1.2 * w[1] * ty, lo[2] + w[2] * tz
    tx[:3], ty[:3], tz[:3] = x[:3], y[:3], z[:3]
    return tx, ty, tz


def gpu_build(torch, F, x, y, z, L, theta, eta, targets=None):
    tg = None if targets is None else tuple(dev(torch, a) for a in targets)
    return F.fmm_build_ex(dev(torch, x), dev(torch, y), dev(torch, z), L, theta, eta=eta, targets=tg)


def gpu_eval_targets(torch, F, tree, q, p, parts=3, precision=0):
    qd = dev(torch, q)
    outs = [torch.empty(tree.m, dtype=torch.float64, device="cuda") for _ in range(4)]
    F.fmm_evaluate_targets(tree, qd, p, *outs, parts=parts, precision=precision)
    torch.cuda.synchronize()
    return [o.cpu().numpy() for o in outs]


def gpu_eval(torch, F, tree, q, p, parts=3):
    qd = dev(torch, q)
    outs = [torch.empty_like(qd) for _ in range(4)]
    F.fmm_evaluate_tree(tree, qd, p, *outs, parts=parts)
    torch.cuda.synchronize()
    return [o.cpu().numpy() for o in outs]


ETA_CASES = [
    # generator, n, levels, theta, eta, p
    ("uniform", 3000, 2, 0.5, 0.0, 6),
    ("gmix", 3000, 2, 0.5, 0.5, 6),
    ("plummer", 4000, 3, 0.5, 0.25, 5),
    ("gmix", 20_000, 3, 0.5, 0.75, 8),
    ("plummer", 2000, 3, 0.6, 0.0, 4),     # eta 0 on clustered data: many empty leaves
]


@pytest.mark.parametrize("gen,n,L,theta,eta,p", ETA_CASES, ids=[f"{c[0]}{c[1]}_L{c[2]}_eta{c[4]}" for c in ETA_CASES])
def test_eta_tree_and_evaluation(torch, F, orc, gen, n, L, theta, eta, p):
    say(f"[eta] {gen} n={n} L={L} eta={eta} p={p}")
    x, y, z, q = make(gen, n, seed=11)
    ot = orc.Tree(x, y, z, L, theta, eta=eta)
    gt = gpu_build(torch, F, x, y, z, L, theta, eta)
    assert_tree_equal(F, gt, ot, L)
    assert_close(gpu_eval(torch, F, gt, q, p), ot.evaluate(q, p), what=f"eta {eta}")
    gt.free()


def test_eta_large_chunked_rounds(torch, F, orc):
    """eta < 1 over 2^18 points: the first rounds run chunked on segments of
    unequal size (read back per round), the later ones one block per
    segment: tree bit for bit, values on sampled leaves."""
    x, y, z, q = W.gaussian_mixture(1 << 18, seed=3)
    L, theta, eta, p = 4, 0.5, 0.5, 8
    say(f"[eta] gmix 2^18 L={L} eta={eta}")
    ot = orc.Tree(x, y, z, L, theta, eta=eta)
    gt = gpu_build(torch, F, x, y, z, L, theta, eta)
    assert_tree_equal(F, gt, ot, L)
    got = gpu_eval(torch, F, gt, q, p)
    leaves = np.array([0, 1000, 2047, 4095])
    ref = ot.evaluate(q, p, leaves=leaves)
    s = ot.start(L)
    pts = np.concatenate([ot.perm()[s[b]:s[b + 1]] for b in leaves])
    assert_close([g[pts] for g in got], [r[pts] for r in ref], what="eta 0.5 sampled leaves")
    gt.free()


CHUNKED_ETA_CASES = [
    # generator, n, levels, eta: unequal segments of at least 8192 points in
    # the first rounds (chunked), then one block per segment
    ("gaussian_mixture", 60_000, 2, 0.3),
    ("spherical_gaussian", 100_000, 2, 0.0),
    ("helix", 50_000, 2, 0.8),
    ("uniform_cube", 70_000, 2, 0.5),
]


@pytest.mark.parametrize("gen,n,L,eta", CHUNKED_ETA_CASES, ids=[f"{c[0]}{c[1]}_eta{c[3]}" for c in CHUNKED_ETA_CASES])
def test_eta_chunked_rounds_unequal_segments(torch, F, orc, gen, n, L, eta):
    say(f"[eta] chunked {gen} n={n} L={L} eta={eta}")
    x, y, z, q = getattr(W, gen)(n, seed=9)
    ot = orc.Tree(x, y, z, L, 0.5, eta=eta)
    gt = gpu_build(torch, F, x, y, z, L, 0.5, eta)
    assert_tree_equal(F, gt, ot, L)
    gt.free()


TARGET_CASES = [
    # generator, n, m, levels, theta, eta, p
    ("uniform", 2000, 500, 2, 0.5, 1.0, 6),
    ("gmix", 2500, 700, 2, 0.5, 0.5, 7),
    ("plummer", 3000, 300, 3, 0.5, 0.0, 4),
    ("gmix", 30_000, 20_000, 3, 0.5, 1.0, 10),
]


@pytest.mark.parametrize("gen,n,m,L,theta,eta,p", TARGET_CASES,
                         ids=[f"{c[0]}{c[1]}_m{c[2]}_L{c[3]}_eta{c[5]}" for c in TARGET_CASES])
def test_targets_parity(torch, F, orc, gen, n, m, L, theta, eta, p):
    say(f"[targets] {gen} n={n} m={m} L={L} eta={eta} p={p}")
    x, y, z, q = make(gen, n, seed=12)
    tx, ty, tz = targets_for(x, y, z, m, seed=13)
    ot = orc.Tree(x, y, z, L, theta, eta=eta, targets=(tx, ty, tz))
    gt = gpu_build(torch, F, x, y, z, L, theta, eta, targets=(tx, ty, tz))
    assert_tree_equal(F, gt, ot, L)
    leaf = F.fmm_tree_targets(gt)
    assert np.array_equal(leaf, [ot.locate(tx[k], ty[k], tz[k]) for k in range(m)])
    for parts in (1, 2, 3):
        got = gpu_eval_targets(torch, F, gt, q, p, parts=parts)
        assert_close(got, ot.evaluate_targets(q, p, parts=parts), what=f"targets parts={parts}")
    mixed = gpu_eval_targets(torch, F, gt, q, p, precision=F.FMM_PREC_MIXED)
    assert_close(mixed, ot.evaluate_targets(q, p), tol=1e-6, what="targets mixed")
    gt.free()


def test_targets_equal_to_sources_bitwise(torch, F):
    """Targets at the sources' own positions give the source evaluation bit
    for bit (same leaves, lists and kernels)."""
    x, y, z, q = W.uniform_cube(5000, seed=14)
    gt = gpu_build(torch, F, x, y, z, 2, 0.5, 1.0, targets=(x, y, z))
    a = gpu_eval(torch, F, gt, q, 7)
    b = gpu_eval_targets(torch, F, gt, q, 7)
    for u, v in zip(a, b):
        assert np.array_equal(u, v)
    gt.free()


def test_targets_accuracy_vs_direct_sum(torch, F, orc):
    """20k sources, 5000 separate random targets, p = 10: the error against
    the direct sum at the targets (a zero-level tree) is below 1e-6."""
    x, y, z, q = W.uniform_cube(20_000, seed=15)
    tx, ty, tz, _ = W.uniform_cube(5000, seed=16)
    gt = gpu_build(torch, F, x, y, z, 3, 0.5, 1.0, targets=(tx, ty, tz))
    got = gpu_eval_targets(torch, F, gt, q, 10)
    d = orc.Tree(x, y, z, 0, 0.5, targets=(tx, ty, tz)).evaluate_targets(q, 0)
    ephi = np.linalg.norm(got[0] - d[0]) / np.linalg.norm(d[0])
    eE = np.linalg.norm(np.concatenate(got[1:]) - np.concatenate(d[1:])) / np.linalg.norm(np.concatenate(d[1:]))
    say(f"[targets] accuracy phi {ephi:.2e} E {eE:.2e}")
    assert ephi < 1e-6 and eE < 1e-6
    gt.free()


def test_f4_argument_checks(torch, F):
    x, y, z, q = W.uniform_cube(300, seed=1)
    with pytest.raises(F.FMMError) as e:
        gpu_build(torch, F, x, y, z, 1, 0.5, 1.5)
    assert e.value.code == F.FMM_EINVAL
    bad = np.array([0.5, np.nan]), np.array([0.5, 0.5]), np.array([0.5, 0.5])
    with pytest.raises(F.FMMError) as e:
        gpu_build(torch, F, x, y, z, 1, 0.5, 1.0, targets=bad)
    assert e.value.code == F.FMM_EINVAL
    # no targets: evaluation at targets does nothing
    gt = gpu_build(torch, F, x, y, z, 1, 0.5, 1.0)
    assert gt.m == 0 and F.fmm_tree_targets(gt).shape == (0,)
    gpu_eval_targets(torch, F, gt, q, 3)
    gt.free()


def test_targets_zero_levels_and_faces(torch, F, orc):
    """Targets at L = 0 (all P2P), and targets placed exactly on the shared
    faces, edges and corners of leaf cells, where several cells contain them:
    the leaf chosen and the values match the oracle."""
    x, y, z, q = W.gaussian_mixture(3000, seed=21)
    # L = 0: one leaf, the direct sum at the targets
    tx, ty, tz = targets_for(x, y, z, 200, seed=22)
    ot = orc.Tree(x, y, z, 0, 0.5, targets=(tx, ty, tz))
    gt = gpu_build(torch, F, x, y, z, 0, 0.5, 1.0, targets=(tx, ty, tz))
    assert_close(gpu_eval_targets(torch, F, gt, q, 3), ot.evaluate_targets(q, 3), what="targets L=0")
    gt.free()
    # cell corners and face centres of the leaves of a 2-level tree (their
    # geometry does not depend on the targets as long as they lie inside the
    # sources' bounding box)
    g = orc.Tree(x, y, z, 2, 0.5).geom(2)
    pts = np.concatenate([g[:, 0:3], g[:, 3:6], np.c_[g[:, 0], g[:, 7], g[:, 8]], np.c_[g[:, 6], g[:, 4], g[:, 8]]])
    tx, ty, tz = (np.ascontiguousarray(pts[:, k]) for k in range(3))
    ot = orc.Tree(x, y, z, 2, 0.5, targets=(tx, ty, tz))
    assert np.array_equal(ot.geom(2), g)
    gt = gpu_build(torch, F, x, y, z, 2, 0.5, 1.0, targets=(tx, ty, tz))
    assert np.array_equal(F.fmm_tree_targets(gt), [ot.locate(*v) for v in pts])
    assert_close(gpu_eval_targets(torch, F, gt, q, 6), ot.evaluate_targets(q, 6), what="targets on faces")
    gt.free()
