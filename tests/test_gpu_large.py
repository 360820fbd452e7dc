"""The 2^24-point Plummer workload (scale radius 0.05, 6 levels) at full
size, checked through properties that hold at any size: every leaf holds the
number of points that repeated floor(n/2) splits give, the permutation is
complete, every point lies in its leaf's cell, and both precisions are within
1e-6 of the direct sum (eq. (2.1)) at 10,000 sampled points.  The direct sum
runs on the GPU as a theta = 0 evaluation at separate targets (all P2P, the
path the parity tests check against the oracle).  Over theta x p, the values
on sampled leaves are also compared with the oracle's, stored by a script
that runs the oracle alone."""
import json
import math
import os

import numpy as np
import pytest

from paper_2002_04894_amd import workloads as W
from test_gpu_parity import FP64_TOL, F, assert_close, dev, say, torch  # noqa: F401 (fixtures)

pytestmark = pytest.mark.gpu


def median_counts(n: int, levels: int) -> np.ndarray:
    """Leaf sizes of 3 * levels rounds of median bisection (low side floor(c/2))."""
    c = np.array([n], dtype=np.int64)
    for _ in range(3 * levels):
        low = c // 2
        c = np.stack([low, c - low], axis=1).reshape(-1)
    return c


def test_median_counts_closed_form():
    assert list(median_counts(5, 1)) == [0, 1, 0, 1, 0, 1, 1, 1]
    assert median_counts(1 << 24, 6).min() == median_counts(1 << 24, 6).max() == 64


def direct_at(torch, F, X, Y, Z, Q, idx):
    T = [a.index_select(0, idx).contiguous() for a in (X, Y, Z)]
    tree = F.fmm_build_ex(X, Y, Z, 2, 0.0, targets=tuple(T))
    d = [torch.empty(idx.numel(), dtype=torch.float64, device="cuda") for _ in range(4)]
    F.fmm_evaluate_targets(tree, Q, 0, *d)
    torch.cuda.synchronize()
    tree.free()
    return [a.cpu().numpy() for a in d]


def rel(g, d):
    ephi = np.linalg.norm(g[0] - d[0]) / np.linalg.norm(d[0])
    eE = np.linalg.norm(np.concatenate(g[1:]) - np.concatenate(d[1:])) / np.linalg.norm(np.concatenate(d[1:]))
    return ephi, eE


def test_plummer16m_full_size(torch, F):
    x, y, z, q, w = W.workload("plummer16m")
    n, L, theta, p = x.shape[0], w["levels"], w["theta"], w["p"]
    say(f"[large] plummer16m: n={n} L={L} theta={theta} p={p}")
    X, Y, Z, Q = (dev(torch, a) for a in (x, y, z, q))
    gt = F.fmm_build(X, Y, Z, L, theta)
    perm = F.fmm_tree_perm(gt)
    assert np.array_equal(np.sort(perm), np.arange(n, dtype=np.int32))
    geom, start = F.fmm_tree_boxes(gt, L)
    counts = np.diff(start)
    assert np.array_equal(counts, median_counts(n, L))
    leaf = np.repeat(np.arange(8 ** L), counts)
    P = np.stack([x[perm], y[perm], z[perm]], axis=1)
    assert np.all(P >= geom[leaf, 0:3]) and np.all(P <= geom[leaf, 3:6])
    del P, leaf
    say("[large] evaluate binary64 and mixed")
    outs = {}
    for prec in (F.FMM_PREC_F64, F.FMM_PREC_MIXED):
        o = [torch.empty_like(X) for _ in range(4)]
        F.fmm_evaluate_tree(gt, Q, p, *o, precision=prec)
        torch.cuda.synchronize()
        outs[prec] = o
    gt.free()
    tg = W.sample_targets(n, 10_000, seed=1)
    idx = torch.from_numpy(tg).to("cuda")
    say("[large] direct sum at 10,000 sampled points")
    d = direct_at(torch, F, X, Y, Z, Q, idx)
    for prec, o in outs.items():
        g = [a.index_select(0, idx).cpu().numpy() for a in o]
        ephi, eE = rel(g, d)
        say(f"[large] precision {prec}: phi {ephi:.2e} E {eE:.2e}")
        assert ephi <= 1e-6 and eE <= 1e-6
    # mixed against binary64 over all points
    a = [t.cpu().numpy() for t in outs[F.FMM_PREC_F64]]
    b = [t.cpu().numpy() for t in outs[F.FMM_PREC_MIXED]]
    dphi, dE = rel(b, a)
    assert dphi <= 1e-6 and dE <= 1e-6


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "plummer16m_grid.json")


@pytest.fixture(scope="module")
def plummer16m(torch, F):
    """The workload on the device, 10,000 sampled indices, the direct sum
    there, and the oracle's stored grid values by theta."""
    x, y, z, q, w = W.workload("plummer16m")
    n = x.shape[0]
    X, Y, Z, Q = (dev(torch, a) for a in (x, y, z, q))
    tg = W.sample_targets(n, 10_000, seed=1)
    idx = torch.from_numpy(tg).to("cuda")
    d = direct_at(torch, F, X, Y, Z, Q, idx)
    with open(GOLDEN) as f:
        golden = {row["theta"]: row for row in json.load(f)["grid"]}
    return X, Y, Z, Q, w["levels"], idx, d, golden


@pytest.mark.parametrize("theta", (0.4, 0.5, 0.6))
def test_plummer16m_theta_p_grid(torch, F, plummer16m, theta):
    """The clustered-cloud grid: theta in {0.4, 0.5, 0.6} x p in {8, 12, 16},
    binary64 and (p <= 15) mixed precision.  Against the oracle's values on
    sampled leaves (tests/golden/plummer16m_grid.json, written by the oracle
    alone): binary64 within FP64_TOL, mixed within 1e-6.  Errors against the
    direct sum at 10,000 sampled points are printed; the error falls with p
    at fixed theta, and p 12 reaches 1e-6 at theta 0.5."""
    X, Y, Z, Q, L, idx, d, golden = plummer16m
    o = [torch.empty_like(X) for _ in range(4)]

    def run(gt, p, prec):
        F.fmm_evaluate_tree(gt, Q, p, *o, precision=prec)
        torch.cuda.synchronize()
        return [a.index_select(0, idx).cpu().numpy() for a in o]

    gt = F.fmm_build(X, Y, Z, L, theta)
    gold = golden[theta]
    gidx = torch.tensor(gold["index"], dtype=torch.int64, device="cuda")
    errs = {}
    for p in (8, 12, 16):
        g64 = run(gt, p, F.FMM_PREC_F64)
        ref = [np.array(gold["orders"][str(p)][k]) for k in ("phi", "ex", "ey", "ez")]
        at = [a.index_select(0, gidx).cpu().numpy() for a in o]
        assert_close(at, ref, what=f"plummer16m theta {theta} p {p} vs oracle")
        errs[p] = max(rel(g64, d))
        line = f"[grid] theta {theta} p {p}: binary64 {errs[p]:.2e}"
        if p <= 15:
            g32 = run(gt, p, F.FMM_PREC_MIXED)
            at32 = [a.index_select(0, gidx).cpu().numpy() for a in o]
            assert_close(at32, ref, tol=1e-6, what=f"plummer16m theta {theta} p {p} mixed vs oracle")
            line += f" mixed {max(rel(g32, d)):.2e} mixed-vs-f64 {max(rel(g32, g64)):.2e}"
            assert max(rel(g32, g64)) <= 1e-6
        say(line)
    ps = sorted(errs)
    assert all(errs[a] > errs[b] for a, b in zip(ps, ps[1:]))
    if theta == 0.5:
        assert errs[12] <= 1e-6
    gt.free()


def test_plummer134m_full_size(torch, F):
    """The 2^27-point Plummer workload (scale radius 0.02, charges in [-1, 1],
    7 levels) at full size, theta 0.5, p 12, through properties that hold at
    any size: leaf counts against the closed form, a complete permutation,
    both precisions within 1e-6 of the direct sum at 10,000 sampled points,
    and mixed precision within 1e-6 of binary64 over all points.  (The
    oracle's lists alone would take about 90 GB of host memory at this size.)"""
    x, y, z, q, w = W.workload("plummer134m")
    n, L, theta, p = x.shape[0], w["levels"], w["theta"], w["p"]
    say(f"[large] plummer134m: n={n} L={L} theta={theta} p={p}")
    X, Y, Z, Q = (dev(torch, a) for a in (x, y, z, q))
    del x, y, z, q
    gt = F.fmm_build(X, Y, Z, L, theta)
    perm = F.fmm_tree_perm(gt)
    assert np.all(np.bincount(perm, minlength=n) == 1)
    del perm
    _, start = F.fmm_tree_boxes(gt, L)
    assert np.array_equal(np.diff(start), median_counts(n, L))
    tg = W.sample_targets(n, 10_000, seed=1)
    idx = torch.from_numpy(tg).to("cuda")
    outs = {}
    for prec in (F.FMM_PREC_F64, F.FMM_PREC_MIXED):
        say(f"[large] plummer134m: evaluate precision {prec}")
        o = [torch.empty_like(X) for _ in range(4)]
        F.fmm_evaluate_tree(gt, Q, p, *o, precision=prec)
        torch.cuda.synchronize()
        outs[prec] = o
    gt.free()
    a, b = outs[F.FMM_PREC_F64], outs[F.FMM_PREC_MIXED]
    dphi = float(torch.linalg.norm(b[0] - a[0]) / torch.linalg.norm(a[0]))
    dE = math.sqrt(sum(float(torch.sum((u - v) ** 2)) for u, v in zip(b[1:], a[1:])) /
                   sum(float(torch.sum(v ** 2)) for v in a[1:]))
    say(f"[large] plummer134m mixed vs binary64: phi {dphi:.2e} E {dE:.2e}")
    assert dphi <= 1e-6 and dE <= 1e-6
    got = {prec: [t.index_select(0, idx).cpu().numpy() for t in o] for prec, o in outs.items()}
    del outs, a, b
    say("[large] plummer134m: direct sum at 10,000 sampled points")
    d = direct_at(torch, F, X, Y, Z, Q, idx)
    for prec, g in got.items():
        ephi, eE = rel(g, d)
        say(f"[large] plummer134m precision {prec}: phi {ephi:.2e} E {eE:.2e}")
        assert ephi <= 1e-6 and eE <= 1e-6


GOLDEN134 = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "plummer134m_leaves.json")


@pytest.fixture(scope="module")
def plummer134m(torch, F):
    """The 2^27-point workload on the device and the oracle's stored values
    at every point of five sampled leaves (targeted-mode oracle)."""
    x, y, z, q, w = W.workload("plummer134m")
    X, Y, Z, Q = (dev(torch, a) for a in (x, y, z, q))
    del x, y, z, q
    with open(GOLDEN134) as f:
        gold = json.load(f)
    return X, Y, Z, Q, w["levels"], gold


@pytest.mark.parametrize("k", range(4))
def test_plummer134m_sampled_leaves_match_the_oracle(torch, F, plummer134m, k):
    """Oracle parity at the largest one-GPU size: the sampled leaves' point
    ranges, point sets and cells bit for bit, and binary64 potential and field
    at all their points within FP64_TOL of the oracle (which ran the whole
    method along the chains of these leaves, tests/golden/make_plummer134m_leaves.py),
    mixed precision within 1e-6."""
    X, Y, Z, Q, L, gold = plummer134m
    st = gold["settings"][k]
    theta, p = st["theta"], st["p"]
    say(f"[large] plummer134m vs oracle: theta {theta} p {p}")
    gt = F.fmm_build(X, Y, Z, L, theta)
    leaves = gold["leaves"]
    geom, start = F.fmm_tree_boxes(gt, L)
    perm = F.fmm_tree_perm(gt)
    for b, s0, pts, cell in zip(leaves, gold["start"], gold["points"], gold["cell_hex"]):
        assert start[b] == s0
        assert np.array_equal(perm[start[b]:start[b + 1]], np.array(pts, dtype=np.int32))
        assert [float(v).hex() for v in geom[b]] == cell
    del perm
    idx = torch.tensor(np.concatenate([np.array(a) for a in gold["points"]]), dtype=torch.int64, device="cuda")
    ref = [np.array(st[c]) for c in ("phi", "ex", "ey", "ez")]
    o = [torch.empty_like(X) for _ in range(4)]
    for prec, tol in ((F.FMM_PREC_F64, FP64_TOL), (F.FMM_PREC_MIXED, 1e-6)):
        F.fmm_evaluate_tree(gt, Q, p, *o, precision=prec)
        torch.cuda.synchronize()
        at = [a.index_select(0, idx).cpu().numpy() for a in o]
        assert_close(at, ref, tol=tol, what=f"plummer134m theta {theta} p {p} precision {prec} vs oracle")
    gt.free()
