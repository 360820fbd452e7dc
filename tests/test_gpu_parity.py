"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Integer work (permutation, point ranges, interaction lists) and the box
geometry must match bit for bit; potentials and fields must match within
FP64_TOL, both normwise and element by element relative to the largest
magnitude of the reference (mixed-sign charges make single values cancel).
"""
import sys

import numpy as np
import pytest

from paper_2002_04894_amd import workloads as W

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as T
    if not T.cuda.is_available():
        pytest.skip("no GPU")
    return T


@pytest.fixture(scope="module")
def F():
    from paper_2002_04894_amd import fmm
    fmm.lib()
    return fmm


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda")


def gpu_tree(torch, F, x, y, z, L, theta):
    return F.fmm_build(dev(torch, x), dev(torch, y), dev(torch, z), L, theta)


def gpu_eval(torch, F, tree, q, p, parts=3):
    qd = dev(torch, q)
    outs = [torch.empty_like(qd) for _ in range(4)]
    F.fmm_evaluate_tree(tree, qd, p, *outs, parts=parts)
    torch.cuda.synchronize()
    return [o.cpu().numpy() for o in outs]


def assert_tree_equal(F, gt, ot, L):
    assert np.array_equal(F.fmm_tree_perm(gt), ot.perm())
    for l in range(L + 1):
        g, s = F.fmm_tree_boxes(gt, l)
        assert np.array_equal(s, ot.start(l)), f"starts level {l}"
        og = ot.geom(l)
        assert np.array_equal(g.view(np.uint64), og.view(np.uint64)), f"geometry level {l}"
        for kind in (0, 1):
            go, gi = F.fmm_tree_lists(gt, l, kind)
            oo, oi = ot.lists(l, kind)
            assert np.array_equal(go, oo) and np.array_equal(gi, oi), f"lists level {l} kind {kind}"


def assert_close(got, ref, tol=FP64_TOL, what=""):
    names = ("phi", "ex", "ey", "ez")
    # potential alone, field as one 3N vector
    pairs = [(got[0], ref[0], "phi"), (np.concatenate(got[1:]), np.concatenate(ref[1:]), "E")]
    for g, r, nm in pairs:
        scale = np.abs(r).max()
        if scale == 0:
            assert np.abs(g).max() == 0, f"{what} {nm}"
            continue
        nrm = np.linalg.norm(g - r) / np.linalg.norm(r)
        ele = np.abs(g - r).max() / scale
        assert nrm <= tol and ele <= tol, f"{what} {nm}: normwise {nrm:.3e} elementwise {ele:.3e}"
    for g, nm in zip(got, names):
        assert np.isfinite(g).all(), f"{what} {nm} not finite"


CASES = [
    # name, generator, n, levels, theta, p
    ("uniform20k", "uniform", 20_000, 3, 0.5, 10),
    ("gmix5k", "gmix", 5_000, 2, 0.5, 8),
    ("plummer3k", "plummer", 3_000, 2, 0.6, 6),
    ("uniform50k_L2_bigleaves", "uniform", 50_000, 2, 0.5, 5),
    ("gmix2k_L0", "gmix", 2_000, 0, 0.5, 4),
    ("uniform3k_theta0", "uniform", 3_000, 2, 0.0, 3),
    ("gmix1500_p0", "gmix", 1_500, 2, 0.5, 0),
    ("uniform1200_p20", "uniform", 1_200, 1, 0.3, 20),
    ("plummer4k_L3_sparse", "plummer", 4_000, 3, 0.45, 7),
    # coordinates on an 8^3 lattice: long runs of equal keys in the medians of
    # the chunked (large-segment) bisection rounds
    ("quantized40k_ties", "quantized", 40_000, 3, 0.5, 4),
]


def make(gen, n, seed=0):
    if gen == "uniform":
        return W.uniform_cube(n, seed=seed)
    if gen == "gmix":
        return W.gaussian_mixture(n, seed=seed)
    if gen == "plummer":
        return W.plummer(n, seed=seed, charges="pm1")
    if gen == "quantized":
        x, y, z, q = W.uniform_cube(n, seed=seed)
        return np.floor(x * 8) / 8 - 0.5, np.floor(y * 8) / 8 - 0.5, np.floor(z * 8) / 8 - 0.5, q
    raise ValueError(gen)


@pytest.mark.parametrize("name,gen,n,L,theta,p", CASES, ids=[c[0] for c in CASES])
def test_parity_full(torch, F, orc, name, gen, n, L, theta, p):
    say(f"[parity] {name}: n={n} L={L} theta={theta} p={p}")
    x, y, z, q = make(gen, n)
    ot = orc.Tree(x, y, z, L, theta)
    gt = gpu_tree(torch, F, x, y, z, L, theta)
    assert_tree_equal(F, gt, ot, L)
    # work counts: weak pairs over all levels; near-field interactions
    n_leaf = np.diff(ot.start(L))
    so, si = ot.lists(L, 0)
    src = np.array([n_leaf[si[so[i]:so[i + 1]]].sum() for i in range(n_leaf.size)], dtype=np.int64)
    m2l_ref = sum(ot.lists(l, 1)[1].size for l in range(1, L + 1))
    assert F.fmm_tree_stats(gt) == (m2l_ref, int((n_leaf * src).sum()) - n)
    for parts, nm in ((1, "near"), (2, "far"), (3, "all")):
        say(f"[parity] {name}: {nm}")
        ref = ot.evaluate(q, p, parts=parts)
        got = gpu_eval(torch, F, gt, q, p, parts=parts)
        assert_close(got, ref, what=f"{name}/{nm}")
    gt.free()


@pytest.mark.parametrize("p", list(range(16)))
def test_parity_far_field_every_mfma_order(torch, F, orc, p):
    """Far field (M2L and the translations) at every order the matrix-core
    M2L takes, on a two-level tree (about 24 weak pairs per leaf: one full
    and one partial batch of 16)."""
    say(f"[orders] p={p}")
    x, y, z, q = make("gmix", 2_000, seed=4)
    ot = orc.Tree(x, y, z, 2, 0.6)
    gt = gpu_tree(torch, F, x, y, z, 2, 0.6)
    ref = ot.evaluate(q, p, parts=2)
    got = gpu_eval(torch, F, gt, q, p, parts=2)
    assert_close(got, ref, what=f"far p={p}")
    gt.free()


EDGE = [
    ("one_point_L0", np.array([[0.3, 0.2, 0.1]]), 0),
    ("one_point_L2", np.array([[0.3, 0.2, 0.1]]), 2),
    ("seven_points_L1", np.random.default_rng(3).random((7, 3)), 1),
    ("five_points_L2", np.random.default_rng(4).random((5, 3)), 2),
    ("duplicates", np.repeat(np.random.default_rng(5).random((4, 3)), 50, axis=0), 2),
    ("all_identical", np.full((33, 3), 0.25), 1),
    ("lattice_ties", np.stack(np.meshgrid(*[np.arange(6.0)] * 3, indexing="ij"), -1).reshape(-1, 3), 2),
    ("negative_zero", np.array([[-0.0, 0.0, 1.0], [0.0, -0.0, 2.0], [1.0, 1.0, -0.0], [0.5, -0.0, 0.5]] * 5), 1),
    ("flat_plane", np.c_[np.random.default_rng(6).random((400, 2)), np.zeros(400)], 2),
    ("far_outlier", np.r_[np.random.default_rng(7).random((500, 3)), [[1e6, -1e6, 1e6]]], 2),
]


@pytest.mark.parametrize("name,P,L", EDGE, ids=[e[0] for e in EDGE])
def test_parity_edge_cases(torch, F, orc, name, P, L):
    say(f"[edge] {name}: n={P.shape[0]} L={L}")
    x, y, z = (np.ascontiguousarray(P[:, k]) for k in range(3))
    q = np.random.default_rng(P.shape[0]).uniform(-1, 1, P.shape[0])
    ot = orc.Tree(x, y, z, L, 0.5)
    gt = gpu_tree(torch, F, x, y, z, L, 0.5)
    assert_tree_equal(F, gt, ot, L)
    ref = ot.evaluate(q, 6)
    got = gpu_eval(torch, F, gt, q, 6)
    assert_close(got, ref, what=name)
    gt.free()


@pytest.mark.parametrize("p", [6, 12])
def test_parity_zero_distance_translations(torch, F, orc, p):
    """A cluster of identical points beside a separated cloud: the cluster's
    boxes have zero extent, so children share their parent's centre and M2M
    and L2L translate by distance zero (the identity) on the matrix-core path,
    while M2L carries those expansions to the cloud.  Checks that such pairs
    and weak pairs exist, then the whole result against the oracle."""
    P = np.r_[np.full((256, 3), 0.25), np.random.default_rng(8).random((768, 3)) + 1.5]
    x, y, z = (np.ascontiguousarray(P[:, k]) for k in range(3))
    q = np.random.default_rng(9).uniform(-1, 1, P.shape[0])
    ot = orc.Tree(x, y, z, 3, 0.5)
    for l in (2, 3):
        g, gp = ot.geom(l), ot.geom(l - 1)
        same = sum(np.array_equal(g[i, 6:9], gp[i >> 3, 6:9]) for i in range(g.shape[0]))
        assert same > 0, f"no child at its parent's centre on level {l}"
        assert ot.lists(l, 1)[1].size > 0
    gt = gpu_tree(torch, F, x, y, z, 3, 0.5)
    assert_tree_equal(F, gt, ot, 3)
    assert_close(gpu_eval(torch, F, gt, q, p), ot.evaluate(q, p), what=f"zero-distance translations p={p}")
    gt.free()


def test_nonfinite_rejected(torch, F):
    say("[edge] nonfinite")
    x, y, z, _ = W.uniform_cube(100, seed=1)
    x[17] = np.nan
    with pytest.raises(F.FMMError) as e:
        gpu_tree(torch, F, x, y, z, 1, 0.5)
    assert e.value.code == F.FMM_EINVAL
    x[17] = np.inf
    with pytest.raises(F.FMMError):
        gpu_tree(torch, F, x, y, z, 1, 0.5)


def test_parts_argument_checked(torch, F):
    x, y, z, q = W.uniform_cube(100, seed=1)
    gt = gpu_tree(torch, F, x, y, z, 1, 0.5)
    qd = dev(torch, q)
    outs = [torch.empty_like(qd) for _ in range(4)]
    with pytest.raises(F.FMMError):
        F.fmm_evaluate_tree(gt, qd, 3, *outs, parts=4)
    gt.free()


def test_deterministic_and_reusable(torch, F):
    say("[det] repeat runs")
    x, y, z, q = W.gaussian_mixture(30_000, seed=2)
    gt = gpu_tree(torch, F, x, y, z, 3, 0.5)
    a = gpu_eval(torch, F, gt, q, 9)
    b = gpu_eval(torch, F, gt, q, 9)
    for u, v in zip(a, b):
        assert np.array_equal(u, v)
    gt2 = gpu_tree(torch, F, x, y, z, 3, 0.5)
    c = gpu_eval(torch, F, gt2, q, 9)
    for u, v in zip(a, c):
        assert np.array_equal(u, v)
    # tree reuse with other charges equals a fresh one-shot evaluation
    q2 = np.random.default_rng(9).uniform(-1, 1, x.shape[0])
    d = gpu_eval(torch, F, gt, q2, 9)
    outs = F.evaluate(dev(torch, x), dev(torch, y), dev(torch, z), dev(torch, q2), 3, 0.5, 9)
    torch.cuda.synchronize()
    for u, v in zip(d, outs):
        assert np.array_equal(u, v.cpu().numpy())
    gt.free()
    gt2.free()


def test_direct_sum_accuracy_uniform20k(torch, F, orc):
    """The uniform 20k workload (3 levels, theta 0.5, p 10) against the
    O(N^2) direct sum of eq. (2.1), all points."""
    say("[accuracy] uniform20k vs direct sum")
    x, y, z, q = W.uniform_cube(20_000, seed=0)
    d = orc.direct(x, y, z, q)
    got = F.evaluate(dev(torch, x), dev(torch, y), dev(torch, z), dev(torch, q), 3, 0.5, 10)
    torch.cuda.synchronize()
    got = [g.cpu().numpy() for g in got]
    ephi = np.linalg.norm(got[0] - d[0]) / np.linalg.norm(d[0])
    eE = np.linalg.norm(np.concatenate(got[1:]) - np.concatenate(d[1:])) / np.linalg.norm(np.concatenate(d[1:]))
    say(f"[accuracy] uniform20k: phi {ephi:.3e} E {eE:.3e}")
    assert ephi <= 1e-6 and eE <= 1e-6


def test_full_size_gmix1m_sampled(torch, F, orc):
    """The 2^20-point Gaussian-mixture workload at full size in the benchmark's
    configuration: tree and lists bit-exact, potentials and fields on every
    point of sampled leaves against the oracle's leaf-subset evaluation, and
    accuracy against the direct sum on sampled targets."""
    x, y, z, q, w = W.workload("gmix1m")
    L, theta, p = w["levels"], w["theta"], w["p"]
    say(f"[full] gmix1m: build n={x.shape[0]} L={L}")
    gt = gpu_tree(torch, F, x, y, z, L, theta)
    ot = orc.Tree(x, y, z, L, theta)
    say("[full] gmix1m: compare tree")
    assert_tree_equal(F, gt, ot, L)
    say("[full] gmix1m: evaluate")
    got = gpu_eval(torch, F, gt, q, p)
    leaves = np.array([0, 4097, 20000, 32767])
    say("[full] gmix1m: oracle on sampled leaves")
    ref = ot.evaluate(q, p, leaves=leaves)
    s = ot.start(L)
    pts = np.concatenate([ot.perm()[s[b]:s[b + 1]] for b in leaves])
    assert_close([g[pts] for g in got], [r[pts] for r in ref], what="gmix1m sampled leaves")
    say("[full] gmix1m: mixed precision")
    qd = dev(torch, q)
    mixed = [torch.empty_like(qd) for _ in range(4)]
    F.fmm_evaluate_tree(gt, qd, p, *mixed, precision=F.FMM_PREC_MIXED)
    torch.cuda.synchronize()
    mixed = [m.cpu().numpy() for m in mixed]
    assert_close([g[pts] for g in mixed], [r[pts] for r in ref], tol=1e-6, what="gmix1m mixed sampled leaves")
    say("[full] gmix1m: direct sum on sampled targets")
    tg = W.sample_targets(x.shape[0], 1000, seed=1)
    d = orc.direct(x, y, z, q, targets=tg)
    dE = np.concatenate(d[1:])
    for res, nm in ((got, "f64"), (mixed, "mixed")):
        ephi = np.linalg.norm(res[0][tg] - d[0]) / np.linalg.norm(d[0])
        gE = np.concatenate([g[tg] for g in res[1:]])
        eE = np.linalg.norm(gE - dE) / np.linalg.norm(dE)
        say(f"[full] gmix1m {nm}: err vs direct phi {ephi:.3e} E {eE:.3e}")
        assert ephi <= 1e-6 and eE <= 1e-6
    gt.free()


@pytest.mark.parametrize("p,L", [(16, 2), (17, 2), (18, 2), (19, 2), (20, 2)])
def test_parity_binary64_orders_16_to_20(torch, F, orc, p, L):
    """Orders above 15 run M2L four lanes per pair in binary64 (one wave per
    SIMD, J and its transpose from one table): with weak pairs, M2M and L2L
    against the oracle."""
    say(f"[quad] p={p} L={L}")
    x, y, z, q = make("gmix", 3000, seed=p)
    ot = orc.Tree(x, y, z, L, 0.5)
    assert ot.lists(L, 1)[1].size > 0
    gt = gpu_tree(torch, F, x, y, z, L, 0.5)
    assert_close(gpu_eval(torch, F, gt, q, p), ot.evaluate(q, p), what=f"p={p} L={L}")
    gt.free()


@pytest.mark.parametrize("k", [-40, 40])
def test_power_of_two_scale_covariance(torch, F, k):
    """Scaling every coordinate by 2^k scales phi by 2^-k and E by 2^-2k (1/r
    is homogeneous of degree -1).  Every step of the path is homogeneous under
    power-of-two scaling too: the bisections and box geometry, the theta
    test, the harmonics, the radius-scaled M2L, the M2M and L2L on the matrix
    cores (distance powers split into a power of a mantissa in [1, 2) and an
    exact power of two) and the near field; so the lists are equal and the
    results agree to rounding.  Binary64 and mixed precision, orders 8 and 13,
    a 3-level tree; a property test that holds at any size, with no oracle."""
    x, y, z, q = make("gmix", 6_000, seed=11)
    s = 2.0 ** k
    t1 = gpu_tree(torch, F, x, y, z, 3, 0.5)
    ts = gpu_tree(torch, F, x * s, y * s, z * s, 3, 0.5)
    for l in range(4):
        for kind in (0, 1):
            a, b = F.fmm_tree_lists(t1, l, kind), F.fmm_tree_lists(ts, l, kind)
            assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]), f"lists level {l} kind {kind}"
    qd = dev(torch, q)
    for p in (8, 13):
        for prec in (F.FMM_PREC_F64, F.FMM_PREC_MIXED):
            say(f"[scale] 2^{k}: p={p} precision={prec}")
            res = []
            for tr in (t1, ts):
                outs = [torch.empty_like(qd) for _ in range(4)]
                F.fmm_evaluate_tree(tr, qd, p, *outs, precision=prec)
                torch.cuda.synchronize()
                res.append([o.cpu().numpy() for o in outs])
            want = [res[0][0] / s] + [e / (s * s) for e in res[0][1:]]
            assert_close(res[1], want, what=f"scale 2^{k} p={p} precision={prec}")
    t1.free()
    ts.free()


@pytest.mark.parametrize("n,L", [(8192, 2), (8300, 3), (12000, 2), (16383, 2)])
def test_parity_sizes_with_one_chunked_round(torch, F, orc, n, L):
    """8192 <= n < 16384 source points: only the first bisection round (one
    segment of n points) runs as chunked blocks.  Its state must be allocated
    for that round too (it once was not, and such builds took a GPU memory
    fault); tree bit for bit and values against the oracle."""
    say(f"[sizes] uniform n={n} L={L}")
    x, y, z, q = W.uniform_cube(n, seed=n)
    ot = orc.Tree(x, y, z, L, 0.5)
    gt = gpu_tree(torch, F, x, y, z, L, 0.5)
    assert_tree_equal(F, gt, ot, L)
    assert_close(gpu_eval(torch, F, gt, q, 4), ot.evaluate(q, 4), what=f"n={n}")
    gt.free()


@pytest.mark.parametrize("p", [16, 19])
def test_parity_first_use_on_side_stream(torch, F, orc, p):
    """Orders that no other test here evaluates, so that their operator
    tables are made during this call, whose work runs on a non-blocking
    stream (no ordering with the null stream): the tables must be complete on
    the device before that stream reads them.  Also the binary64 path above
    order 15 with weak pairs, M2M and L2L (two levels), against the oracle."""
    say(f"[side stream] first use of p={p}")
    x, y, z, q = make("gmix", 3000, seed=4)
    ot = orc.Tree(x, y, z, 2, 0.5)
    assert ot.lists(2, 1)[1].size > 0  # weak pairs on level 2
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        gt = F.fmm_build(dev(torch, x), dev(torch, y), dev(torch, z), 2, 0.5, s)
        qd = dev(torch, q)
        outs = [torch.empty_like(qd) for _ in range(4)]
        F.fmm_evaluate_tree(gt, qd, p, *outs, s)
        got = [o.cpu().numpy() for o in outs]
        gt.free()
    s.synchronize()
    assert_close(got, ot.evaluate(q, p), what=f"side stream p={p}")


def test_threads_on_own_streams_match_serial(torch, F):
    """Host threads, each with its own non-blocking stream, build and evaluate
    at the same time (orders on both sides of the MFMA limit, both
    precisions): every result equals the same call made alone."""
    import threading
    say("[threads] 6 threads x 3 solves")
    jobs = []  # (generator, n, levels, p, precision, seed)
    for k in range(18):
        gen = ("uniform", "gmix", "plummer")[k % 3]
        p = (5, 9, 17, 20, 11, 3)[k % 6]
        prec = F.FMM_PREC_MIXED if (k % 2 and p <= 15) else F.FMM_PREC_F64
        jobs.append((gen, 2000 + 700 * k, 2 + k % 2, p, prec, 100 + k))

    def solve(job, stream):
        gen, n, L, p, prec, seed = job
        x, y, z, q = make(gen, n, seed=seed)
        with torch.cuda.stream(stream):
            d = [dev(torch, a) for a in (x, y, z, q)]
            outs = [torch.empty_like(d[0]) for _ in range(4)]
            t = F.fmm_build(d[0], d[1], d[2], L, 0.5, stream)
            F.fmm_evaluate_tree(t, d[3], p, *outs, stream, precision=prec)
            res = [o.cpu().numpy() for o in outs]
            t.free()
        return res

    serial_stream = torch.cuda.Stream()
    serial = [solve(j, serial_stream) for j in jobs]
    results = [None] * len(jobs)
    errors = []

    def worker(w):
        st = torch.cuda.Stream()
        try:
            for i in range(w, len(jobs), 6):
                results[i] = solve(jobs[i], st)
        except Exception as exc:  # reported below
            errors.append(repr(exc))

    threads = [threading.Thread(target=worker, args=(w,)) for w in range(6)]
    for th in threads:
        th.start()
    for th in threads:
        th.join()
    assert not errors, errors
    for i, (a, b) in enumerate(zip(serial, results)):
        for u, v in zip(a, b):
            assert np.array_equal(u, v), f"job {i} {jobs[i]}"
