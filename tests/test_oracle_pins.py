"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: closed forms
(golden fixtures), high-precision brute force (mpmath), textbook identities of
polynomial interpolation, and structural invariants of Alg. 1.  Together they
are meant to catch a dropped term, a wrong sign, a wrong index or a transposed
operand anywhere in the oracle.
"""
import math

import mpmath as mp
import numpy as np
import pytest

import oracle
from paper_2003_01836_amd import inputs
from tests.conftest import read_golden

mp.mp.dps = 40


# --------------------------------------------------------------------------
# Chebyshev points and barycentric weights, eqs. (6)-(7)
# --------------------------------------------------------------------------
def test_chebyshev_golden_n4():
    rows = read_golden("chebyshev_n4.txt")
    s, w = oracle.chebyshev(4)
    for k, sk, wk in rows:
        assert abs(s[int(k)] - sk) <= 1e-15
        assert w[int(k)] == wk


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8, 13])
def test_chebyshev_points_are_extrema_of_T_n(n):
    # the 2nd-kind points are where T_n reaches +-1: T_n(s_k) = (-1)^k
    s, _ = oracle.chebyshev(n)
    coef = np.zeros(n + 1)
    coef[n] = 1.0
    vals = np.polynomial.chebyshev.chebval(s, coef)
    assert np.allclose(vals, [(-1.0) ** k for k in range(n + 1)], atol=1e-13)
    assert s[0] == 1.0 and abs(s[n] + 1.0) < 1e-15


def test_chebyshev_linear_map():
    a, b = -0.3, 1.7
    s, w = oracle.chebyshev(6, a, b)
    s0, w0 = oracle.chebyshev(6)
    assert np.allclose(s, (a + b) / 2 + (b - a) / 2 * s0, atol=1e-15)
    assert np.array_equal(w, w0)        # weights unchanged by the map (Sec. II-A)
    assert abs(s[0] - b) < 1e-15 and abs(s[6] - a) < 1e-15


@pytest.mark.parametrize("n", [1, 2, 4, 7, 10])
def test_weights_match_product_form(n):
    # eq. (4): w_k = 1/prod_{j != k}(s_k - s_j); eq. (7) equals it up to one common factor
    s, w = oracle.chebyshev(n)
    sm = [mp.cos(mp.pi * k / n) for k in range(n + 1)]
    prod = []
    for k in range(n + 1):
        p = mp.mpf(1)
        for j in range(n + 1):
            if j != k:
                p *= sm[k] - sm[j]
        prod.append(1 / p)
    ratio = [float(prod[k] / w[k]) for k in range(n + 1)]
    assert np.allclose(ratio, ratio[0], rtol=1e-13)


# --------------------------------------------------------------------------
# Barycentric Lagrange basis, eqs. (3)-(5)
# --------------------------------------------------------------------------
def _lagrange_product_form(sm, k, x):
    x = mp.mpf(x)
    v = mp.mpf(1)
    for j in range(len(sm)):
        if j != k:
            v *= (x - sm[j]) / (sm[k] - sm[j])
    return v


@pytest.mark.parametrize("n", [1, 3, 6, 9, 12])
def test_lagrange_matches_product_form(n):
    a, b = -0.7, 0.4
    s, w = oracle.chebyshev(n, a, b)
    sm = [mp.mpf(v) for v in s]          # the oracle's own nodes, exactly
    g = np.random.default_rng(n)
    for x in np.concatenate([g.uniform(a, b, 6), [a - 0.1, b + 0.05]]):
        L = oracle.lagrange(n, s, w, x)
        ref = [float(_lagrange_product_form(sm, k, x)) for k in range(n + 1)]
        assert np.allclose(L, ref, rtol=1e-11, atol=1e-13)
        assert abs(L.sum() - 1.0) < 1e-13          # partition of unity


def test_lagrange_removable_singularity():
    n = 5
    s, w = oracle.chebyshev(n, 0.1, 0.9)
    for j in range(n + 1):
        L = oracle.lagrange(n, s, w, s[j])
        assert np.array_equal(L, np.eye(n + 1)[j])           # eq. (5), exact
        # a subnormal offset is still "coincident" (tolerance DBL_MIN, Sec. II-C)
        L = oracle.lagrange(n, s, w, s[j] + 1e-310 if s[j] == 0 else s[j])
        assert np.array_equal(L, np.eye(n + 1)[j])
    # zero node with a subnormal offset
    s0, w0 = oracle.chebyshev(2)
    assert s0[1] == pytest.approx(0.0, abs=1e-16)
    z = np.array([1.0, 0.0, -1.0])
    L = oracle.lagrange(2, z, w0, 5e-324)
    assert np.array_equal(L, [0.0, 1.0, 0.0])
    # just above the tolerance the barycentric formula is used and is still ~one-hot
    L = oracle.lagrange(2, z, w0, 1e-300)
    assert np.allclose(L, [0.0, 1.0, 0.0], atol=1e-15)


# --------------------------------------------------------------------------
# Direct sum, eqs. (1)-(2)
# --------------------------------------------------------------------------
def test_direct_cube_corners_golden():
    corners = np.array([[i, j, k] for i in (0, 1) for j in (0, 1) for k in (0, 1)], dtype=float)
    q = np.ones(8)
    for kappa, phi_ref in read_golden("cube_corners.txt"):
        kern = oracle.COULOMB if kappa == 0 else oracle.YUKAWA
        phi = oracle.direct(corners, corners, q, kernel=kern, kappa=kappa)
        assert np.allclose(phi, phi_ref, rtol=1e-15)


def test_direct_two_body_golden():
    for d, q2, kappa, phi_ref in read_golden("two_body.txt"):
        pts = np.array([[0.0, 0.0, 0.0], [d, 0.0, 0.0]])
        kern = oracle.COULOMB if kappa == 0 else oracle.YUKAWA
        phi = oracle.direct(pts, pts, np.array([0.3, q2]), kernel=kern, kappa=kappa)
        assert phi[0] == pytest.approx(phi_ref, rel=1e-15)


def test_direct_regularized_two_body_golden():
    for d, q2, delta, phi_ref in read_golden("regularized_two_body.txt"):
        pts = np.array([[0.0, 0.0, 0.0], [0.0, d, 0.0]])
        phi = oracle.direct(pts, pts, np.array([0.3, q2]), kernel=oracle.REGULARIZED, kappa=delta)
        assert phi[0] == pytest.approx(phi_ref, rel=1e-15)


def test_regularized_kernel_limits():
    g = np.random.default_rng(5)
    t = g.uniform(-1, 1, (50, 3))
    s = g.uniform(-1, 1, (300, 3))
    q = g.uniform(-1, 1, 300)
    # delta -> 0: the Coulomb kernel (delta^2 underflows next to r^2)
    assert np.array_equal(oracle.direct(t, s, q, kernel=oracle.REGULARIZED, kappa=1e-200),
                          oracle.direct(t, s, q, kernel=oracle.COULOMB))
    # delta >> r: G -> 1/delta, phi -> sum(q)/delta with relative error <= (r/delta)^2 / 2
    phi = oracle.direct(t, s, q, kernel=oracle.REGULARIZED, kappa=1e4)
    assert np.allclose(phi * 1e4, q.sum(), rtol=0, atol=np.abs(q).sum() * 12 / 2e8)
    # below the Coulomb value everywhere for positive charges
    pos = np.abs(q)
    assert np.all(oracle.direct(t, s, pos, kernel=oracle.REGULARIZED, kappa=0.1) <
                  oracle.direct(t, s, pos, kernel=oracle.COULOMB))


@pytest.mark.parametrize("kernel,kappa", [(oracle.COULOMB, 0.0), (oracle.YUKAWA, 0.5),
                                          (oracle.REGULARIZED, 0.05)])
def test_direct_vs_high_precision(kernel, kappa):
    g = np.random.default_rng(3)
    t = g.uniform(-1, 1, (7, 3))
    s = g.uniform(-1, 1, (40, 3))
    q = g.uniform(-1, 1, (2, 40))
    phi = oracle.direct(t, s, q, kernel=kernel, kappa=kappa)
    for m in range(2):
        for i in range(7):
            acc = mp.mpf(0)
            for j in range(40):
                r = mp.sqrt(sum((mp.mpf(t[i, c]) - mp.mpf(s[j, c])) ** 2 for c in range(3)))
                if kernel == oracle.REGULARIZED:
                    acc += mp.mpf(q[m, j]) / mp.sqrt(r * r + mp.mpf(kappa) ** 2)
                else:
                    acc += mp.e ** (-mp.mpf(kappa) * r) / r * mp.mpf(q[m, j])
            assert phi[m, i] == pytest.approx(float(acc), rel=1e-13, abs=1e-14)


def test_direct_skips_zero_distance():
    pts = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 0.0], [1.0, 0.0, 0.0]])
    q = np.array([1.0, 2.0, 4.0])
    phi = oracle.direct(pts, pts, q)
    assert np.allclose(phi, [4.0, 4.0, 3.0])


def test_yukawa_kappa_zero_is_coulomb():
    pos, q = inputs.uniform_cube(300, 11)
    a = oracle.direct(pos, pos, q[0], kernel=oracle.COULOMB)
    b = oracle.direct(pos, pos, q[0], kernel=oracle.YUKAWA, kappa=0.0)
    assert np.array_equal(a, b)


# --------------------------------------------------------------------------
# Trees and batches (Sec. II-D, Sec. III-A)
# --------------------------------------------------------------------------
def _walk(tc):
    return [tc.cluster(i) for i in range(tc.n_clusters)]


@pytest.mark.parametrize("dist", ["cube", "plummer"])
def test_tree_invariants(dist):
    if dist == "cube":
        pos, _ = inputs.uniform_cube(6000, 5)
    else:
        pos, _ = inputs.plummer_sphere(6000, 5)
    leaf = 100
    tc = oracle.Treecode(pos, pos, 0.7, 3, leaf, leaf)
    order = tc.source_order()
    assert np.array_equal(np.sort(order), np.arange(len(pos)))
    nodes = _walk(tc)
    for nd in nodes:
        mem = pos[order[nd["begin"]:nd["begin"] + nd["count"]]]
        assert np.array_equal(mem.min(axis=0), nd["lo"])     # minimal box
        assert np.array_equal(mem.max(axis=0), nd["hi"])
        if nd["children"]:
            assert nd["count"] > leaf
            assert 2 <= len(nd["children"]) <= 8
            kids = [nodes[c] for c in nd["children"]]
            assert sum(k["count"] for k in kids) == nd["count"]
            assert kids[0]["begin"] == nd["begin"]
            for a, b in zip(kids, kids[1:]):
                assert a["begin"] + a["count"] == b["begin"]
            L = nd["hi"] - nd["lo"]
            split = 2 * L * L >= L.max() ** 2
            c = (nd["lo"] + nd["hi"]) / 2
            assert len(kids) <= 2 ** int(split.sum())
            for k in kids:
                kl = pos[order[k["begin"]:k["begin"] + k["count"]]]
                for d in range(3):
                    if split[d]:
                        side = kl[:, d] >= c[d]
                        assert side.all() or (~side).all()
                    # unsplit dimensions are not separated
            for k in kids:
                assert k["level"] == nd["level"] + 1
        else:
            assert nd["count"] <= leaf or np.all(nd["hi"] == nd["lo"])


def test_aspect_ratio_rule_splits_only_long_dims():
    # a slab: x extent 1, y extent 0.5, z extent 0.05 -> only x is split at the root
    g = np.random.default_rng(1)
    pos = np.stack([g.uniform(0, 1, 4000), g.uniform(0, 0.5, 4000), g.uniform(0, 0.05, 4000)], 1)
    tc = oracle.Treecode(pos, pos, 0.7, 2, 1000, 1000)
    root = tc.cluster(0)
    assert len(root["children"]) == 2
    # a 1 x 0.8 x 0.75 box splits in all three dimensions (0.75 >= 1/sqrt 2)
    pos2 = pos * np.array([1.0, 1.6, 15.0])
    tc2 = oracle.Treecode(pos2, pos2, 0.7, 2, 1000, 1000)
    assert len(tc2.cluster(0)["children"]) == 8


def test_identical_points_make_a_leaf():
    pos = np.zeros((50, 3)) + 0.25
    tc = oracle.Treecode(pos, pos, 0.7, 2, 10, 10)
    assert tc.n_clusters == 1 and tc.n_batches == 1
    q = np.ones(50)
    assert np.all(tc.potential(q) == 0.0)          # every pair at zero distance


def test_batches_equal_leaves_when_targets_are_sources():
    pos, _ = inputs.uniform_cube(5000, 9)
    tc = oracle.Treecode(pos, pos, 0.7, 3, 200, 200)
    leaves = [nd for nd in _walk(tc) if not nd["children"]]
    assert tc.n_batches == len(leaves)
    for b in range(tc.n_batches):
        bb = tc.batch(b)
        assert any(np.array_equal(bb["lo"], l["lo"]) and bb["count"] == l["count"] for l in leaves)


# --------------------------------------------------------------------------
# Interaction lists: Alg. 1 and the MAC of eq. (13)
# --------------------------------------------------------------------------
def _coverage(tc, pos_t):
    b, c, k = tc.items()
    tord = tc.target_order()
    ns = tc.ns
    for bi in range(tc.n_batches):
        cover = np.zeros(ns, dtype=np.int64)
        for cl in c[b == bi]:
            cover[tc.cluster_members(cl)] += 1
        assert np.all(cover == 1), "every source once per batch"


@pytest.mark.parametrize("theta,degree", [(0.5, 2), (0.7, 1), (0.9, 3)])
def test_each_pair_covered_exactly_once(theta, degree):
    pos, _ = inputs.uniform_cube(4000, 21)
    tc = oracle.Treecode(pos, pos, theta, degree, 64, 64)
    _coverage(tc, pos)


def test_coverage_distinct_targets_and_sources():
    g = np.random.default_rng(4)
    src = g.uniform(-1, 1, (3000, 3))
    tgt = g.uniform(-0.5, 1.5, (2000, 3))
    tc = oracle.Treecode(tgt, src, 0.6, 2, 50, 80)
    _coverage(tc, tgt)


def test_mac_decisions_follow_alg1():
    pos, _ = inputs.uniform_cube(8000, 13)
    theta, n = 0.7, 2
    P = (n + 1) ** 3
    tc = oracle.Treecode(pos, pos, theta, n, 100, 100)
    nodes = _walk(tc)
    parent = {}
    for i, nd in enumerate(nodes):
        for ch in nd["children"]:
            parent[ch] = i

    def center_radius(nd):
        L = nd["hi"] - nd["lo"]
        return (nd["lo"] + nd["hi"]) / 2, 0.5 * math.sqrt(L[0] * L[0] + L[1] * L[1] + L[2] * L[2])

    b, c, k = tc.items()
    for bi, cl, kind in zip(b, c, k):
        cb, rb = center_radius(tc.batch(bi))
        cc, rc = center_radius(nodes[cl])
        d = cb - cc
        R = math.sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2])
        geom = rb + rc < theta * R
        size = P < nodes[cl]["count"]
        if kind == 0:
            assert geom and size
        else:
            assert (not geom and not nodes[cl]["children"]) or (geom and not size)
        # every ancestor failed the geometric test
        a = parent.get(cl)
        while a is not None:
            ca, ra = center_radius(nodes[a])
            da = cb - ca
            Ra = math.sqrt(da[0] * da[0] + da[1] * da[1] + da[2] * da[2])
            assert not (rb + ra < theta * Ra)
            a = parent.get(a)


# --------------------------------------------------------------------------
# Modified charges, eq. (12): polynomial reproduction and moments
# --------------------------------------------------------------------------
def _cluster_setup(n=5, npts=3000, seed=17):
    pos, q = inputs.uniform_cube(npts, seed)
    tc = oracle.Treecode(pos, pos, 0.7, n, npts // 6, npts // 6)
    return pos, q, tc


def _tensor_poly(g, degs):
    c = g.standard_normal((degs[0] + 1, degs[1] + 1, degs[2] + 1))

    def p(x, y, z):
        return np.polynomial.polynomial.polyval3d(x, y, z, c)
    return p


@pytest.mark.parametrize("cluster", [0, 1, 5])
def test_modified_charges_reproduce_tensor_polynomials(cluster):
    n = 5
    pos, q, tc = _cluster_setup(n)
    mem = tc.cluster_members(cluster)
    qh = tc.modified_charges(cluster, q[0])
    s = tc.cluster_nodes(cluster)
    S1, S2, S3 = np.meshgrid(s[0], s[1], s[2], indexing="ij")
    g = np.random.default_rng(cluster)
    for degs in [(n, n, n), (n, 0, 2), (1, n, 3)]:
        p = _tensor_poly(g, degs)
        lhs = np.sum(qh * p(S1, S2, S3))
        rhs = np.sum(q[0][mem] * p(*pos[mem].T))
        assert lhs == pytest.approx(rhs, rel=1e-10, abs=1e-10 * np.sum(np.abs(q[0][mem])))
    # degree n+1 in one variable is not reproduced in general (the test has teeth)
    p = _tensor_poly(g, (n + 1, 0, 0))
    lhs = np.sum(qh * p(S1, S2, S3))
    rhs = np.sum(q[0][mem] * p(*pos[mem].T))
    assert abs(lhs - rhs) > 1e-8


def test_single_particle_modified_charges_are_lagrange_products():
    pos, q, tc = _cluster_setup(4)
    mem = tc.cluster_members(2)
    s = tc.cluster_nodes(2)
    j = mem[7]
    qq = np.zeros(tc.ns)
    qq[j] = 1.0
    qh = tc.modified_charges(2, qq)
    sm = [[mp.mpf(v) for v in s[d]] for d in range(3)]
    for k1, k2, k3 in [(0, 0, 0), (1, 3, 2), (4, 0, 3)]:
        ref = (_lagrange_product_form(sm[0], k1, pos[j, 0]) *
               _lagrange_product_form(sm[1], k2, pos[j, 1]) *
               _lagrange_product_form(sm[2], k3, pos[j, 2]))
        assert qh[k1, k2, k3] == pytest.approx(float(ref), rel=1e-10, abs=1e-12)


def test_charge_conservation_and_multiple_vectors():
    pos, _, tc = _cluster_setup(4)
    q = np.random.default_rng(2).uniform(-1, 1, (3, tc.ns))
    for c in range(tc.n_clusters):
        mem = tc.cluster_members(c)
        qh = tc.modified_charges(c, q)
        for m in range(3):
            assert qh[m].sum() == pytest.approx(q[m][mem].sum(), abs=1e-11)
            assert np.array_equal(qh[m], tc.modified_charges(c, q[m]))


def test_particle_on_a_node_deposits_its_charge_there():
    # a cluster whose corner particles sit exactly on grid nodes (k = 0 at hi, k = n at lo)
    pts = np.array([[0.0, 0.0, 0.0], [1.0, 1.0, 1.0], [0.25, 0.6, 0.3], [0.7, 0.2, 0.9]])
    tc = oracle.Treecode(pts, pts, 0.7, 3, 10, 10)
    s = tc.cluster_nodes(0)
    assert s[0][0] == 1.0 and s[0][3] == 0.0
    qq = np.array([2.0, 0.0, 0.0, 0.0])
    qh = tc.modified_charges(0, qq)
    expect = np.zeros((4, 4, 4))
    expect[3, 3, 3] = 2.0
    assert np.array_equal(qh, expect)


def test_parent_modified_charges_from_children():
    # q^parent_k = sum_child sum_m L^P_k(s^child_m) q^child_m: exact for degree-n polynomials
    n = 4
    pos, q, tc = _cluster_setup(n, npts=4000, seed=23)
    parent = 0
    kids = tc.cluster(parent)["children"]
    sp = tc.cluster_nodes(parent)
    _, w = oracle.chebyshev(n)
    total = np.zeros((n + 1,) * 3)
    for ch in kids:
        sc = tc.cluster_nodes(ch)
        T = [np.array([oracle.lagrange(n, sp[d], w, x) for x in sc[d]]) for d in range(3)]
        qc = tc.modified_charges(ch, q[0])
        total += np.einsum("ai,bj,ck,abc->ijk", T[0], T[1], T[2], qc)
    qp = tc.modified_charges(parent, q[0])
    assert np.allclose(total, qp, rtol=1e-9, atol=1e-9 * np.abs(qp).max())


# --------------------------------------------------------------------------
# Treecode vs direct sum
# --------------------------------------------------------------------------
def test_theta_zero_is_direct_sum():
    pos, q = inputs.uniform_cube(3000, 31)
    tc = oracle.Treecode(pos, pos, 0.0, 4, 100, 100)
    b, c, k = tc.items()
    assert np.all(k == 1)
    d = oracle.direct(pos, pos, q[0])
    assert oracle.rel_l2(d, tc.potential(q[0])) < 1e-14


def test_large_degree_means_all_direct():
    pos, q = inputs.uniform_cube(2000, 32)
    tc = oracle.Treecode(pos, pos, 0.9, 12, 50, 50)    # P = 2197 > N
    _, _, k = tc.items()
    assert np.all(k == 1)
    d = oracle.direct(pos, pos, q[0], kernel=oracle.YUKAWA, kappa=0.5)
    p = tc.potential(q[0], kernel=oracle.YUKAWA, kappa=0.5)
    assert oracle.rel_l2(d, p) < 1e-14


@pytest.mark.parametrize("kernel,kappa", [(oracle.COULOMB, 0.0), (oracle.YUKAWA, 0.5),
                                          (oracle.REGULARIZED, 0.02)])
def test_error_decreases_with_degree(kernel, kappa):
    pos, q = inputs.uniform_cube(12000, 41)
    d = oracle.direct(pos, pos, q[0], kernel=kernel, kappa=kappa)
    errs = []
    for n in (1, 2, 3, 4, 6, 8):
        tc = oracle.Treecode(pos, pos, 0.7, n, 40, 40)
        errs.append(oracle.rel_l2(d, tc.potential(q[0], kernel=kernel, kappa=kappa)))
    assert all(b < a for a, b in zip(errs, errs[1:])), errs
    assert errs[-1] < 1e-6 and errs[0] > 1e-4


def test_single_pair_approximation_converges():
    # one well-separated batch/cluster pair: eq. (11) vs eq. (9) as n grows
    g = np.random.default_rng(8)
    src = g.uniform(0, 1, (1500, 3))
    tgt = g.uniform(0, 1, (300, 3)) + np.array([4.0, 0.5, -1.0])
    q = g.uniform(-1, 1, 1500)
    d = oracle.direct(tgt, src, q)
    errs = []
    for n in (2, 4, 6, 8, 10):
        tc = oracle.Treecode(tgt, src, 0.9, n, 2000, 2000)
        _, _, k = tc.items()
        assert list(k) == [0]
        errs.append(oracle.rel_l2(d, tc.potential(q)))
    assert all(b < 0.2 * a for a, b in zip(errs, errs[1:])), errs
    assert errs[-1] < 1e-10


def test_sampled_mode_matches_full_mode():
    pos, q = inputs.uniform_cube(5000, 51)
    tc = oracle.Treecode(pos, pos, 0.7, 3, 150, 150)
    full = tc.potential(q[0], kernel=oracle.YUKAWA, kappa=0.5)
    smp = inputs.sample_indices(5000, 300, 52)
    part = tc.potential(q[0], kernel=oracle.YUKAWA, kappa=0.5, sample=smp)
    assert np.array_equal(full[smp], part)


def test_error_band_against_printed_values():
    # theta = 0.8, n = 8, N_L = N_B = 4000 gives 5-6 digit accuracy (Sec. IV: 4.0e-6 and
    # 3.0e-6 at 16M, 5.9e-6 and 7.2e-6 at 64M).  At 2e5 particles the tree is shallower,
    # so only the upper end of the band is checked; exact values are not pinned.
    pos, q = inputs.uniform_cube(200000, 61)
    smp = inputs.sample_indices(200000, 300, 62)
    tc = oracle.Treecode(pos, pos, 0.8, 8, 4000, 4000)
    for kern, kappa in ((oracle.COULOMB, 0.0), (oracle.YUKAWA, 0.5)):
        p = tc.potential(q[0], kernel=kern, kappa=kappa, sample=smp)
        d = oracle.direct(pos[smp], pos, q[0], kernel=kern, kappa=kappa)
        e = oracle.rel_l2(d, p)
        assert 1e-9 < e < 7.2e-6, e


def test_split_plane_tie_goes_to_upper_child():
    # a lattice whose root midpoint coincides with particle coordinates (reading: y >= c is upper)
    v = np.array([0.0, 0.5, 1.0])
    pos = np.array([[a, b, c] for a in v for b in v for c in v])
    tc = oracle.Treecode(pos, pos, 0.7, 1, 8, 8)
    order = tc.source_order()
    root = tc.cluster(0)
    assert len(root["children"]) == 8
    for ch in root["children"]:
        nd = tc.cluster(ch)
        mem = pos[order[nd["begin"]:nd["begin"] + nd["count"]]]
        for d in range(3):
            # each child holds either {0} or {0.5, 1} along every axis
            vals = set(mem[:, d].tolist())
            assert vals in ({0.0}, {0.5, 1.0})
