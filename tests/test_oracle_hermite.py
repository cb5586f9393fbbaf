"""Pins of the oracle's barycentric Hermite treecode (readings 25-27), against
facts independent of its code:

* the 1-D Hermite basis on the Chebyshev points reproduces every polynomial of
  degree <= 2n+1 from its values and first derivatives at the nodes, and not
  degree 2n+2 (this determines the basis uniquely);
* the kernel derivatives g1 = G'/r, g2 = g1'/r, g3 = g2'/r agree with
  40-digit numerical differentiation for the three kernels;
* the modified charges reproduce moments: sum_k sum_a qhat^a_k d^a p(s_k) =
  sum_j q_j p(y_j) for tensor polynomials of degree <= 2n+1 per variable;
* theta = 0 is the direct sum; the error against the direct sum falls with n,
  for a single well-separated pair geometrically.
"""
import mpmath as mp
import numpy as np
import pytest

import oracle
from paper_2003_01836_amd import inputs

mp.mp.dps = 40


@pytest.mark.parametrize("n,a,b", [(1, -1.0, 1.0), (3, 0.2, 0.7), (6, -2.0, 5.0), (10, -1.0, 1.0)])
def test_hermite_basis_reproduces_degree_2n_plus_1(n, a, b):
    s, w = oracle.chebyshev(n, a, b)
    g = np.random.default_rng(n)
    xs = list(g.uniform(a, b, 5)) + [s[0], s[n // 2], s[n] + 1e-9 * (b - a)]
    for deg, exact in ((2 * n + 1, True), (2 * n + 2, False)):
        c = g.uniform(-1, 1, deg + 1)
        p = np.polynomial.Polynomial(c)
        dp = p.deriv()
        worst = 0.0
        for x in xs:
            A, B = oracle.hermite_basis(n, s, w, x)
            val = np.dot(p(s), A) + np.dot(dp(s), B)
            worst = max(worst, abs(val - p(x)) / max(1.0, np.abs(c).sum() * max(abs(a), abs(b), 1) ** deg))
        if exact:
            assert worst < 1e-11
        else:
            assert worst > 1e-9


def test_hermite_basis_at_nodes_and_degenerate_nodes():
    s, w = oracle.chebyshev(4, -1.0, 1.0)
    for k in range(5):
        A, B = oracle.hermite_basis(4, s, w, s[k])
        assert np.array_equal(A, np.eye(5)[k]) and np.all(B == 0.0)
    s0, w0 = oracle.chebyshev(4, 0.5, 0.5)          # zero-width box: all nodes equal
    A, B = oracle.hermite_basis(4, s0, w0, 0.5)
    assert np.array_equal(A, np.eye(5)[0]) and np.all(B == 0.0)


@pytest.mark.parametrize("kernel,param", [(oracle.COULOMB, 0.0), (oracle.YUKAWA, 0.8),
                                          (oracle.REGULARIZED, 0.3)])
def test_kernel_derivatives_against_numerical_differentiation(kernel, param):
    par = mp.mpf(param)

    def G(t):
        if kernel == oracle.YUKAWA:
            return mp.e ** (-par * t) / t
        if kernel == oracle.REGULARIZED:
            return 1 / mp.sqrt(t * t + par * par)
        return 1 / t

    g1 = lambda t: mp.diff(G, t) / t
    g2 = lambda t: mp.diff(g1, t) / t
    g3 = lambda t: mp.diff(g2, t) / t
    for r in (0.05, 0.4, 1.7, 6.0):
        got = oracle.kernel_derivatives(r, kernel, param)
        ref = [G(mp.mpf(r)), g1(mp.mpf(r)), g2(mp.mpf(r)), g3(mp.mpf(r))]
        for a, b in zip(got, ref):
            assert a == pytest.approx(float(b), rel=1e-13)


def _tensor_poly(deg, seed):
    g = np.random.default_rng(seed)
    cs = [np.polynomial.Polynomial(g.uniform(-1, 1, deg + 1)) for _ in range(3)]
    return cs


@pytest.mark.parametrize("n", [1, 2, 4])
def test_hermite_charges_reproduce_moments(n):
    pos, q = inputs.uniform_cube(3000, 40 + n)
    tc = oracle.Treecode(pos, pos, 0.7, n, 400, 400, hermite=True)
    c = 1                                     # a child of the root
    info = tc.cluster(c)
    members = tc.source_order()[info["begin"]:info["begin"] + info["count"]]
    Q = tc.hermite_charges(c, q[0])
    nodes = tc.cluster_nodes(c)
    for deg, exact in ((2 * n + 1, True), (2 * n + 2, False)):
        px, py, pz = _tensor_poly(deg, 7 * n + deg)
        fx = [px(nodes[0]), px.deriv()(nodes[0])]
        fy = [py(nodes[1]), py.deriv()(nodes[1])]
        fz = [pz(nodes[2]), pz.deriv()(nodes[2])]
        lhs = 0.0
        for a in range(8):
            a1, a2, a3 = (a >> 2) & 1, (a >> 1) & 1, a & 1
            lhs += np.einsum("ijk,i,j,k->", Q[a], fx[a1], fy[a2], fz[a3])
        y = pos[members]
        rhs = np.sum(q[0][members] * px(y[:, 0]) * py(y[:, 1]) * pz(y[:, 2]))
        scale = np.sum(np.abs(q[0][members])) * 10.0 ** 3
        if exact:
            assert abs(lhs - rhs) <= 1e-11 * scale
        else:
            assert abs(lhs - rhs) > 1e-12 * scale


def test_theta_zero_is_direct_sum():
    pos, q = inputs.uniform_cube(3000, 50)
    tc = oracle.Treecode(pos, pos, 0.0, 3, 100, 100, hermite=True)
    assert oracle.rel_l2(oracle.direct(pos, pos, q[0]), tc.potential(q[0])) <= 1e-14


@pytest.mark.parametrize("kernel,param", [(oracle.COULOMB, 0.0), (oracle.YUKAWA, 0.5),
                                          (oracle.REGULARIZED, 0.02)])
def test_error_decreases_with_degree(kernel, param):
    pos, q = inputs.uniform_cube(40000, 51)
    smp = inputs.sample_indices(40000, 400, 52)
    d = oracle.direct(pos[smp], pos, q[0], kernel=kernel, kappa=param)
    errs = []
    for n in (1, 2, 3, 4):
        tc = oracle.Treecode(pos, pos, 0.7, n, 5000, 5000, hermite=True)
        assert np.sum(tc.items()[2] == 0) > 0
        errs.append(oracle.rel_l2(d, tc.potential(q[0], kernel=kernel, kappa=param, sample=smp)))
    assert all(b < 0.5 * a for a, b in zip(errs, errs[1:])), errs


def test_single_pair_converges_geometrically():
    g = np.random.default_rng(53)
    src = g.uniform(0.0, 1.0, (2500, 3))
    tgt = g.uniform(0.0, 1.0, (50, 3)) + np.array([4.0, 0.0, 0.0])
    q = g.uniform(-1, 1, 2500)
    d = oracle.direct(tgt, src, q)
    errs = []
    for n in (1, 2, 3, 4, 5):
        tc = oracle.Treecode(tgt, src, 0.9, n, 2500, 2500, hermite=True)
        b, c, k = tc.items()
        assert list(k) == [0]
        errs.append(oracle.rel_l2(d, tc.potential(q)))
    ratios = [b / a for a, b in zip(errs, errs[1:])]
    assert all(r < 0.1 for r in ratios), errs


def test_size_test_counts_eight_values_per_node():
    # one well-separated pair, 50 sources, n = 1: (n+1)^3 = 8 < 50 <= 8 (n+1)^3 = 64:
    # the BLTC approximates, the Hermite treecode sums directly (reading 27)
    g = np.random.default_rng(54)
    src = g.uniform(0.0, 1.0, (50, 3))
    tgt = g.uniform(0.0, 1.0, (10, 3)) + np.array([5.0, 0.0, 0.0])
    assert list(oracle.Treecode(tgt, src, 0.9, 1, 50, 50).items()[2]) == [0]
    assert list(oracle.Treecode(tgt, src, 0.9, 1, 50, 50, hermite=True).items()[2]) == [1]
    src = g.uniform(0.0, 1.0, (65, 3))
    assert list(oracle.Treecode(tgt, src, 0.9, 1, 65, 65, hermite=True).items()[2]) == [0]
