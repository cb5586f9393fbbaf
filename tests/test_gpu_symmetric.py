"""Mutual direct leaf pairs evaluated once for both directions (targets are
the sources).  The symmetric path must give the potentials of the plain path:
in FP64 up to rounding order (and both equal the oracle to the usual 1e-12 /
1e-13), in FP32-mixed within the mixed path's own error against the oracle."""
import numpy as np
import pytest

import oracle
from tests.conftest import KERNEL_CASES, assert_mixed, kernel_kwargs
from paper_2003_01836_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2003_01836_amd as bltc
    bltc.version()
    return torch.device("cuda:0")


def _soa(pos, dev):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(pos, dtype=np.float64).T)).to(dev)


def _both(dev, pos, q, **kw):
    import paper_2003_01836_amd as bltc
    t = _soa(pos, dev)
    qd = torch.from_numpy(np.ascontiguousarray(q)).to(dev)
    ps = bltc.Plan(t, t, **kw)
    pn = bltc.Plan(t, t, symmetry=False, **kw)
    a = ps.execute(qd).cpu().numpy()
    b = pn.execute(qd).cpu().numpy()
    return ps, pn, a, b


def _close(ref, got, rel_max=1e-12, rel_l2=1e-13):
    scale = np.max(np.abs(ref))
    assert np.all(np.isfinite(got))
    assert np.max(np.abs(ref - got)) <= rel_max * scale
    assert oracle.rel_l2(ref, got) <= rel_l2


@pytest.mark.parametrize("kernel,kappa", KERNEL_CASES)
@pytest.mark.parametrize("n,leaf,degree", [(30000, 700, 5), (20000, 97, 3), (40000, 1500, 6)])
def test_fp64_symmetric_equals_plain_and_oracle(dev, kernel, kappa, n, leaf, degree):
    # leaves of ragged sizes: not multiples of 64 or 8, more than 512 targets
    # (several register chunks per unit) and fewer than 64
    pos, q = inputs.uniform_cube(n, 400 + leaf)
    kk, kern, kpar = kernel_kwargs(kernel, kappa)
    ps, pn, a, b = _both(dev, pos, q[0], theta=0.7, degree=degree, leaf_size=leaf,
                         batch_size=leaf, **kk)
    assert ps.stats()["mutual_pair_evals"] > 0
    assert pn.stats()["mutual_pair_evals"] == 0
    _close(b, a, 1e-13, 1e-14)
    ref = oracle.Treecode(pos, pos, 0.7, degree, leaf, leaf).potential(q[0], kernel=kern,
                                                                       kappa=kpar)
    _close(ref, a)


@pytest.mark.parametrize("kernel,kappa", KERNEL_CASES)
def test_mixed_symmetric_matches_oracle(dev, kernel, kappa):
    pos, q = inputs.plummer_sphere(40000, 410)
    kk, kern, kpar = kernel_kwargs(kernel, kappa)
    ps, pn, a, b = _both(dev, pos, q[0], theta=0.7, degree=6, leaf_size=900, batch_size=900,
                         precision="fp32_mixed", **kk)
    assert ps.stats()["mutual_pair_evals"] > 0
    ref = oracle.Treecode(pos, pos, 0.7, 6, 900, 900).potential(q[0], kernel=kern, kappa=kpar)
    assert_mixed(ref, a, pos, pos, q[0], kern, kpar, what="mutual pairs")
    assert_mixed(ref, b, pos, pos, q[0], kern, kpar, what="plain lists")
    assert oracle.rel_l2(b, a) <= 1e-6


def test_mixed_symmetric_close_pairs(dev):
    # pairs at separations 1e-7 .. 1e-3 across leaf boundaries: the FP64 kernel values
    g = np.random.default_rng(411)
    base, q = inputs.uniform_cube(30000, 412)
    k = 600
    offs = g.standard_normal((k, 3))
    offs *= (10.0 ** g.uniform(-7, -3, k) / np.linalg.norm(offs, axis=1))[:, None]
    pos = np.concatenate([base, base[:k] + offs])
    qq = np.concatenate([q[0], g.uniform(-1, 1, k)])
    ps, _, a, b = _both(dev, pos, qq, theta=0.7, degree=6, leaf_size=600, batch_size=600,
                        precision="fp32_mixed")
    assert ps.stats()["mutual_pair_evals"] > 0
    ref = oracle.Treecode(pos, pos, 0.7, 6, 600, 600).potential(qq)
    assert_mixed(ref, a, pos, pos, qq, what="planted")
    close = np.arange(len(base), len(base) + k)
    assert_mixed(ref[close], a[close], pos, pos, qq, idx=close, what="planted targets")


def test_hermite_symmetric_equals_plain(dev):
    pos, q = inputs.uniform_cube(30000, 413)
    ps, pn, a, b = _both(dev, pos, q[0], method="hermite", theta=0.7, degree=3, leaf_size=800,
                         batch_size=800)
    assert ps.stats()["mutual_pair_evals"] > 0
    _close(b, a, 1e-13, 1e-14)
    ref = oracle.Treecode(pos, pos, 0.7, 3, 800, 800, hermite=True).potential(q[0])
    _close(ref, a)


def test_symmetric_repeatable_and_host_plan_identical(dev):
    import paper_2003_01836_amd as bltc
    pos, q = inputs.uniform_cube(30000, 414)
    t = _soa(pos, dev)
    th = np.ascontiguousarray(pos.T)
    qd = torch.from_numpy(q[0]).to(dev)
    for prec in ("fp64", "fp32_mixed"):
        kw = dict(theta=0.7, degree=5, leaf_size=500, batch_size=500, precision=prec)
        pd = bltc.Plan(t, t, **kw)
        ph = bltc.Plan(th, th, host=True, **kw)
        a = pd.execute(qd).cpu().numpy()
        assert np.array_equal(a, pd.execute(qd).cpu().numpy())
        assert np.array_equal(a, ph.execute(qd).cpu().numpy())
        assert pd.stats()["mutual_pair_evals"] == ph.stats()["mutual_pair_evals"] > 0


def test_symmetric_not_used_where_it_does_not_apply(dev):
    import paper_2003_01836_amd as bltc
    pos, q = inputs.uniform_cube(20000, 415)
    t = _soa(pos, dev)
    t2 = t.clone()                      # same points, different arrays
    assert bltc.Plan(t, t2, leaf_size=400, batch_size=400).stats()["mutual_pair_evals"] == 0
    assert bltc.Plan(t, t, leaf_size=400, batch_size=300).stats()["mutual_pair_evals"] == 0
    assert bltc.Plan(t, t, leaf_size=400, batch_size=400, max_q=2).stats()["mutual_pair_evals"] == 0
    assert bltc.Plan(t, t, leaf_size=400, batch_size=300, method="cp").stats()["mutual_pair_evals"] == 0



@pytest.mark.parametrize("precision", ["fp64", "fp32_mixed"])
def test_symmetric_large_leaves(dev, precision):
    # leaves of ~8800 particles: many sub-units per pair (256 or 512 targets each)
    import paper_2003_01836_amd as bltc
    big, qb = inputs.uniform_cube(70000, 416)
    tb = _soa(big, dev)
    p = bltc.Plan(tb, tb, leaf_size=9000, batch_size=9000, degree=4, theta=0.8,
                  precision=precision)
    assert p.stats()["mutual_pair_evals"] > 0
    phi = p.execute(torch.from_numpy(qb[0]).to(dev)).cpu().numpy()
    smp = inputs.sample_indices(70000, 300, 417)
    ref = oracle.Treecode(big, big, 0.8, 4, 9000, 9000).potential(qb[0], sample=smp)
    if precision == "fp64":
        _close(ref, phi[smp])
    else:
        assert_mixed(ref, phi[smp], big, big, qb[0], idx=smp, what="large leaves")


@pytest.mark.parametrize("precision", ["fp64", "fp32_mixed"])
@pytest.mark.parametrize("n,leaf", [(3000, 7), (40000, 1030), (30000, 513)])
def test_symmetric_block_and_subunit_boundaries(dev, precision, n, leaf):
    # leaves below one source block (fewer than 8 particles), and leaves just
    # above one or two sub-units of targets (256 / 512): a last sub-unit of a
    # few targets, a last block of a few sources
    pos, q = inputs.uniform_cube(n, 420 + leaf)
    ps, pn, a, b = _both(dev, pos, q[0], theta=0.6, degree=2 if leaf < 64 else 4, leaf_size=leaf,
                         batch_size=leaf, precision=precision)
    assert ps.stats()["mutual_pair_evals"] > 0
    ref = oracle.Treecode(pos, pos, 0.6, 2 if leaf < 64 else 4, leaf, leaf).potential(q[0])
    if precision == "fp64":
        _close(b, a, 1e-13, 1e-14)
        _close(ref, a)
    else:
        assert_mixed(ref, a, pos, pos, q[0], what=f"leaf {leaf}")


@pytest.mark.parametrize("method", ["cc", "cp"])
@pytest.mark.parametrize("precision", ["fp64", "fp32_mixed"])
@pytest.mark.parametrize("kernel,kappa", KERNEL_CASES)
def test_cluster_cluster_and_particle_symmetric(dev, method, precision, kernel, kappa):
    # the dual walk (cc) and the walk of the source batches (cp) on one tree
    # give mutual direct leaf pairs as well
    pos, q = inputs.uniform_cube(30000, 430)
    kk, kern, kpar = kernel_kwargs(kernel, kappa)
    ps, pn, a, b = _both(dev, pos, q[0], method=method, theta=0.7, degree=4, leaf_size=300,
                         batch_size=300, precision=precision, **kk)
    assert ps.stats()["mutual_pair_evals"] > 0
    assert pn.stats()["mutual_pair_evals"] == 0
    cls = oracle.ClusterCluster if method == "cc" else oracle.ClusterParticle
    ref = cls(pos, pos, 0.7, 4, 300, 300).potential(q[0], kernel=kern, kappa=kpar)
    if precision == "fp64":
        _close(b, a, 1e-13, 1e-14)
        _close(ref, a)
    else:
        assert_mixed(ref, a, pos, pos, q[0], kern, kpar, what=f"{method} mutual pairs")
        assert_mixed(ref, b, pos, pos, q[0], kern, kpar, what=f"{method} plain lists")
