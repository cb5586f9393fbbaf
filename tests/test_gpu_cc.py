"""GPU cluster-cluster treecode (method "cc") against the oracle's.

The library and the oracle build the same trees and pairs (checked on the
host in test_cc_structure.py), so in FP64 they differ only in rounding order:
max|d| <= 1e-12 max|phi| and rel-L2 <= 1e-13, as for the BLTC.  The
FP32-mixed path is held to rel-L2 <= 1e-6 against the FP64 oracle.
"""
import numpy as np
import pytest

import oracle
from tests.conftest import KERNEL_CASES, assert_mixed, kernel_kwargs
from paper_2003_01836_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

REL_MAX = 1e-12
REL_L2 = 1e-13
MIXED_L2 = 1e-6


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2003_01836_amd as bltc
    bltc.version()
    return torch.device("cuda:0")


def _soa(pos):
    return np.ascontiguousarray(np.asarray(pos, dtype=np.float64).T)


def _close(ref, got, rel_max=REL_MAX, rel_l2=REL_L2):
    ref = np.asarray(ref)
    got = np.asarray(got)
    assert np.all(np.isfinite(got))
    scale = np.max(np.abs(ref)) if ref.size else 1.0
    assert np.max(np.abs(ref - got)) <= rel_max * max(scale, 1e-300)
    assert oracle.rel_l2(ref, got) <= rel_l2


def _run(dev, tgt, src, q, **kw):
    import paper_2003_01836_amd as bltc
    t = torch.from_numpy(_soa(tgt)).to(dev)
    s = t if src is tgt else torch.from_numpy(_soa(src)).to(dev)
    plan = bltc.Plan(t, s, method="cc", **kw)
    phi = plan.execute(torch.from_numpy(np.ascontiguousarray(q)).to(dev))
    torch.cuda.synchronize()
    return plan, phi.cpu().numpy()


@pytest.mark.parametrize("kernel,kappa", KERNEL_CASES)
def test_cc_fp64_small_config(dev, kernel, kappa):
    pos, q = inputs.uniform_cube(10000, inputs.config_seed(0))
    plan, phi = _run(dev, pos, pos, q[0], theta=0.7, degree=4, leaf_size=500, batch_size=500,
                     **kernel_kwargs(kernel, kappa)[0])
    kern = kernel_kwargs(kernel, kappa)[1]
    oc = oracle.ClusterCluster(pos, pos, 0.7, 4, 500, 500)
    ref = oc.potential(q[0], kernel=kern, kappa=kappa)
    _close(ref, phi)
    st = plan.stats()
    assert st["approx_pairs"] > 0 and st["direct_pairs"] > 0


def test_cc_proxy_potentials_match_oracle(dev):
    pos, q = inputs.uniform_cube(40000, 81)
    plan, _ = _run(dev, pos, pos, q[0], theta=0.7, degree=4, leaf_size=300, batch_size=300)
    oc = oracle.ClusterCluster(pos, pos, 0.7, 4, 300, 300)
    v = plan.view()
    tord = v["target_order"]
    okey = {}
    for c in range(oc.n_target_nodes):
        info = oc.node(0, c)
        okey[tuple(np.sort(tord[info["begin"]:info["begin"] + info["count"]]))] = c
    kinds = v["item_kind"]
    targets = np.unique(v["item_batch"][(kinds == 0) | (kinds == 2)])
    checked = 0
    for c in targets:
        key = tuple(np.sort(tord[v["batch_begin"][c]:v["batch_begin"][c] + v["batch_count"][c]]))
        ref = oc.proxy_potentials(okey[key], q[0]).reshape(-1)
        got = np.asarray(plan.modified_charges(c)).reshape(-1)
        assert np.max(np.abs(ref - got)) <= 1e-12 * np.max(np.abs(ref)), c
        checked += 1
    assert checked > 10
    assert np.sum(kinds == 0) > 0 and np.sum(kinds == 1) > 0 and np.sum(kinds == 2) > 0


@pytest.mark.parametrize("degree,n,leaf", [(1, 12000, 64), (2, 12000, 64), (7, 12000, 256),
                                           (12, 60000, 2500), (16, 60000, 2500)])
def test_cc_fp64_degrees(dev, degree, n, leaf):
    pos, q = inputs.uniform_cube(n, 90 + degree)
    plan, phi = _run(dev, pos, pos, q[0], theta=0.8, degree=degree, leaf_size=leaf, batch_size=300)
    assert plan.stats()["approx_pairs"] > 0
    smp = inputs.sample_indices(n, 600, 91 + degree)
    ref = oracle.ClusterCluster(pos, pos, 0.8, degree, leaf, 300).potential(q[0], sample=smp)
    _close(ref, phi[smp])


def test_cc_fp64_distinct_sets_yukawa(dev):
    g = np.random.default_rng(82)
    tgt = g.uniform(-1, 1, (9000, 3))
    src = g.uniform(-0.4, 1.6, (11000, 3))
    q = g.uniform(-1, 1, 11000)
    _, phi = _run(dev, tgt, src, q, theta=0.7, degree=5, leaf_size=250, batch_size=150,
                  kernel="yukawa", kappa=0.8)
    ref = oracle.ClusterCluster(tgt, src, 0.7, 5, 250, 150).potential(q, kernel=oracle.YUKAWA,
                                                                        kappa=0.8)
    _close(ref, phi)


def test_cc_fp64_plummer(dev):
    pos, q = inputs.plummer_sphere(30000, 83)
    _, phi = _run(dev, pos, pos, q[0], theta=0.7, degree=6, leaf_size=400, batch_size=400)
    ref = oracle.ClusterCluster(pos, pos, 0.7, 6, 400, 400).potential(q[0])
    _close(ref, phi)


def test_cc_theta_zero_is_direct_sum(dev):
    pos, q = inputs.uniform_cube(4000, 84)
    plan, phi = _run(dev, pos, pos, q[0], theta=0.0, degree=4, leaf_size=100, batch_size=100)
    assert plan.stats()["approx_pairs"] == 0
    _close(oracle.direct(pos, pos, q[0]), phi, 1e-13, 1e-14)


@pytest.mark.parametrize("precision", ["fp64", "fp32_mixed"])
def test_cc_device_and_host_plans_agree(dev, precision):
    import paper_2003_01836_amd as bltc
    pos, q = inputs.uniform_cube(30000, 85)
    kw = dict(method="cc", theta=0.7, degree=6, leaf_size=400, batch_size=250, precision=precision)
    th = _soa(pos)
    td = torch.from_numpy(th).to(dev)
    pd = bltc.Plan(td, td, **kw)
    ph = bltc.Plan(th, th, host=True, **kw)
    vd, vh = pd.view(), ph.view()
    for k in vd:
        assert np.array_equal(vd[k], vh[k]), k
    qd = torch.from_numpy(q[0]).to(dev)
    assert np.array_equal(pd.execute(qd).cpu().numpy(), ph.execute(qd).cpu().numpy())


@pytest.mark.parametrize("kernel,kappa", KERNEL_CASES)
def test_cc_mixed_matches_oracle(dev, kernel, kappa):
    pos, q = inputs.uniform_cube(20000, 86)
    _, phi = _run(dev, pos, pos, q[0], theta=0.7, degree=6, leaf_size=400, batch_size=400,
                  **kernel_kwargs(kernel, kappa)[0], precision="fp32_mixed")
    kern = kernel_kwargs(kernel, kappa)[1]
    ref = oracle.ClusterCluster(pos, pos, 0.7, 6, 400, 400).potential(q[0], kernel=kern,
                                                                        kappa=kappa)
    assert np.all(np.isfinite(phi))
    assert_mixed(ref, phi, pos, pos, q[0], kern, kappa, what=f"cc {kernel}")


def test_cc_full_size_sampled(dev):
    # 10^6 uniform, theta 0.7, n 8, N_L = N_B = 2000; oracle on 1000 sampled targets
    pos, q = inputs.uniform_cube(1_000_000, inputs.config_seed(1))
    smp = inputs.sample_indices(1_000_000, 1000, inputs.sample_seed(1))
    ref = oracle.ClusterCluster(pos, pos, 0.7, 8, 2000, 2000).potential(q[0], sample=smp)
    for precision in ("fp64", "fp32_mixed"):
        _, phi = _run(dev, pos, pos, q[0], theta=0.7, degree=8, leaf_size=2000, batch_size=2000,
                      precision=precision)
        if precision == "fp64":
            _close(ref, phi[smp])
        else:
            assert_mixed(ref, phi[smp], pos, pos, q[0], idx=smp, what="cc 1M sampled")


@pytest.mark.parametrize("precision", ["fp64", "fp32_mixed"])
def test_cc_edge_cases(dev, precision):
    import paper_2003_01836_amd as bltc
    g = np.random.default_rng(87)
    e = torch.zeros((3, 0), dtype=torch.float64, device=dev)
    pos = g.uniform(-1, 1, (500, 3))
    q = g.uniform(-1, 1, 500)
    pd = torch.from_numpy(_soa(pos)).to(dev)
    qd = torch.from_numpy(q).to(dev)
    # no targets: nothing to do; no sources: zeros
    assert bltc.Plan(e, pd, method="cc", precision=precision).execute(qd).numel() == 0
    z = bltc.Plan(pd, e, method="cc", precision=precision).execute(
        torch.zeros(0, dtype=torch.float64, device=dev))
    assert torch.all(z == 0)
    # one target, ragged sizes, duplicates, identical points
    cases = [(pos[:1], pos, 4, 64, 64), (pos[:257], pos, 3, 50, 33),
             (np.concatenate([pos, pos[:50]]), pos, 4, 40, 40),
             (np.full((300, 3), 0.5), pos, 2, 10, 10)]
    for tgt, src, n, leaf, batch in cases:
        t = torch.from_numpy(_soa(tgt)).to(dev)
        phi = bltc.Plan(t, pd, method="cc", degree=n, leaf_size=leaf, batch_size=batch,
                        precision=precision).execute(qd).cpu().numpy()
        ref = oracle.ClusterCluster(tgt, src, 0.7, n, leaf, batch).potential(q)
        if precision == "fp64":
            _close(ref, phi)
        else:
            assert_mixed(ref, phi, tgt, src, q, what=f"cc edge n={n} leaf={leaf}")


def test_cc_rejects_unsupported(dev):
    import paper_2003_01836_amd as bltc
    pos, q = inputs.uniform_cube(1000, 88)
    t = torch.from_numpy(_soa(pos)).to(dev)
    with pytest.raises(bltc.BLTCError):
        bltc.Plan(t, t, method="cc", max_q=4)
    plan = bltc.Plan(t, t, method="cc")
    with pytest.raises(bltc.BLTCError):
        plan.execute(torch.from_numpy(np.stack([q[0], q[0]])).to(dev))
    with pytest.raises(bltc.BLTCError):
        bltc.Batch([plan])
