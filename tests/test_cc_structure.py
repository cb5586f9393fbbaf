"""Cluster-cluster plans on the host: trees and the pairs of the dual walk
against the oracle's cluster-cluster treecode (CPU only)."""
import numpy as np
import pytest

import oracle
import paper_2003_01836_amd as bltc
from paper_2003_01836_amd import inputs


def _soa(pos):
    return np.ascontiguousarray(np.asarray(pos, dtype=np.float64).T)


def _key(order, b, c):
    return tuple(np.sort(order[b:b + c]).tolist())


def _compare(tgt, src, theta, degree, leaf, batch):
    th = _soa(tgt)
    sh = th if src is tgt else _soa(src)
    plan = bltc.Plan(th, sh, host=True, method="cc", theta=theta, degree=degree, leaf_size=leaf,
                     batch_size=batch)
    v = plan.view()
    oc = oracle.ClusterCluster(tgt, src, theta, degree, leaf, batch)
    otord, osord = oc.orders()
    assert np.array_equal(v["target_order"], otord)
    assert np.array_equal(v["source_order"], osord)
    assert len(v["cluster_begin"]) == oc.n_source_nodes and len(v["batch_begin"]) == oc.n_target_nodes
    smine = {_key(osord, b, c): i for i, (b, c) in enumerate(zip(v["cluster_begin"], v["cluster_count"]))}
    tmine = {_key(otord, b, c): i for i, (b, c) in enumerate(zip(v["batch_begin"], v["batch_count"]))}
    smap = {}
    for i in range(oc.n_source_nodes):
        nd = oc.node(1, i)
        smap[i] = smine[_key(osord, nd["begin"], nd["count"])]
        assert np.array_equal(v["cluster_lo"][smap[i]], nd["lo"])
    tmap = {}
    for i in range(oc.n_target_nodes):
        nd = oc.node(0, i)
        tmap[i] = tmine[_key(otord, nd["begin"], nd["count"])]
        assert np.array_equal(v["batch_hi"][tmap[i]], nd["hi"])
    t, s, k = oc.pairs()
    # the same pairs in the same (walk) order
    assert np.array_equal(v["item_batch"], np.array([tmap[a] for a in t], dtype=np.int32))
    assert np.array_equal(v["item_cluster"], np.array([smap[b] for b in s], dtype=np.int32))
    assert np.array_equal(v["item_kind"], k)
    st = plan.stats()
    assert st["direct_pairs"] == int(np.sum(k == 3)) and st["approx_pairs"] == int(np.sum(k < 3))
    return plan, oc


@pytest.mark.parametrize("n,theta,degree,leaf,batch", [
    (10000, 0.7, 3, 300, 300),
    (20000, 0.5, 2, 100, 200),
    (8000, 0.9, 4, 400, 64),
    (4000, 0.0, 3, 100, 100),
])
def test_cc_structure_matches_oracle(n, theta, degree, leaf, batch):
    pos, _ = inputs.uniform_cube(n, 500 + n)
    plan, oc = _compare(pos, pos, theta, degree, leaf, batch)
    if theta > 0:
        assert np.sum(oc.pairs()[2] == 0) > 0


def test_cc_structure_distinct_sets():
    g = np.random.default_rng(61)
    tgt = g.uniform(-1, 1, (7000, 3))
    src = g.uniform(-0.5, 1.5, (9000, 3))
    _compare(tgt, src, 0.7, 3, 250, 150)


def test_cc_structure_plummer():
    pos, _ = inputs.plummer_sphere(15000, 62)
    _compare(pos, pos, 0.7, 3, 300, 300)


def test_cc_rejects_several_charge_vectors():
    pos, _ = inputs.uniform_cube(100, 63)
    with pytest.raises(bltc.BLTCError):
        bltc.Plan(_soa(pos), _soa(pos), host=True, method="cc", max_q=2)
