"""Cluster-particle plans on the host: trees, source batches and interaction
items against the oracle's cluster-particle treecode (CPU only)."""
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
    plan = bltc.Plan(th, sh, host=True, method="cp", theta=theta, degree=degree, leaf_size=leaf,
                     batch_size=batch)
    v = plan.view()
    oc = oracle.ClusterParticle(tgt, src, theta, degree, leaf, batch)
    assert np.array_equal(v["target_order"], oc.target_order())
    assert np.array_equal(v["source_order"], oc.source_order())
    assert len(v["cluster_begin"]) == oc.n_clusters and len(v["batch_begin"]) == oc.n_batches
    # target clusters matched by their member sets, with identical boxes
    tord = v["target_order"]
    mine = {_key(tord, b, c): i for i, (b, c) in enumerate(zip(v["cluster_begin"], v["cluster_count"]))}
    theirs = {}
    for i in range(oc.n_clusters):
        info = oc.cluster(i)
        theirs[i] = mine[_key(tord, info["begin"], info["count"])]
        assert np.array_equal(v["cluster_lo"][theirs[i]], info["lo"])
        assert np.array_equal(v["cluster_hi"][theirs[i]], info["hi"])
    for b in range(oc.n_batches):
        ob = oc.batch(b)
        assert (v["batch_begin"][b], v["batch_count"][b]) == (ob["begin"], ob["count"])
    # items: the same (source batch, target cluster, kind) triples (the plan
    # stores a batch's approximations before its direct pairs)
    ob, oc_, ok = oc.items()
    mine_items = sorted(zip(v["item_batch"].tolist(), v["item_kind"].tolist(), v["item_cluster"].tolist()))
    their_items = sorted(zip(ob.tolist(), ok.tolist(), [theirs[c] for c in oc_]))
    assert mine_items == their_items
    st = plan.stats()
    P = (degree + 1) ** 3
    assert st["approx_pairs"] == int(np.sum(ok == 0)) and st["direct_pairs"] == int(np.sum(ok == 1))
    far = sum(P * v["batch_count"][b] for b, k in zip(v["item_batch"], v["item_kind"]) if k == 0)
    near = sum(v["cluster_count"][c] * v["batch_count"][b]
               for b, c, k in zip(v["item_batch"], v["item_cluster"], v["item_kind"]) if k == 1)
    assert st["far_evals"] == far and st["near_evals"] == near
    return plan, oc


@pytest.mark.parametrize("n,theta,degree,leaf,batch", [
    (10000, 0.7, 4, 500, 500),
    (20000, 0.5, 3, 200, 120),
    (8000, 0.9, 6, 400, 64),
    (4000, 0.0, 4, 100, 100),
])
def test_cp_structure_matches_oracle(n, theta, degree, leaf, batch):
    pos, _ = inputs.uniform_cube(n, 300 + n)
    _compare(pos, pos, theta, degree, leaf, batch)


def test_cp_structure_distinct_sets():
    g = np.random.default_rng(31)
    tgt = g.uniform(-1, 1, (7000, 3))
    src = g.uniform(-0.5, 1.5, (9000, 3))
    _compare(tgt, src, 0.7, 4, 150, 250)


def test_cp_structure_plummer():
    pos, _ = inputs.plummer_sphere(15000, 32)
    _compare(pos, pos, 0.7, 4, 300, 300)


def test_cp_rejects_several_charge_vectors():
    pos, _ = inputs.uniform_cube(100, 33)
    with pytest.raises(bltc.BLTCError):
        bltc.Plan(_soa(pos), _soa(pos), host=True, method="cp", max_q=2)
