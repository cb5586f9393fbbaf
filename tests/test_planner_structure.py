"""Host-side checks of the library (no GPU): the C ABI loads and exports every
declared symbol, argument checks, and structural parity of the planner's tree,
batches and interaction lists with the oracle's (Alg. 1, eq. 13)."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import paper_2003_01836_amd as bltc
from paper_2003_01836_amd import _capi, inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    lib = _capi.load()
    header = open(os.path.join(ROOT, "include", "bltc.h")).read()
    declared = set(re.findall(r"\b(bltc_[a-z_]+)\s*\(", header))
    assert declared == set(_capi.EXPORTS)
    for name in declared:
        assert hasattr(lib, name), name
    assert b"gfx950" in lib.bltc_version()


def test_status_strings():
    lib = _capi.load()
    for code in (0, -1, -2, -3, -4, -5):
        assert lib.bltc_status_string(code)


def _soa(pos):
    return np.ascontiguousarray(pos.T)


@pytest.mark.parametrize("bad", [
    dict(theta=1.0), dict(theta=-0.1), dict(degree=0), dict(degree=17), dict(leaf_size=0),
    dict(batch_size=0), dict(leaf_size=-1, batch_size=-1), dict(kappa=-1.0), dict(kernel=5),
    dict(precision=7), dict(threads_per_target=3), dict(workspace_limit=-1),
])
def test_invalid_parameters_are_rejected(bad):
    pos, _ = inputs.uniform_cube(100, 1)
    with pytest.raises(bltc.InvalidArgument):
        bltc.Plan(_soa(pos), _soa(pos), host=True, **bad)


def test_zero_sizes_and_threads_on_host_plans():
    # leaf_size = batch_size = 0 asks the tuner, which times plans on the device:
    # a host plan cannot, and says so; threads_per_target = 0 is one lane there
    pos, _ = inputs.uniform_cube(3000, 5)
    with pytest.raises(bltc.BLTCError) as ei:
        bltc.Plan(_soa(pos), _soa(pos), host=True, leaf_size=0, batch_size=0)
    assert ei.value.code == _capi.BLTC_EUNSUPPORTED
    assert "device coordinates" in str(ei.value)
    p = bltc.Plan(_soa(pos), _soa(pos), host=True, leaf_size=300, batch_size=300,
                  threads_per_target=0)
    st = p.stats()
    assert st["threads_per_target"] == 1 and st["leaf_size"] == 300
    # the C defaults: one lane, no workspace limit
    d = _capi.Params()
    _capi.load().bltc_params_default(ctypes.byref(d))
    assert d.threads_per_target == 1 and d.workspace_limit == 0 and d.leaf_size == 2000


def test_workspace_is_not_held_by_host_plans():
    pos, _ = inputs.uniform_cube(3000, 6)
    st = bltc.Plan(_soa(pos), _soa(pos), host=True, leaf_size=200, batch_size=200,
                   workspace_limit=1 << 20).stats()
    # no device side yet: nothing held, no pair rounds planned
    assert st["workspace_bytes"] == 0 and st["pair_rounds"] == 0


@pytest.mark.parametrize("method", ["bltc", "cp", "cc", "hermite"])
def test_fp32_mixed_coordinate_range(method):
    # FP32-mixed kernels square coordinate differences in FP32: points spread
    # over more than 2^60 are refused (FP64 takes them), up to 2^60 accepted
    pos, _ = inputs.uniform_cube(2000, 7)
    deg = 2 if method == "hermite" else 4
    kw = dict(host=True, method=method, leaf_size=200, batch_size=200, degree=deg)
    wide = pos * 2.0 ** 60          # side 2^61
    with pytest.raises(bltc.BLTCError) as ei:
        bltc.Plan(_soa(wide), _soa(wide), precision="fp32_mixed", **kw)
    assert ei.value.code == _capi.BLTC_EUNSUPPORTED and "2^60" in str(ei.value)
    bltc.Plan(_soa(wide), _soa(wide), precision="fp64", **kw)
    ok = pos * 2.0 ** 58            # side 2^59
    bltc.Plan(_soa(ok), _soa(ok), precision="fp32_mixed", **kw)
    # targets and sources apart: the box around both counts
    far = pos.copy()
    far[:, 0] += 2.0 ** 61
    with pytest.raises(bltc.BLTCError) as ei:
        bltc.Plan(_soa(far), _soa(pos), precision="fp32_mixed", **kw)
    assert ei.value.code == _capi.BLTC_EUNSUPPORTED


def test_nonfinite_coordinates_are_rejected():
    pos, _ = inputs.uniform_cube(100, 1)
    pos[17, 1] = np.nan
    with pytest.raises(bltc.InvalidArgument, match="not finite"):
        bltc.Plan(_soa(pos), _soa(pos), host=True)
    pos[17, 1] = np.inf
    with pytest.raises(bltc.InvalidArgument):
        bltc.Plan(_soa(pos), _soa(pos), host=True)


def test_empty_inputs_plan():
    e = np.zeros((3, 0))
    pos, _ = inputs.uniform_cube(50, 2)
    p = bltc.Plan(e, _soa(pos), host=True)
    assert p.stats()["batches"] == 0
    p = bltc.Plan(_soa(pos), e, host=True)
    st = p.stats()
    assert st["clusters"] == 0 and st["approx_pairs"] == 0 and st["direct_pairs"] == 0


def _cluster_key(order, begin, count):
    return tuple(np.sort(order[begin:begin + count]).tolist())


def _compare_with_oracle(tgt, src, theta, degree, leaf, batch, hermite=False):
    plan = bltc.Plan(_soa(tgt), _soa(src), host=True, theta=theta, degree=degree,
                     leaf_size=leaf, batch_size=batch, method="hermite" if hermite else "bltc")
    v = plan.view()
    oc = oracle.Treecode(tgt, src, theta, degree, leaf, batch, hermite=hermite)
    # clusters as sets of source indices, with boxes
    mine = {}
    for c in range(len(v["cluster_begin"])):
        k = _cluster_key(v["source_order"], v["cluster_begin"][c], v["cluster_count"][c])
        mine[k] = (c, v["cluster_lo"][c], v["cluster_hi"][c])
    oorder = oc.source_order()
    theirs = {}
    for c in range(oc.n_clusters):
        info = oc.cluster(c)
        theirs[_cluster_key(oorder, info["begin"], info["count"])] = (c, info["lo"], info["hi"])
    assert set(mine) == set(theirs)
    for k in mine:
        assert np.array_equal(mine[k][1], theirs[k][1]) and np.array_equal(mine[k][2], theirs[k][2])
    # batches as sets of target indices
    bmine = [_cluster_key(v["target_order"], b, c) for b, c in zip(v["batch_begin"], v["batch_count"])]
    otord = oc.target_order()
    btheirs = [_cluster_key(otord, oc.batch(b)["begin"], oc.batch(b)["count"]) for b in range(oc.n_batches)]
    assert set(bmine) == set(btheirs)
    # interaction items
    cmine = {c: k for k, (c, _, _) in mine.items()}
    ctheirs = {c: k for k, (c, _, _) in theirs.items()}
    items_mine = {(bmine[b], cmine[c], kd) for b, c, kd in
                  zip(v["item_batch"], v["item_cluster"], v["item_kind"])}
    ob, occ, ok = oc.items()
    items_theirs = {(btheirs[b], ctheirs[c], kd) for b, c, kd in zip(ob, occ, ok)}
    assert len(items_mine) == len(v["item_batch"])
    assert items_mine == items_theirs
    st = plan.stats()
    assert st["approx_pairs"] == int(np.sum(ok == 0)) and st["direct_pairs"] == int(np.sum(ok == 1))
    return plan, oc


@pytest.mark.parametrize("n,theta,degree,leaf", [
    (10000, 0.7, 4, 500),       # the paper's workload at small scale
    (20000, 0.5, 3, 200),
    (20000, 0.8, 2, 64),
    (5000, 0.0, 4, 100),        # all direct
    (3000, 0.9, 12, 100),       # (n+1)^3 > N: size test fails everywhere
])
def test_structure_matches_oracle_uniform(n, theta, degree, leaf):
    pos, _ = inputs.uniform_cube(n, 100 + n)
    _compare_with_oracle(pos, pos, theta, degree, leaf, leaf)


def test_structure_matches_oracle_plummer():
    pos, _ = inputs.plummer_sphere(20000, 7)
    _compare_with_oracle(pos, pos, 0.7, 4, 300, 300)


def test_structure_matches_oracle_distinct_targets():
    g = np.random.default_rng(5)
    src = g.uniform(-1, 1, (8000, 3))
    tgt = g.uniform(-0.5, 1.5, (6000, 3))
    _compare_with_oracle(tgt, src, 0.7, 3, 150, 90)


def test_structure_with_duplicates_and_lattice():
    v = np.linspace(0.0, 1.0, 9)
    lat = np.array([[a, b, c] for a in v for b in v for c in v])
    pos = np.concatenate([lat, lat[:100]])        # exact duplicates and split-plane ties
    _compare_with_oracle(pos, pos, 0.6, 2, 20, 20)


def test_stats_counts():
    pos, _ = inputs.uniform_cube(10000, 3)
    plan, oc = _compare_with_oracle(pos, pos, 0.7, 4, 500, 500)
    st = plan.stats()
    v = plan.view()
    P = 5 ** 3
    far = sum(v["batch_count"][b] * P for b, k in zip(v["item_batch"], v["item_kind"]) if k == 0)
    near = sum(v["batch_count"][b] * v["cluster_count"][c]
               for b, c, k in zip(v["item_batch"], v["item_cluster"], v["item_kind"]) if k == 1)
    assert st["far_evals"] == far and st["near_evals"] == near
    assert st["batches"] == oc.n_batches and st["clusters"] == oc.n_clusters
    assert st["degree"] == 4 and st["leaf_size"] == 500


# --- barycentric Hermite treecode: same walk, size test against 8 (n+1)^3 ---

@pytest.mark.parametrize("n,theta,degree,leaf", [
    (10000, 0.7, 2, 500),
    (20000, 0.6, 1, 100),
    (20000, 0.8, 3, 700),
    (3000, 0.9, 4, 100),        # 8 (n+1)^3 > N: size test fails everywhere
])
def test_hermite_structure_matches_oracle(n, theta, degree, leaf):
    pos, _ = inputs.uniform_cube(n, 300 + n)
    _compare_with_oracle(pos, pos, theta, degree, leaf, leaf, hermite=True)


def test_hermite_structure_plummer_and_lattice():
    pos, _ = inputs.plummer_sphere(20000, 8)
    _compare_with_oracle(pos, pos, 0.7, 2, 400, 300, hermite=True)
    v = np.linspace(0.0, 1.0, 9)
    lat = np.array([[a, b, c] for a in v for b in v for c in v])
    _compare_with_oracle(lat, lat, 0.6, 1, 80, 20, hermite=True)


def test_hermite_size_test_differs_from_lagrange():
    # clusters with (n+1)^3 < N_C <= 8 (n+1)^3 are approximated by the BLTC only
    pos, _ = inputs.uniform_cube(20000, 9)
    pl, _ = _compare_with_oracle(pos, pos, 0.7, 2, 150, 150)
    ph, _ = _compare_with_oracle(pos, pos, 0.7, 2, 150, 150, hermite=True)
    assert ph.stats()["approx_pairs"] < pl.stats()["approx_pairs"]
    st = ph.stats()
    v = ph.view()
    far = sum(v["batch_count"][b] * 8 * 27 for b, k in zip(v["item_batch"], v["item_kind"]) if k == 0)
    assert st["far_evals"] == far


def test_hermite_unsupported_options_are_rejected():
    pos, _ = inputs.uniform_cube(200, 1)
    t = _soa(pos)
    with pytest.raises(bltc.BLTCError):
        bltc.Plan(t, t, host=True, method="hermite", degree=11)
    with pytest.raises(bltc.BLTCError):
        bltc.Plan(t, t, host=True, method="hermite", max_q=2)
    bltc.Plan(t, t, host=True, method="hermite", degree=10)
    bltc.Plan(t, t, host=True, method="hermite", precision="fp32_mixed")


def test_threads_per_target_options():
    pos, _ = inputs.uniform_cube(300, 2)
    t = _soa(pos)
    for bad in (3, 5, -1):
        with pytest.raises(bltc.BLTCError):
            bltc.Plan(t, t, host=True, threads_per_target=bad)
    # several lanes per target: one-vector BLTC plans only
    with pytest.raises(bltc.BLTCError):
        bltc.Plan(t, t, host=True, threads_per_target=2, method="cp")
    with pytest.raises(bltc.BLTCError):
        bltc.Plan(t, t, host=True, threads_per_target=4, max_q=2)
    for tpt, want in ((0, 1), (1, 1), (2, 2), (4, 4)):
        assert bltc.Plan(t, t, host=True, threads_per_target=tpt).stats()["threads_per_target"] == want
    assert bltc.Plan(t, t, host=True, threads_per_target=2,
                     method="hermite").stats()["threads_per_target"] == 2
