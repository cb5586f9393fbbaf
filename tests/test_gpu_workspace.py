"""Device workspace of a plan (bltc_params.workspace_limit), mutual-pair
results in rounds, parameters left to the tuner (zeros), and the one-shot
batch over plans[].

Rounds change only the order in which each target's mutual-pair terms are
added (per round, then across rounds, in a fixed order), so an FP64 plan
under a limit matches the unlimited plan to rounding order (1e-13 of the
largest potential) and the oracle to the usual 1e-12; FP32-mixed plans are
held to the mixed bounds against the oracle."""
import numpy as np
import pytest

import oracle
from tests.conftest import assert_mixed
from paper_2003_01836_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

BLTC_ENOMEM = -2


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2003_01836_amd as bltc
    bltc.version()
    return torch.device("cuda:0")


def _soa(pos, dev):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(pos, dtype=np.float64).T)).to(dev)


def _close(ref, got, rel_max=1e-12, rel_l2=1e-13):
    scale = np.max(np.abs(ref))
    assert np.all(np.isfinite(got))
    assert np.max(np.abs(ref - got)) <= rel_max * scale, np.max(np.abs(ref - got)) / scale
    assert oracle.rel_l2(ref, got) <= rel_l2


def _limit_for_rounds(st0, fraction):
    """A limit that leaves `fraction` of the one-round pair workspace."""
    return st0["workspace_bytes"] - st0["pair_workspace_bytes"] + int(
        st0["pair_workspace_bytes"] * fraction)


@pytest.mark.parametrize("precision", ["fp64", "fp32_mixed"])
@pytest.mark.parametrize("tpt", [1, 4])
def test_pair_rounds_under_a_limit_match_oracle(dev, precision, tpt):
    import paper_2003_01836_amd as bltc
    pos, q = inputs.uniform_cube(30000, 801)
    t = _soa(pos, dev)
    qd = torch.from_numpy(q[0]).to(dev)
    kw = dict(theta=0.7, degree=5, leaf_size=500, batch_size=500, precision=precision,
              threads_per_target=tpt)
    p0 = bltc.Plan(t, t, **kw)
    st0 = p0.stats()
    assert st0["pair_rounds"] == 1 and st0["mutual_pairs"] > 0
    assert 0 < st0["pair_workspace_bytes"] < st0["workspace_bytes"]
    a = p0.execute(qd).cpu().numpy()
    limit = _limit_for_rounds(st0, 0.35)
    p1 = bltc.Plan(t, t, workspace_limit=limit, **kw)
    st1 = p1.stats()
    print(f"[rounds] {precision} tpt {tpt}: {st1['pair_rounds']} rounds, "
          f"{st1['workspace_bytes']} of {limit} bytes", flush=True)
    assert st1["pair_rounds"] > 1
    assert st1["workspace_bytes"] <= limit
    assert st1["mutual_pairs"] == st0["mutual_pairs"]
    assert st1["mutual_pair_evals"] == st0["mutual_pair_evals"]
    b = p1.execute(qd).cpu().numpy()
    assert np.array_equal(b, p1.execute(qd).cpu().numpy())      # fixed order: repeatable
    ref = oracle.Treecode(pos, pos, 0.7, 5, 500, 500).potential(q[0])
    if precision == "fp64":
        _close(a, b, 1e-13, 1e-14)
        _close(ref, b)
    else:
        assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(a))
        assert_mixed(ref, b, pos, pos, q[0], what=f"rounds tpt {tpt}")


@pytest.mark.parametrize("method", ["cc", "cp", "hermite"])
def test_pair_rounds_other_methods(dev, method):
    import paper_2003_01836_amd as bltc
    pos, q = inputs.uniform_cube(30000, 802)
    t = _soa(pos, dev)
    qd = torch.from_numpy(q[0]).to(dev)
    deg = 3 if method == "hermite" else 4
    kw = dict(method=method, theta=0.7, degree=deg, leaf_size=400, batch_size=400)
    p0 = bltc.Plan(t, t, **kw)
    st0 = p0.stats()
    assert st0["mutual_pairs"] > 0
    p1 = bltc.Plan(t, t, workspace_limit=_limit_for_rounds(st0, 0.4), **kw)
    assert p1.stats()["pair_rounds"] > 1
    a = p0.execute(qd).cpu().numpy()
    b = p1.execute(qd).cpu().numpy()
    _close(a, b, 1e-13, 1e-14)
    if method == "cc":
        ref = oracle.ClusterCluster(pos, pos, 0.7, deg, 400, 400).potential(q[0])
    elif method == "cp":
        ref = oracle.ClusterParticle(pos, pos, 0.7, deg, 400, 400).potential(q[0])
    else:
        ref = oracle.Treecode(pos, pos, 0.7, deg, 400, 400, hermite=True).potential(q[0])
    _close(ref, b)


def test_workspace_limit_below_what_the_plan_needs(dev):
    import paper_2003_01836_amd as bltc
    pos, q = inputs.uniform_cube(30000, 803)
    t = _soa(pos, dev)
    qd = torch.from_numpy(q[0]).to(dev)
    kw = dict(theta=0.7, degree=5, leaf_size=500, batch_size=500)
    st0 = bltc.Plan(t, t, **kw).stats()
    # far below the plan's own arrays
    with pytest.raises(bltc.BLTCError) as ei:
        bltc.Plan(t, t, workspace_limit=4096, **kw)
    assert ei.value.code == BLTC_ENOMEM and "workspace_limit" in str(ei.value)
    # the arrays fit, the mutual-pair results of the largest pair do not
    with pytest.raises(bltc.BLTCError) as ei:
        bltc.Plan(t, t, workspace_limit=st0["workspace_bytes"] - st0["pair_workspace_bytes"] + 1024,
                  **kw)
    assert ei.value.code == BLTC_ENOMEM and "mutual leaf pair" in str(ei.value)
    # ... which runs without the mutual pairs
    p = bltc.Plan(t, t, symmetry=False,
                  workspace_limit=st0["workspace_bytes"] - st0["pair_workspace_bytes"] + 1024, **kw)
    assert p.stats()["mutual_pairs"] == 0
    ref = oracle.Treecode(pos, pos, 0.7, 5, 500, 500).potential(q[0])
    _close(ref, p.execute(qd).cpu().numpy())
    # the device is fine afterwards: a plan without a limit evaluates as usual
    _close(ref, bltc.Plan(t, t, **kw).execute(qd).cpu().numpy())
    # a limit on a one-shot evaluation
    with pytest.raises(bltc.BLTCError) as ei:
        bltc.potential(t, t, qd, workspace_limit=4096, **kw)
    assert ei.value.code == BLTC_ENOMEM


def test_zero_sizes_and_threads_are_tuned(dev, tmp_path, monkeypatch):
    import paper_2003_01836_amd as bltc
    monkeypatch.setenv("BLTC_TUNE_CACHE", str(tmp_path / "tune.txt"))
    pos, q = inputs.uniform_cube(60000, 804)
    t = _soa(pos, dev)
    qd = torch.from_numpy(q[0]).to(dev)
    p = bltc.Plan(t, t, leaf_size=0, batch_size=0, threads_per_target=0, degree=4, theta=0.7)
    st = p.stats()
    assert st["leaf_size"] == st["batch_size"] and st["leaf_size"] in (1000, 2000, 3000, 4000)
    assert st["threads_per_target"] in (1, 2, 4)
    assert (tmp_path / "tune.txt").exists()
    phi = p.execute(qd).cpu().numpy()
    ref = oracle.Treecode(pos, pos, 0.7, 4, st["leaf_size"], st["leaf_size"]).potential(q[0])
    _close(ref, phi)
    # the one-shot call takes the cached choice: the same plan, the same bits
    one = bltc.potential(t, t, qd, leaf_size=0, batch_size=0, threads_per_target=0, degree=4,
                         theta=0.7).cpu().numpy()
    assert np.array_equal(one, phi)
    # threads per target alone, at fixed (unequal) sizes
    g = np.random.default_rng(805)
    tgt = g.uniform(-1, 1, (20000, 3))
    p2 = bltc.Plan(_soa(tgt, dev), t, leaf_size=1500, batch_size=700, threads_per_target=0,
                   degree=4, theta=0.7)
    st2 = p2.stats()
    assert (st2["leaf_size"], st2["batch_size"]) == (1500, 700)
    assert st2["threads_per_target"] in (1, 2, 4)
    ref2 = oracle.Treecode(tgt, pos, 0.7, 4, 1500, 700).potential(q[0])
    _close(ref2, p2.execute(qd).cpu().numpy())
    # several charge vectors: sizes tuned, threads per target stays one lane
    p3 = bltc.Plan(t, t, leaf_size=0, batch_size=0, threads_per_target=0, degree=4, theta=0.7,
                   max_q=16)
    st3 = p3.stats()
    assert st3["leaf_size"] in (1000, 2000, 3000, 4000) and st3["threads_per_target"] == 1


def test_batch_potential_over_plans_matches_batch(dev):
    import paper_2003_01836_amd as bltc
    plans, qs = [], []
    for k, n in enumerate((3000, 11000, 700)):
        pos, q = inputs.uniform_cube(n, 806 + k, m=16)
        t = _soa(pos, dev)
        plans.append(bltc.Plan(t, t, theta=0.7, degree=5, leaf_size=300, batch_size=300, max_q=16))
        qs.append(torch.from_numpy(np.ascontiguousarray(q[: 16 - 5 * k])).to(dev))
    a = [o.cpu().numpy() for o in bltc.Batch(plans).execute(qs)]
    b = [o.cpu().numpy() for o in bltc.batch_potential(plans, qs)]
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    pos, q = inputs.uniform_cube(700, 808, m=16)
    ref = oracle.Treecode(pos, pos, 0.7, 5, 300, 300).potential(q[:6])
    for i in range(6):
        _close(ref[i], b[2][i])
