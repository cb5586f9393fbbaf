"""GPU parity: the HIP path through the C ABI against the CPU oracle.

FP64 path bar: the library and the oracle evaluate the same tree, batches and
lists (structural parity is tested on the host), so they differ only in the
order of rounding (two-step modified charges of eqs. 14-15 versus eq. 12;
refined hardware 1/sqrt versus sqrt and divide).  Per-element differences are
bounded relative to the largest potential: max|d| <= 1e-12 * max|phi|, and the
relative 2-norm difference (eq. 16) <= 1e-13.  These bounds are far inside the
1e-6 relative-L2 target.
"""
import numpy as np
import pytest

import oracle
from tests.conftest import EPS32, KERNEL_CASES, assert_mixed, kernel_kwargs
from paper_2003_01836_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

REL_MAX = 1e-12
REL_L2 = 1e-13


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2003_01836_amd as bltc
    bltc.version()   # fails loudly if the HIP library is missing
    return torch.device("cuda:0")


def _dev_soa(pos, dev):
    return torch.from_numpy(np.ascontiguousarray(pos.T)).to(dev)


def _close(ref, got, rel_max=REL_MAX, rel_l2=REL_L2):
    ref = np.asarray(ref)
    got = np.asarray(got)
    scale = np.max(np.abs(ref)) if ref.size else 1.0
    assert np.all(np.isfinite(got))
    assert np.max(np.abs(ref - got)) <= rel_max * max(scale, 1e-300), np.max(np.abs(ref - got)) / scale
    assert oracle.rel_l2(ref, got) <= rel_l2


def _run_plan(dev, tgt, src, q, **kw):
    import paper_2003_01836_amd as bltc
    t = _dev_soa(tgt, dev)
    s = t if src is tgt else _dev_soa(src, dev)
    qd = torch.from_numpy(np.ascontiguousarray(q)).to(dev)
    plan = bltc.Plan(t, s, max_q=(q.shape[0] if q.ndim == 2 else 1), **kw)
    phi = plan.execute(qd)
    torch.cuda.synchronize()
    return plan, phi.cpu().numpy()


@pytest.mark.parametrize("kernel,kappa", KERNEL_CASES)
def test_gpu_direct_sum_matches_oracle(dev, kernel, kappa):
    import paper_2003_01836_amd as bltc
    pos, q = inputs.uniform_cube(3001, 71)
    t = _dev_soa(pos, dev)
    phi = bltc.direct(t, t, torch.from_numpy(q[0]).to(dev), **kernel_kwargs(kernel, kappa)[0])
    ref = oracle.direct(pos, pos, q[0], kernel=kernel_kwargs(kernel, kappa)[1], kappa=kappa)
    _close(ref, phi.cpu().numpy(), 1e-13, 1e-14)


@pytest.mark.parametrize("kernel,kappa", KERNEL_CASES)
def test_fp64_treecode_small_config(dev, kernel, kappa):
    # N = 10^4 uniform cube, theta 0.7, n = 4, N_L = N_B = 500 (several tiles, ragged batches)
    pos, q = inputs.uniform_cube(10000, inputs.config_seed(0))
    plan, phi = _run_plan(dev, pos, pos, q[0], theta=0.7, degree=4, leaf_size=500, batch_size=500,
                          **kernel_kwargs(kernel, kappa)[0])
    oc = oracle.Treecode(pos, pos, 0.7, 4, 500, 500)
    kern = kernel_kwargs(kernel, kappa)[1]
    ref = oc.potential(q[0], kernel=kern, kappa=kappa)
    _close(ref, phi)
    # the method error itself (eq. 16) is the oracle's
    d = oracle.direct(pos, pos, q[0], kernel=kern, kappa=kappa)
    assert abs(oracle.rel_l2(d, phi) - oracle.rel_l2(d, ref)) <= 1e-3 * oracle.rel_l2(d, ref)


def test_fp64_modified_charges_match_oracle(dev):
    pos, q = inputs.uniform_cube(20000, 72)
    plan, _ = _run_plan(dev, pos, pos, q[0], theta=0.7, degree=5, leaf_size=300, batch_size=300)
    oc = oracle.Treecode(pos, pos, 0.7, 5, 300, 300)
    v = plan.view()
    okey = {}
    oorder = oc.source_order()
    for c in range(oc.n_clusters):
        info = oc.cluster(c)
        okey[tuple(np.sort(oorder[info["begin"]:info["begin"] + info["count"]]))] = c
    checked = 0
    for c in np.unique(v["item_cluster"][v["item_kind"] == 0]):
        key = tuple(np.sort(v["source_order"][v["cluster_begin"][c]:v["cluster_begin"][c] + v["cluster_count"][c]]))
        ref = oc.modified_charges(okey[key], q[0])
        got = plan.modified_charges(c)
        assert np.max(np.abs(ref - got)) <= 1e-12 * np.max(np.abs(ref)), c
        checked += 1
    assert checked > 10


def test_gpu_parent_modified_charges_from_children(dev):
    # The parent's Lagrange polynomials have degree n in each variable, so
    # interpolating the children's modified charges onto the parent's grid
    # reproduces the parent's: q^P_k = sum_child sum_m prod_l L^P_kl(s^child_ml) q^child_m.
    # Checks the device upward pass level against level, with no oracle q-hat.
    n = 4
    pos, q = inputs.uniform_cube(120000, 73)
    plan, _ = _run_plan(dev, pos, pos, q[0], theta=0.7, degree=n, leaf_size=150, batch_size=150)
    v = plan.view()
    have = set(np.unique(v["item_cluster"][v["item_kind"] == 0]).tolist())
    _, w = oracle.chebyshev(n)

    def nodes(c):
        return [oracle.chebyshev(n, v["cluster_lo"][c][d], v["cluster_hi"][c][d])[0] for d in range(3)]

    checked = 0
    for p in sorted(have):
        nk = v["cluster_nchild"][p]
        kids = list(range(v["cluster_first_child"][p], v["cluster_first_child"][p] + nk)) if nk > 0 else []
        if not kids or not all(k in have for k in kids):
            continue
        sp = nodes(p)
        total = np.zeros((n + 1,) * 3)
        for ch in kids:
            sc = nodes(ch)
            T = [np.array([oracle.lagrange(n, sp[d], w, x) for x in sc[d]]) for d in range(3)]
            total += np.einsum("ai,bj,ck,abc->ijk", T[0], T[1], T[2],
                               plan.modified_charges(ch).reshape((n + 1,) * 3))
        qp = plan.modified_charges(p).reshape((n + 1,) * 3)
        assert np.max(np.abs(total - qp)) <= 1e-11 * np.max(np.abs(qp)), p
        checked += 1
        if checked == 6:
            break
    assert checked >= 1


@pytest.mark.parametrize("degree", [1, 2, 3, 6, 8, 11, 16])
def test_fp64_all_degrees(dev, degree):
    pos, q = inputs.uniform_cube(6000, 80 + degree)
    leaf = max(64, min(1500, (degree + 1) ** 3 + 50))
    _, phi = _run_plan(dev, pos, pos, q[0], theta=0.8, degree=degree, leaf_size=leaf, batch_size=leaf)
    ref = oracle.Treecode(pos, pos, 0.8, degree, leaf, leaf).potential(q[0])
    _close(ref, phi)


def test_fp64_distinct_targets_and_sources(dev):
    g = np.random.default_rng(9)
    src = g.uniform(-1, 1, (12000, 3))
    tgt = g.uniform(-0.3, 1.4, (7001, 3))
    q = g.uniform(-1, 1, 12000)
    _, phi = _run_plan(dev, tgt, src, q, theta=0.6, degree=6, leaf_size=400, batch_size=333)
    ref = oracle.Treecode(tgt, src, 0.6, 6, 400, 333).potential(q)
    _close(ref, phi)


def test_fp64_plummer_yukawa(dev):
    pos, q = inputs.plummer_sphere(30000, 73)
    _, phi = _run_plan(dev, pos, pos, q[0], theta=0.7, degree=6, leaf_size=400, batch_size=400,
                       kernel="yukawa", kappa=0.5)
    ref = oracle.Treecode(pos, pos, 0.7, 6, 400, 400).potential(q[0], kernel=oracle.YUKAWA, kappa=0.5)
    _close(ref, phi)


def test_fp64_theta_zero_is_direct_sum(dev):
    pos, q = inputs.uniform_cube(4000, 74)
    _, phi = _run_plan(dev, pos, pos, q[0], theta=0.0, degree=4, leaf_size=100, batch_size=100)
    _close(oracle.direct(pos, pos, q[0]), phi)


def test_fp64_multiple_charge_vectors(dev):
    pos, q = inputs.uniform_cube(8000, 75, m=3)
    _, phi = _run_plan(dev, pos, pos, q, theta=0.7, degree=4, leaf_size=300, batch_size=300)
    oc = oracle.Treecode(pos, pos, 0.7, 4, 300, 300)
    ref = oc.potential(q)
    for m in range(3):
        _close(ref[m], phi[m])


def test_fp64_repeatable_bitwise(dev):
    import paper_2003_01836_amd as bltc
    pos, q = inputs.uniform_cube(20000, 76)
    t = _dev_soa(pos, dev)
    qd = torch.from_numpy(q[0]).to(dev)
    plan = bltc.Plan(t, t, theta=0.7, degree=6, leaf_size=500, batch_size=500)
    a = plan.execute(qd).cpu().numpy()
    b = plan.execute(qd).cpu().numpy()
    assert np.array_equal(a, b)


@pytest.mark.parametrize("precision", ["fp64", "fp32_mixed"])
def test_edge_cases(dev, precision):
    import functools
    import paper_2003_01836_amd as bltc
    bltc_potential = bltc.potential
    bltc = type("B", (), {"potential": staticmethod(functools.partial(bltc_potential, precision=precision))})
    pos, q = inputs.uniform_cube(500, 77)
    t = _dev_soa(pos, dev)
    qd = torch.from_numpy(q[0]).to(dev)
    empty = torch.zeros((3, 0), dtype=torch.float64, device=dev)
    # no sources: potentials are zero
    phi = bltc.potential(t, empty, torch.zeros(0, dtype=torch.float64, device=dev))
    assert phi.shape == (500,) and torch.all(phi == 0)
    # no targets: nothing to do
    phi = bltc.potential(empty, t, qd)
    assert phi.shape == (0,)
    # one particle: its own potential is zero (self pair skipped)
    one = t[:, :1].contiguous()
    phi = bltc.potential(one, one, qd[:1].contiguous())
    assert phi.item() == 0.0
    # identical particles: every pair at zero distance
    same = torch.full((3, 300), 0.25, dtype=torch.float64, device=dev)
    phi = bltc.potential(same, same, torch.ones(300, dtype=torch.float64, device=dev), leaf_size=10,
                         batch_size=10)
    assert torch.all(phi == 0)
    # duplicates among distinct points
    dup = np.concatenate([pos, pos[:50]])
    qq = np.concatenate([q[0], q[0][:50]])
    phi = bltc.potential(_dev_soa(dup, dev), _dev_soa(dup, dev), torch.from_numpy(qq).to(dev),
                         theta=0.5, degree=2, leaf_size=40, batch_size=40)
    ref = oracle.Treecode(dup, dup, 0.5, 2, 40, 40).potential(qq)
    if precision == "fp64":
        _close(ref, phi.cpu().numpy())
    else:
        assert_mixed(ref, phi.cpu().numpy(), dup, dup, qq, what="duplicates")
    # isolated particles: one-particle leaves and batches (zero-extent boxes)
    g = np.random.default_rng(3)
    iso = np.concatenate([g.uniform(-1, 1, (300, 3)), g.uniform(-1, 1, (20, 3)) * 50.0])
    qi = g.uniform(-1, 1, len(iso))
    ti = _dev_soa(iso, dev)
    phi = bltc.potential(ti, ti, torch.from_numpy(qi).to(dev), theta=0.7, degree=2, leaf_size=30,
                         batch_size=30, kernel="yukawa", kappa=0.5)
    ref = oracle.Treecode(iso, iso, 0.7, 2, 30, 30).potential(qi, kernel=oracle.YUKAWA, kappa=0.5)
    got = phi.cpu().numpy()
    assert np.all(np.isfinite(got))
    if precision == "fp64":
        assert oracle.rel_l2(ref, got) <= 1e-13
    else:
        assert_mixed(ref, got, iso, iso, qi, oracle.YUKAWA, 0.5, what="isolated")


def test_invalid_arguments_on_device(dev):
    import paper_2003_01836_amd as bltc
    pos, q = inputs.uniform_cube(100, 78)
    t = _dev_soa(pos, dev)
    bad = t.clone()
    bad[0, 5] = float("nan")
    with pytest.raises(bltc.InvalidArgument):
        bltc.Plan(bad, bad)
    plan = bltc.Plan(t, t, max_q=1)
    with pytest.raises(bltc.InvalidArgument):
        plan.execute(torch.zeros((2, 100), dtype=torch.float64, device=dev))


@pytest.fixture(scope="module")
def uniform_1m():
    """The benchmark workload: N = 10^6 uniform cube, theta 0.7, n = 8, N_L = N_B = 2000;
    the oracle evaluates 1000 sampled targets through their own batches."""
    n = 1_000_000
    pos, q = inputs.uniform_cube(n, inputs.config_seed(1))
    smp = inputs.sample_indices(n, 1000, inputs.sample_seed(1))
    ref = oracle.Treecode(pos, pos, 0.7, 8, 2000, 2000).potential(q[0], sample=smp)
    return pos, q, smp, ref


def test_fp64_full_size_sampled(dev, uniform_1m):
    pos, q, smp, ref = uniform_1m
    _, phi = _run_plan(dev, pos, pos, q[0], theta=0.7, degree=8, leaf_size=2000, batch_size=2000)
    _close(ref, phi[smp])


@pytest.mark.parametrize("precision", ["fp64", "fp32_mixed"])
def test_benchmark_plan_four_threads_per_target(dev, uniform_1m, precision):
    # the plan the benchmark times: 4 lanes per target, mutual leaf pairs on
    pos, q, smp, ref = uniform_1m
    plan, phi = _run_plan(dev, pos, pos, q[0], theta=0.7, degree=8, leaf_size=2000,
                          batch_size=2000, threads_per_target=4, precision=precision)
    st = plan.stats()
    assert st["threads_per_target"] == 4 and st["mutual_pairs"] > 0 and st["pair_rounds"] == 1
    if precision == "fp64":
        _close(ref, phi[smp])
    else:
        assert_mixed(ref, phi[smp], pos, pos, q[0], idx=smp, what="1M 4 lanes per target")


@pytest.mark.parametrize("precision", ["fp64", "fp32_mixed"])
def test_benchmark_points_sixteen_vectors(dev, precision):
    # the multi-vector plan of the multi-1M benchmark: the headline points with
    # 16 charge vectors; the oracle's treecode on the sampled targets, vectors
    # 0, 7 and 15 (vector 0 is the headline's charge vector)
    import paper_2003_01836_amd as bltc
    n, m = 1_000_000, 16
    pos, q = inputs.uniform_cube(n, inputs.config_seed(1), m=m)
    smp = inputs.sample_indices(n, 1000, inputs.sample_seed(1))
    vec = [0, 7, 15]
    ref = oracle.Treecode(pos, pos, 0.7, 8, 2000, 2000).potential(q[vec], sample=smp)
    t = _dev_soa(pos, dev)
    plan = bltc.Plan(t, t, theta=0.7, degree=8, leaf_size=2000, batch_size=2000, max_q=m,
                     precision=precision)
    phi = plan.execute(torch.from_numpy(np.ascontiguousarray(q)).to(dev))
    torch.cuda.synchronize()
    got = phi.cpu().numpy()
    for i, v in enumerate(vec):
        if precision == "fp64":
            _close(ref[i], got[v][smp])
        else:
            assert_mixed(ref[i], got[v][smp], pos, pos, q[v], idx=smp, what=f"1M vector {v}")


# --------------------------------------------------------------------------
# FP32-mixed path against the FP64 oracle: relative 2-norm <= 1e-6, largest
# difference <= 1e-5 of the largest potential, and per target at most a stated
# multiple of eps32 * sum_j |G q_j| (tests/conftest.py: assert_mixed)
# --------------------------------------------------------------------------
MIXED_REL_L2 = 1e-6


@pytest.mark.parametrize("kernel,kappa", KERNEL_CASES)
def test_mixed_small_config(dev, kernel, kappa):
    pos, q = inputs.uniform_cube(10000, inputs.config_seed(0))
    _, phi = _run_plan(dev, pos, pos, q[0], theta=0.7, degree=4, leaf_size=500, batch_size=500,
                       **kernel_kwargs(kernel, kappa)[0], precision="fp32_mixed")
    kern = kernel_kwargs(kernel, kappa)[1]
    ref = oracle.Treecode(pos, pos, 0.7, 4, 500, 500).potential(q[0], kernel=kern, kappa=kappa)
    assert_mixed(ref, phi, pos, pos, q[0], kern, kappa, what=kernel)
    d = oracle.direct(pos, pos, q[0], kernel=kern, kappa=kappa)
    # equal accuracy: the treecode error is not made worse by the FP32 arithmetic
    assert oracle.rel_l2(d, phi) <= 1.1 * oracle.rel_l2(d, ref)


@pytest.mark.parametrize("degree", [1, 4, 8, 12, 16])
def test_mixed_all_degrees(dev, degree):
    pos, q = inputs.uniform_cube(6000, 90 + degree)
    leaf = max(64, min(1500, (degree + 1) ** 3 + 50))
    _, phi = _run_plan(dev, pos, pos, q[0], theta=0.8, degree=degree, leaf_size=leaf,
                       batch_size=leaf, precision="fp32_mixed")
    ref = oracle.Treecode(pos, pos, 0.8, degree, leaf, leaf).potential(q[0])
    assert_mixed(ref, phi, pos, pos, q[0], what=f"n={degree}")


def test_mixed_planted_close_pairs(dev):
    # pairs at separations 1e-7 .. 1e-3 and exact duplicates take the FP64 branch
    g = np.random.default_rng(12)
    base, q = inputs.uniform_cube(20000, 91)
    k = 400
    offs = g.standard_normal((k, 3))
    offs *= (10.0 ** g.uniform(-7, -3, k) / np.linalg.norm(offs, axis=1))[:, None]
    pos = np.concatenate([base, base[:k] + offs, base[k:k + 50]])
    qq = np.concatenate([q[0], g.uniform(-1, 1, k + 50)])
    _, phi = _run_plan(dev, pos, pos, qq, theta=0.7, degree=6, leaf_size=600, batch_size=600,
                       precision="fp32_mixed")
    ref = oracle.Treecode(pos, pos, 0.7, 6, 600, 600).potential(qq)
    assert_mixed(ref, phi, pos, pos, qq, what="planted")
    close = np.arange(len(base) - 0, len(base) + k)
    # the planted targets themselves, where the close terms dominate
    assert_mixed(ref[close], phi[close], pos, pos, qq, idx=close, what="planted targets")


def test_mixed_plummer_yukawa(dev):
    pos, q = inputs.plummer_sphere(30000, 93)
    _, phi = _run_plan(dev, pos, pos, q[0], theta=0.7, degree=6, leaf_size=400, batch_size=400,
                       kernel="yukawa", kappa=0.5, precision="fp32_mixed")
    ref = oracle.Treecode(pos, pos, 0.7, 6, 400, 400).potential(q[0], kernel=oracle.YUKAWA, kappa=0.5)
    assert_mixed(ref, phi, pos, pos, q[0], oracle.YUKAWA, 0.5, what="plummer yukawa")


def test_mixed_distinct_targets_and_multiple_vectors(dev):
    g = np.random.default_rng(19)
    src = g.uniform(-1, 1, (12000, 3))
    tgt = g.uniform(-0.3, 1.4, (7001, 3))
    q = g.uniform(-1, 1, (2, 12000))
    _, phi = _run_plan(dev, tgt, src, q, theta=0.6, degree=6, leaf_size=400, batch_size=333,
                       precision="fp32_mixed")
    ref = oracle.Treecode(tgt, src, 0.6, 6, 400, 333).potential(q)
    for m in range(2):
        assert_mixed(ref[m], phi[m], tgt, src, q[m], what=f"vector {m}")


def test_mixed_full_size_sampled_and_full_n_vs_fp64(dev, uniform_1m):
    # the benchmark workload; FP32-mixed against the oracle on 1000 sampled targets, and
    # against the GPU FP64 path (itself parity-checked above) on all 10^6 targets
    pos, q, smp, ref = uniform_1m
    _, mixed = _run_plan(dev, pos, pos, q[0], theta=0.7, degree=8, leaf_size=2000, batch_size=2000,
                         precision="fp32_mixed")
    _, full = _run_plan(dev, pos, pos, q[0], theta=0.7, degree=8, leaf_size=2000, batch_size=2000)
    assert_mixed(ref, mixed[smp], pos, pos, q[0], idx=smp, what="1M sampled")
    # every target against the FP64 path: norm and largest difference
    assert_mixed(full, mixed, what="1M full-N vs FP64")


# --------------------------------------------------------------------------
# several charge vectors: kernel values shared, contraction on the matrix cores
# --------------------------------------------------------------------------
@pytest.mark.parametrize("m", [2, 16, 21])
@pytest.mark.parametrize("kernel,kappa", KERNEL_CASES)
def test_fp64_many_charge_vectors(dev, m, kernel, kappa):
    pos, q = inputs.uniform_cube(9001, 100 + m, m=m)
    _, phi = _run_plan(dev, pos, pos, q, theta=0.7, degree=5, leaf_size=400, batch_size=400,
                       **kernel_kwargs(kernel, kappa)[0])
    kern = kernel_kwargs(kernel, kappa)[1]
    ref = oracle.Treecode(pos, pos, 0.7, 5, 400, 400).potential(q, kernel=kern, kappa=kappa)
    for i in range(m):
        _close(ref[i], phi[i])


@pytest.mark.parametrize("m", [3, 16])
@pytest.mark.parametrize("kernel,kappa", KERNEL_CASES)
def test_mixed_many_charge_vectors(dev, m, kernel, kappa):
    pos, q = inputs.uniform_cube(9001, 120 + m, m=m)
    _, phi = _run_plan(dev, pos, pos, q, theta=0.7, degree=6, leaf_size=400, batch_size=400,
                       **kernel_kwargs(kernel, kappa)[0], precision="fp32_mixed")
    kern = kernel_kwargs(kernel, kappa)[1]
    ref = oracle.Treecode(pos, pos, 0.7, 6, 400, 400).potential(q, kernel=kern, kappa=kappa)
    for i in range(m):
        assert_mixed(ref[i], phi[i], pos, pos, q[i], kern, kappa, what=f"{kernel} vector {i}")


@pytest.mark.parametrize("precision", ["fp64", "fp32_mixed"])
@pytest.mark.parametrize("degree,leaf", [(1, 3), (1, 13), (2, 7), (3, 25)])
def test_many_vectors_short_lists(dev, precision, degree, leaf):
    """Source lists and proxy grids (8, 27, 64 points) shorter than a round of
    the multi-vector kernels' prefetch (3 steps of 4 sources on the FP32 path),
    through one plan and through a work-queue batch of two systems: the
    padded steps must carry zero charges."""
    import paper_2003_01836_amd as bltc
    systems = [inputs.uniform_cube(n, 140 + leaf + n, m=16) for n in (3001, 1207)]
    refs = [oracle.Treecode(pos, pos, 0.7, degree, leaf, leaf).potential(q) for pos, q in systems]

    def check(ref, got, pos, q):
        for i in range(16):
            if precision == "fp64":
                _close(ref[i], got[i])
            else:
                assert_mixed(ref[i], got[i], pos, pos, q[i], what=f"vector {i}")

    pos, q = systems[0]
    _, phi = _run_plan(dev, pos, pos, q, theta=0.7, degree=degree, leaf_size=leaf,
                       batch_size=leaf, precision=precision)
    check(refs[0], phi, pos, q)
    plans, qd, outs = [], [], []
    for pos, q in systems:
        t = _dev_soa(pos, dev)
        plans.append(bltc.Plan(t, t, theta=0.7, degree=degree, leaf_size=leaf, batch_size=leaf,
                               max_q=16, precision=precision))
        qd.append(torch.from_numpy(np.ascontiguousarray(q)).to(dev))
        outs.append(torch.full((16, pos.shape[0]), float("nan"), dtype=torch.float64, device=dev))
    bltc.Batch(plans).execute(qd, outs)
    torch.cuda.synchronize()
    for ref, o, (pos, q) in zip(refs, outs, systems):
        check(ref, o.cpu().numpy(), pos, q)


def test_many_vectors_plummer_distinct_targets(dev):
    g = np.random.default_rng(29)
    src, q = inputs.plummer_sphere(15000, 131, m=16)
    tgt = g.uniform(-2, 2, (5003, 3))
    for precision in ("fp64", "fp32_mixed"):
        _, phi = _run_plan(dev, tgt, src, q, theta=0.7, degree=7, leaf_size=700, batch_size=300,
                           precision=precision)
        ref = oracle.Treecode(tgt, src, 0.7, 7, 700, 300).potential(q)
        for i in range(16):
            if precision == "fp64":
                _close(ref[i], phi[i])
            else:
                assert_mixed(ref[i], phi[i], tgt, src, q[i], what=f"vector {i}")


@pytest.mark.parametrize("m", [1, 16])
def test_modified_charges_multi_chunk_clusters(dev, m):
    # clusters larger than one upward-pass chunk (8192 sources) are summed over chunks
    pos, q = inputs.uniform_cube(40000, 140 + m, m=m)
    # a near target cloud and a distant one: the root (5 chunks) and its children are approximated
    g = np.random.default_rng(140 + m)
    tgt = np.concatenate([g.uniform(-1, 1, (3000, 3)), g.uniform(-1, 1, (3000, 3)) + [8.0, 1.0, 0.0]])
    plan, _ = _run_plan(dev, tgt, pos, q if m > 1 else q[0], theta=0.9, degree=4, leaf_size=2000,
                        batch_size=2000)
    oc = oracle.Treecode(tgt, pos, 0.9, 4, 2000, 2000)
    v = plan.view()
    oorder = oc.source_order()
    okey = {}
    for c in range(oc.n_clusters):
        info = oc.cluster(c)
        okey[tuple(np.sort(oorder[info["begin"]:info["begin"] + info["count"]]))] = c
    approx = np.unique(v["item_cluster"][v["item_kind"] == 0])
    big = [c for c in approx if v["cluster_count"][c] > 8192]
    assert big, "the test needs clusters that span several chunks"
    for c in list(big) + list(approx[:5]):
        key = tuple(np.sort(v["source_order"][v["cluster_begin"][c]:v["cluster_begin"][c] + v["cluster_count"][c]]))
        ref = oc.modified_charges(okey[key], q)
        for qi in ([0] if m == 1 else [0, 7, 15]):
            got = plan.modified_charges(c, qi)
            assert np.max(np.abs(ref[qi] - got)) <= 1e-12 * np.max(np.abs(ref[qi])), (c, qi)


def _abs_moments(oc, c, q, degree):
    """sum_j |q_jm| |L1_k1(y_j)| |L2_k2(y_j)| |L3_k3(y_j)| of oracle cluster c (eq. 12
    with every term taken by magnitude): the scale of the FP32 rounding of q-hat."""
    info = oc.cluster(c)
    members = oc.cluster_members(c)
    q2 = np.atleast_2d(q)[:, members]
    pos = oc._s[members]
    L = []
    for l in range(3):
        nodes, w = oracle.chebyshev(degree, info["lo"][l], info["hi"][l])
        L.append(np.abs(np.array([oracle.lagrange(degree, nodes, w, x) for x in pos[:, l]])))
    return np.einsum("mj,ja,jb,jc->mabc", np.abs(q2), L[0], L[1], L[2])


@pytest.mark.parametrize("m", [1, 16])
def test_mixed_modified_charges_fp32_products(dev, m):
    # FP32-mixed plans form the factors in FP64 and run the upward products on
    # FP32 matrix cores (partial tiles of at most 256 sources, summed in FP64):
    # every q-hat entry within 16 eps32 of the sum of its terms' magnitudes, on
    # clusters that span several upward chunks and on leaves
    pos, q = inputs.uniform_cube(40000, 160 + m, m=m)
    g = np.random.default_rng(160 + m)
    tgt = np.concatenate([g.uniform(-1, 1, (3000, 3)), g.uniform(-1, 1, (3000, 3)) + [8.0, 1.0, 0.0]])
    plan, _ = _run_plan(dev, tgt, pos, q if m > 1 else q[0], theta=0.9, degree=4, leaf_size=2000,
                        batch_size=2000, precision="fp32_mixed")
    oc = oracle.Treecode(tgt, pos, 0.9, 4, 2000, 2000)
    v = plan.view()
    oorder = oc.source_order()
    okey = {}
    for c in range(oc.n_clusters):
        info = oc.cluster(c)
        okey[tuple(np.sort(oorder[info["begin"]:info["begin"] + info["count"]]))] = c
    approx = np.unique(v["item_cluster"][v["item_kind"] == 0])
    big = [c for c in approx if v["cluster_count"][c] > 8192]
    assert big, "the test needs clusters that span several chunks"
    worst = 0.0
    for c in list(big) + list(approx[:4]):
        key = tuple(np.sort(v["source_order"][v["cluster_begin"][c]:v["cluster_begin"][c] + v["cluster_count"][c]]))
        oc_c = okey[key]
        ref = oc.modified_charges(oc_c, q)       # (m, 5, 5, 5), or (5, 5, 5) for one vector
        scale = _abs_moments(oc, oc_c, q, 4)     # (m, 5, 5, 5)
        if m == 1:
            ref = ref[None]
        for qi in ([0] if m == 1 else [0, 7, 15]):
            got = plan.modified_charges(c, qi)
            ratio = np.max(np.abs(ref[qi] - got) / (EPS32 * scale[qi]))
            worst = max(worst, float(ratio))
            assert ratio <= 16.0, (c, qi, ratio)
    print(f"[qhat fp32] worst {worst:.2f} eps32 sum|terms|", flush=True)


@pytest.mark.parametrize("degree", list(range(1, 17)))
def test_modified_charges_every_degree(dev, degree):
    # one charge vector at every degree (n + 1 = 2..17 points per dimension):
    # the root spans several upward-pass chunks with a ragged last one, its
    # children one chunk each; some sources sit on Chebyshev points of the
    # root in one, two or three coordinates (the rule of eq. 5)
    g = np.random.default_rng(150 + degree)
    src = g.uniform(-1, 1, (9001, 3))
    src[0] = (-1.0, -1.0, -1.0)
    src[1] = (1.0, 1.0, 1.0)          # root box [-1, 1]^3
    s, _ = oracle.chebyshev(degree, -1.0, 1.0)
    k = len(s)
    for i in range(k):
        src[2 + 3 * i, 0] = s[i]
        src[3 + 3 * i, :2] = (s[i], s[(i + 1) % k])
        src[4 + 3 * i] = (s[i], s[(i + 2) % k], s[(i + 3) % k])
    q = g.uniform(-1, 1, len(src))
    tgt = np.concatenate([g.uniform(-1, 1, (2000, 3)) + [9.0, 0.0, 0.0],
                          g.uniform(-1, 1, (2000, 3)) + [2.6, 0.0, 0.0]])
    plan, phi = _run_plan(dev, tgt, src, q, theta=0.7, degree=degree, leaf_size=2000,
                          batch_size=300)
    oc = oracle.Treecode(tgt, src, 0.7, degree, 2000, 300)
    v = plan.view()
    oorder = oc.source_order()
    okey = {}
    for c in range(oc.n_clusters):
        info = oc.cluster(c)
        okey[tuple(np.sort(oorder[info["begin"]:info["begin"] + info["count"]]))] = c
    approx = np.unique(v["item_cluster"][v["item_kind"] == 0])
    assert approx.size and v["cluster_count"][approx].max() == len(src)
    for c in approx:
        key = tuple(np.sort(v["source_order"][v["cluster_begin"][c]:v["cluster_begin"][c] + v["cluster_count"][c]]))
        ref = oc.modified_charges(okey[key], q)
        got = plan.modified_charges(c)
        assert np.max(np.abs(ref - got)) <= 1e-12 * np.max(np.abs(ref)), c
    _close(oc.potential(q), phi)


@pytest.mark.parametrize("precision", ["fp64", "fp32_mixed"])
@pytest.mark.parametrize("same", [True, False])
def test_threads_per_target(dev, precision, same):
    # 2 and 4 lanes per target split each batch's lists into contiguous pieces;
    # the per-entry sums are unchanged, only the FP64 order across entries moves
    g = np.random.default_rng(160)
    src = g.uniform(-1, 1, (9000, 3))
    tgt = src if same else g.uniform(-0.8, 1.3, (7001, 3))
    q = g.uniform(-1, 1, len(src))
    kw = dict(theta=0.7, degree=5, leaf_size=300, batch_size=300 if same else 251,
              precision=precision)
    plan1, phi1 = _run_plan(dev, tgt, src, q, **kw)
    assert (plan1.stats()["mutual_pair_evals"] > 0) == same
    for tpt in (2, 4):
        plan, phi = _run_plan(dev, tgt, src, q, threads_per_target=tpt, **kw)
        assert plan.stats()["threads_per_target"] == tpt
        assert np.max(np.abs(phi - phi1)) <= 1e-12 * np.max(np.abs(phi1)), tpt
    if precision == "fp64":
        ref = oracle.Treecode(tgt, src, 0.7, 5, 300, 300 if same else 251).potential(q)
        _close(ref, phi)


@pytest.mark.parametrize("tpt", [2, 4])
def test_threads_per_target_edge_cases(dev, tpt):
    # one target; batches with fewer list entries than pieces (empty pieces);
    # theta = 0 (all direct); a Plummer sphere in FP32-mixed
    g = np.random.default_rng(162)
    one = g.uniform(-1, 1, (1, 3))
    src = g.uniform(-1, 1, (300, 3))
    q = g.uniform(-1, 1, 300)
    _, phi = _run_plan(dev, one, src, q, theta=0.7, degree=3, leaf_size=40, batch_size=40,
                       threads_per_target=tpt)
    _close(oracle.direct(one, src, q), phi, rel_max=1e-6, rel_l2=1e-6)
    _, phi1 = _run_plan(dev, one, src, q, theta=0.7, degree=3, leaf_size=40, batch_size=40)
    assert np.max(np.abs(phi - phi1)) <= 1e-12 * np.max(np.abs(phi1))
    small = g.uniform(-1, 1, (257, 3))
    qs = g.uniform(-1, 1, 257)
    for theta in (0.0, 0.9):
        _, a = _run_plan(dev, small, small, qs, theta=theta, degree=2, leaf_size=9, batch_size=9,
                         threads_per_target=tpt)
        _, b = _run_plan(dev, small, small, qs, theta=theta, degree=2, leaf_size=9, batch_size=9)
        assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(b)), theta
    pos, qp = inputs.plummer_sphere(30000, 163)
    kw = dict(theta=0.7, degree=6, leaf_size=400, batch_size=400, precision="fp32_mixed",
              kernel="yukawa", kappa=0.5)
    _, a = _run_plan(dev, pos, pos, qp[0], threads_per_target=tpt, **kw)
    _, b = _run_plan(dev, pos, pos, qp[0], **kw)
    assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(b))
    ref = oracle.Treecode(pos, pos, 0.7, 6, 400, 400).potential(qp[0], kernel=oracle.YUKAWA,
                                                                 kappa=0.5)
    assert_mixed(ref, a, pos, pos, qp[0], oracle.YUKAWA, 0.5, what=f"tpt {tpt}")


def test_threads_per_target_autotuned(dev):
    import paper_2003_01836_amd as bltc
    pos, q = inputs.uniform_cube(4000, 161)
    t = _dev_soa(pos, dev)
    size, tpt, ms = bltc.autotune(t, t, candidates=(200, 400), use_cache=False, full=True,
                                  theta=0.7, degree=4)
    assert size in (200, 400) and tpt in (1, 2, 4) and ms > 0
    plan = bltc.Plan(t, t, theta=0.7, degree=4, leaf_size=size, batch_size=size,
                     threads_per_target=tpt)
    phi = plan.execute(torch.from_numpy(q[0]).to(dev)).cpu().numpy()
    _close(oracle.Treecode(pos, pos, 0.7, 4, size, size).potential(q[0]), phi)
    # a fixed choice is kept
    _, tpt_fixed, _ = bltc.autotune(t, t, candidates=(200,), use_cache=False, full=True,
                                    theta=0.7, degree=4, threads_per_target=1)
    assert tpt_fixed == 1


# --------------------------------------------------------------------------
# many systems in one work-queue launch, replayed from a hipGraph
# --------------------------------------------------------------------------
def _systems(seed, sizes, m):
    out = []
    for k, n in enumerate(sizes):
        if k % 3 == 2:
            pos, q = inputs.plummer_sphere(n, seed + k, m=m)
        else:
            pos, q = inputs.uniform_cube(n, seed + k, m=m)
        out.append((pos, q))
    return out


@pytest.mark.parametrize("precision", ["fp64", "fp32_mixed"])
def test_batch_graph_replays_match_oracle(dev, precision):
    import paper_2003_01836_amd as bltc
    sizes = [3000, 17000, 800, 9000, 25000, 5000]
    systems = _systems(500, sizes, 16)
    plans, qd, refs = [], [], []
    for k, (pos, q) in enumerate(systems):
        leaf = 400 if k % 2 else 700
        t = _dev_soa(pos, dev)
        plans.append(bltc.Plan(t, t, theta=0.7, degree=6, leaf_size=leaf, batch_size=leaf, max_q=16,
                               precision=precision))
        mk = 16 if k != 3 else 5                   # one system with fewer vectors
        qd.append(torch.from_numpy(np.ascontiguousarray(q[:mk])).to(dev))
        refs.append(oracle.Treecode(pos, pos, 0.7, 6, leaf, leaf).potential(q[:mk]))
    batch = bltc.Batch(plans)
    outs = [torch.empty((qd[k].shape[0], sizes[k]), dtype=torch.float64, device=dev) for k in range(6)]
    first = None
    for rep in range(3):
        for o in outs:
            o.fill_(float("nan"))
        batch.execute(qd, outs)
        torch.cuda.synchronize()
        got = [o.cpu().numpy() for o in outs]
        for k in range(6):
            for i in range(qd[k].shape[0]):
                if precision == "fp64":
                    _close(refs[k][i], got[k][i])
                elif rep == 0:
                    pos, q = systems[k]
                    assert_mixed(refs[k][i], got[k][i], pos, pos, q[i], what=f"system {k} vector {i}")
                else:
                    assert oracle.rel_l2(refs[k][i], got[k][i]) <= MIXED_REL_L2
        if first is None:
            first = got
        else:
            for a, b in zip(first, got):
                assert np.array_equal(a, b)         # every replay identical
        # eager work between replays
        plans[0].execute(qd[0][:3].contiguous())
        torch.cuda.synchronize()
    info = batch.info()
    assert info["graph_captures"] == 1 and info["launches"] == 3 and info["systems"] == 6
    # the same without the graph
    batch.set_graph(False)
    batch.execute(qd, outs)
    torch.cuda.synchronize()
    for a, o in zip(first, outs):
        assert np.array_equal(a, o.cpu().numpy())
    # new output buffers: captured again
    batch.set_graph(True)
    outs2 = [torch.empty_like(o) for o in outs]
    batch.execute(qd, outs2)
    torch.cuda.synchronize()
    for a, o in zip(first, outs2):
        assert np.array_equal(a, o.cpu().numpy())
    assert batch.info()["graph_captures"] == 2


def test_batch_rejects_bad_plans(dev):
    import paper_2003_01836_amd as bltc
    pos, q = inputs.uniform_cube(2000, 600)
    t = _dev_soa(pos, dev)
    p1 = bltc.Plan(t, t, max_q=1, leaf_size=200, batch_size=200)
    with pytest.raises(bltc.InvalidArgument):
        bltc.Batch([p1])
    p2 = bltc.Plan(t, t, max_q=4, leaf_size=200, batch_size=200)
    p3 = bltc.Plan(t, t, max_q=4, leaf_size=200, batch_size=200, precision="fp32_mixed")
    with pytest.raises(bltc.InvalidArgument):
        bltc.Batch([p2, p3])
    b = bltc.Batch([p2])
    with pytest.raises(bltc.InvalidArgument):
        b.execute([torch.zeros((5, 2000), dtype=torch.float64, device=dev)])   # 5 > max_q


def test_autotune_picks_a_candidate_and_caches(dev, tmp_path, monkeypatch):
    import paper_2003_01836_amd as bltc
    monkeypatch.setenv("BLTC_TUNE_CACHE", str(tmp_path / "tune.txt"))
    pos, q = inputs.uniform_cube(60000, 700)
    t = _dev_soa(pos, dev)
    cands = (150, 400, 1200)
    leaf, ms = bltc.autotune(t, t, cands, degree=4, theta=0.7)
    assert leaf in cands and ms > 0
    text = (tmp_path / "tune.txt").read_text()
    assert f"|{leaf} " in text
    # a second call is answered from the cache (same value, no new entry)
    leaf2, ms2 = bltc.autotune(t, t, cands, degree=4, theta=0.7)
    assert (leaf2, ms2) == (leaf, pytest.approx(ms, rel=1e-5))
    assert (tmp_path / "tune.txt").read_text() == text
    # the tuned plan is still exact against the oracle at its own leaf size
    _, phi = _run_plan(dev, pos, pos, q[0], degree=4, theta=0.7, leaf_size=leaf, batch_size=leaf)
    _close(oracle.Treecode(pos, pos, 0.7, 4, leaf, leaf).potential(q[0]), phi)
