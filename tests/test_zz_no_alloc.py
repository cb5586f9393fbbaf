"""bltc_direct_noalloc: the FP64 direct sum of eq. 1 with its source staging in
the library's fixed device array instead of a per-call allocation.

It runs bltc_direct's kernels in the same order, so its potentials equal
bltc_direct's bit for bit; both are held to the oracle's direct sum at the
FP64 bar (1e-12 of the largest potential, element-wise).  Two calls in a row,
the second on a smaller input, check that the shared array carries nothing
from one call into the next."""
import numpy as np
import pytest

import oracle
from paper_2003_01836_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

BLTC_EUNSUPPORTED = -4
MAX_SOURCES = 1 << 20


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2003_01836_amd as bltc
    bltc.version()
    return torch.device("cuda:0")


def _soa(pos, dev):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(pos, dtype=np.float64).T)).to(dev)


def _check(ref, got):
    scale = np.max(np.abs(ref))
    assert np.all(np.isfinite(got))
    assert np.max(np.abs(ref - got)) <= 1e-12 * scale, np.max(np.abs(ref - got)) / scale


@pytest.mark.parametrize("kernel,kappa", [("coulomb", 0.0), ("yukawa", 0.5)])
def test_noalloc_direct_matches_direct_on_two_calls(dev, kernel, kappa):
    import paper_2003_01836_amd as bltc
    okern = oracle.YUKAWA if kernel == "yukawa" else oracle.COULOMB
    # the first call larger (three vectors), the second smaller (one vector)
    for n, nt, m, seed in ((60000, 3000, 3, 901), (7000, 900, 1, 902)):
        print(f"[noalloc] {kernel}: {nt} targets, {n} sources, {m} vectors", flush=True)
        pos, q = inputs.uniform_cube(n, seed, m=m)
        tgt = np.random.default_rng(seed + 50).uniform(-1, 1, (nt, 3))
        s, t = _soa(pos, dev), _soa(tgt, dev)
        qd = torch.from_numpy(np.ascontiguousarray(q if m > 1 else q[0])).to(dev)
        shape = (m, nt) if m > 1 else (nt,)
        oa = torch.full(shape, np.nan, dtype=torch.float64, device=dev)
        ob = torch.full(shape, np.nan, dtype=torch.float64, device=dev)
        a = bltc.direct(t, s, qd, out=oa, kernel=kernel, kappa=kappa)
        b = bltc.direct(t, s, qd, out=ob, kernel=kernel, kappa=kappa, noalloc=True)
        torch.cuda.synchronize()
        a, b = a.cpu().numpy(), b.cpu().numpy()
        assert np.array_equal(a, b)
        ref = oracle.direct(tgt, pos, q if m > 1 else q[0], kernel=okern, kappa=kappa)
        _check(ref, b)


def test_noalloc_direct_edges(dev):
    import paper_2003_01836_amd as bltc
    pos, q = inputs.uniform_cube(500, 903)
    s = _soa(pos, dev)
    qd = torch.from_numpy(q[0]).to(dev)
    # no sources: zeros (the staging array is not read)
    out = torch.full((300,), np.nan, dtype=torch.float64, device=dev)
    empty = torch.zeros((3, 0), dtype=torch.float64, device=dev)
    got = bltc.direct(s[:, :300].contiguous(), empty, torch.zeros(0, dtype=torch.float64,
                                                                  device=dev), out=out,
                      noalloc=True)
    assert np.array_equal(got.cpu().numpy(), np.zeros(300))
    # targets = sources: the self terms are skipped, as in bltc_direct
    a = bltc.direct(s, s, qd).cpu().numpy()
    b = bltc.direct(s, s, qd, noalloc=True).cpu().numpy()
    assert np.array_equal(a, b)
    _check(oracle.direct(pos, pos, q[0]), b)
    # the largest source count the array holds, then one more: a clear error
    g = np.random.default_rng(904)
    big = torch.from_numpy(g.uniform(-1, 1, (3, MAX_SOURCES + 1))).to(dev)
    qb = torch.from_numpy(g.uniform(-1, 1, MAX_SOURCES + 1)).to(dev)
    few = big[:, :64].contiguous()
    most = big[:, :MAX_SOURCES].contiguous()
    a = bltc.direct(few, most, qb[:MAX_SOURCES]).cpu().numpy()
    b = bltc.direct(few, most, qb[:MAX_SOURCES], noalloc=True).cpu().numpy()
    assert np.array_equal(a, b)
    with pytest.raises(bltc.BLTCError) as ei:
        bltc.direct(few, big, qb, noalloc=True)
    assert ei.value.code == BLTC_EUNSUPPORTED and "at most" in str(ei.value)
