import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


def read_golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            rows.append([float(v) for v in line.split()])
    return rows


# kernel cases of the GPU parity tests: (library kernel name, its parameter)
KERNEL_CASES = [("coulomb", 0.0), ("yukawa", 0.5), ("regularized", 0.01)]


def kernel_kwargs(kernel, param):
    """Library keyword arguments and the oracle's (kernel id, parameter) for a
    kernel case; the oracle takes delta of the regularized kernel as kappa."""
    import oracle
    if kernel == "regularized":
        return {"kernel": kernel, "delta": param}, oracle.REGULARIZED, param
    if kernel == "yukawa":
        return {"kernel": kernel, "kappa": param}, oracle.YUKAWA, param
    return {"kernel": kernel}, oracle.COULOMB, 0.0


# --------------------------------------------------------------------------
# FP32-mixed bounds against the FP64 oracle
# --------------------------------------------------------------------------
EPS32 = 2.0 ** -24
# relative 2-norm difference (eq. 16) over the compared targets
MIXED_REL_L2 = 1e-6
# largest difference relative to the largest potential
MIXED_REL_MAX = 1e-5
# per target: |d phi_i| <= MIXED_K * eps32 * sum_j |G(x_i, y_j) q_j|.  Error model
# of the mixed path: kernel values from FP32 coordinates local to a batch or leaf,
# with pairs closer than 0.024 of the local extent taken in FP64 (coordinate
# rounding at most ~42 eps32 of a term), FP32 partial sums over at most 128 terms,
# far-field terms over modified charges whose magnitudes exceed the charges' by
# the cube of the Chebyshev Lebesgue constant (~14 at n = 8); the sum of |G q|
# over the sources bounds the terms of every list.
MIXED_K = 256


def abs_potential(targets, sources, charges, kernel, kappa):
    """sum_j |G(x_i, y_j) q_j| for every target (the kernels are positive)."""
    import numpy as np
    import oracle
    return oracle.direct(targets, sources, np.abs(charges), kernel=kernel, kappa=kappa)


def assert_mixed(ref, got, targets=None, sources=None, charges=None, kernel=None, kappa=0.0,
                 idx=None, rel_l2=MIXED_REL_L2, rel_max=MIXED_REL_MAX, k=MIXED_K, what=""):
    """FP32-mixed potentials `got` against FP64 oracle potentials `ref` (same targets):
    relative 2-norm, largest difference against the largest potential and, when the
    particles are given, the per-target bound of the error model above.  `idx`
    selects the rows of `targets` that ref/got belong to (sampled targets); at most
    4000 of them are checked per target (evenly spaced)."""
    import numpy as np
    import oracle
    ref = np.asarray(ref, dtype=np.float64)
    got = np.asarray(got, dtype=np.float64)
    assert ref.shape == got.shape
    assert np.all(np.isfinite(got)), what
    d = np.abs(ref - got)
    scale = max(float(np.max(np.abs(ref))), 1e-300) if ref.size else 1.0
    e2 = oracle.rel_l2(ref, got)
    emax = float(np.max(d)) / scale if ref.size else 0.0
    msg = f"{what} rel-L2 {e2:.3e} max {emax:.3e}"
    if targets is not None and ref.size:
        if kernel is None:
            kernel = oracle.COULOMB
        rows = np.arange(ref.size) if idx is None else np.asarray(idx)
        pick = np.unique(np.linspace(0, ref.size - 1, min(ref.size, 4000)).astype(np.int64))
        a = abs_potential(np.asarray(targets)[rows[pick]], sources, charges, kernel, kappa)
        ratio = d[pick] / (EPS32 * np.maximum(a, 1e-300))
        worst = float(np.max(ratio))
        msg += f" per-target {worst:.1f} eps32 sum|Gq|"
        print(f"[mixed] {msg}", flush=True)
        assert worst <= k, msg
    else:
        print(f"[mixed] {msg}", flush=True)
    assert e2 <= rel_l2, msg
    assert emax <= rel_max, msg
