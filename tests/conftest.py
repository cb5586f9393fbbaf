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
