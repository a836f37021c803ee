"""Shared fixtures.  GPU tests are marked ``gpu``; everything else runs on the CPU."""
import json
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs a HIP device (MI355X) and the built libdeflan.so")
    config.addinivalue_line("markers", "slow: long CPU test")


def kappa_entry(name):
    with open(os.path.join(GOLDEN, "kappa.json")) as fh:
        return json.load(fh)[name]


@pytest.fixture(scope="session")
def gpu_ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0901_3163_amd import deflan
    ctx = deflan.Context(0)
    yield ctx
    ctx.close()


@pytest.fixture(scope="session")
def c1_config():
    """The 4^4 near-critical workload: links seed and kappa from the oracle's kappa search."""
    from lattice_inputs import su3_links
    e = kappa_entry("4x4x4x4")
    dims = tuple(e["dims"])
    return dict(dims=dims, seed=e["seed"], kappa=e["kappa"], links=su3_links(dims, e["seed"], e["eps"]),
                min_abs_eig=e["min_abs_eig"])
