import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line(
        "markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def oracle_lib():
    import oracle
    oracle.build(force_rebuild=False)
    return oracle


@pytest.fixture(scope="session")
def cuda():
    """The GPU device; fails (does not skip) when the HIP path is absent."""
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    import paper_1211_4864_amd as hsr
    hsr.load()
    return torch.device("cuda:0")


def to_dev(w, device):
    import torch
    pos = torch.from_numpy(w.pos).to(device)
    mass = torch.from_numpy(w.mass).to(device)
    return pos, mass


def sample_targets(n, keys=None, k=2000, seed=0):
    """Random targets plus, when cell keys are given, targets from the most
    populated cells (the clustered tail)."""
    import numpy as np
    rng = np.random.default_rng(seed)
    pick = rng.choice(n, min(n, k * 3 // 4), replace=False)
    if keys is not None:
        counts = np.bincount(keys)
        dense = np.argsort(-counts[keys], kind="stable")[: k // 4]
        pick = np.unique(np.concatenate([pick, dense]))
    return np.sort(pick)
