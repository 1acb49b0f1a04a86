import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")


@pytest.fixture(scope="session")
def oracle_lib():
    import oracle
    oracle.build(force=False)
    return oracle


@pytest.fixture(scope="session")
def dsmc_gpu():
    """The HIP library on a visible GPU; fails loudly (no fallback) otherwise."""
    import torch
    import paper_cs_9902024_amd as P
    if not torch.cuda.is_available():
        raise RuntimeError("GPU test run without a visible GPU")
    if not os.path.exists(P.LIB_PATH):
        raise RuntimeError(f"{P.LIB_PATH} is not built")
    P.lib()
    return P
