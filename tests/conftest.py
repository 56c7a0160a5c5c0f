import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")

# Text of the paper (for the appendix's embedded two-sphere mesh), from the file PFT_PAPER_TEXT names;
# without it the tests that need the text skip.
PAPER_TEXT = os.environ.get("PFT_PAPER_TEXT", "")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an AMD GPU (MI355X) and the built HIP library")
    config.addinivalue_line("markers", "slow: longer CPU checks")


@pytest.fixture(scope="session")
def paper_text():
    """The paper's text, or a skip when no copy is available."""
    if not PAPER_TEXT or not os.path.exists(PAPER_TEXT):
        pytest.skip("paper text not available (set PFT_PAPER_TEXT)")
    with open(PAPER_TEXT) as f:
        return f.read()


@pytest.fixture(scope="session")
def gpu():
    """The GPU device for parity tests; fails (never skips) when no GPU is present."""
    import torch

    if not torch.cuda.is_available():
        pytest.fail("GPU test selected but no HIP device is visible")
    return torch.device("cuda:0")
