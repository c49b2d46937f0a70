import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) and the built HIP library")
    config.addinivalue_line("markers", "slow: longer CPU-only oracle checks")


@pytest.fixture(scope="session")
def klr():
    """The HIP library binding; the product path fails loudly without a GPU or library."""
    from paper_1911_02373_amd import klr as mod
    return mod.Library.get()
