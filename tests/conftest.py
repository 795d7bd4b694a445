import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) to run")
    config.addinivalue_line("markers", "slow: longer CPU test")


import pytest  # noqa: E402


@pytest.fixture(autouse=True)
def _library_default_paths(monkeypatch):
    """Every test starts from the library's default code paths: the AH_*
    switches it reads from the environment at setup are cleared (a test that
    forces a path sets its own)."""
    for k in list(os.environ):
        if k.startswith("AH_"):
            monkeypatch.delenv(k, raising=False)
