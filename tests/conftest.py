import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
HERE = os.path.dirname(os.path.abspath(__file__))
if HERE not in sys.path:
    sys.path.insert(0, HERE)

# PyTorch ships its own HIP runtime; when a test uses torch next to libcmflb,
# torch must be loaded first so that the library binds to the same runtime
# (a second runtime loaded later sees no device).
try:
    import torch  # noqa: F401
except ImportError:
    pass


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: longer statistical runs")


@pytest.fixture(scope="session")
def paper():
    import json
    with open(os.path.join(HERE, "golden", "paper_constants.json")) as fh:
        return json.load(fh)
