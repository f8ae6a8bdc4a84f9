import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# PyTorch ships its own HIP runtime under the same soname as the system one
# libmx.so links; whichever is loaded first serves the whole process, and
# torch's other libraries find no device when the system runtime came first.
# Importing torch here loads torch's first, whatever tests are selected.
try:
    import torch  # noqa: F401
except ImportError:
    pass


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")
