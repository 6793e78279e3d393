import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: oracle checks that take tens of seconds")


ROM_DIR = os.path.join(ROOT, 'roms')


def rom_path(name):
    return os.path.join(ROM_DIR, name + '.rom')


@pytest.fixture(scope='session')
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a GPU")
    from paper_2307_16894_amd import lib
    lib()  # fails loudly when the library is not built
    return torch.device('cuda:0')
