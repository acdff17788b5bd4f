import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")
    # The host tests load the HIP library (its analysis phase needs no
    # device): build it when it is missing, so that they fail on a broken
    # build instead of skipping.
    lib = os.path.join(ROOT, "paper_2202_09288_amd", "libspchol.so")
    if not os.path.exists(lib):
        from paper_2202_09288_amd import build
        build.build()
