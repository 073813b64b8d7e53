import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: longer CPU-side oracle checks")
    # The oracle and the generator are plain C compiled with gcc.  Their
    # loaders never compile; build them here, before any test can touch a
    # GPU, when a checkout has not been built yet.
    import oracle
    import synth

    for mod in (oracle, synth):
        if not os.path.exists(mod._SO):
            mod.build()
