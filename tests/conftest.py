import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    # the autotuner's on-disk cache must not carry a choice from an earlier
    # run (or a bench) into the tests: a private file per session
    import tempfile
    os.environ["DC_TUNE_CACHE"] = os.path.join(tempfile.mkdtemp(prefix="dc_tune_"), "tune.json")
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: full-size workloads (minutes)")
