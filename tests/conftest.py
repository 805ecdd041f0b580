import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    # the autotuner's own table file for this test session: results never
    # depend on, or add to, the user's table (the table shipped with the
    # library still applies)
    if "RAC_TUNE_CACHE" not in os.environ:
        import tempfile
        fd, path = tempfile.mkstemp(prefix="rac_tune_", suffix=".txt")
        os.close(fd)
        os.environ["RAC_TUNE_CACHE"] = path
