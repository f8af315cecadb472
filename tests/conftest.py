import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
HERE = os.path.dirname(os.path.abspath(__file__))
if HERE not in sys.path:
    sys.path.insert(0, HERE)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (run through the HIP library)")
    config.addinivalue_line("markers", "slow: longer CPU checks")


def pytest_collection_modifyitems(config, items):
    # make sure the oracle is built before any test uses it
    from oracle import oracle as _o
    if not os.path.exists(_o.LIBPATH):
        from oracle.build_oracle import build
        build()
