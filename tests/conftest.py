import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running statistical check")


@pytest.fixture(scope="session")
def oracle_lib():
    import oracle
    from oracle import oracle as _o
    return _o.load()


@pytest.fixture(scope="session")
def planted(tmp_path_factory):
    """Build the oracle with one ORACLE_PLANT_* mistake compiled in."""
    from oracle import oracle as _o
    cache = {}
    d = tmp_path_factory.mktemp("planted")

    def make(flag):
        if flag not in cache:
            path = str(d / f"lib_{flag}.so")
            _o.build(extra_flags=[f"-D{flag}"], out_path=path)
            cache[flag] = _o.load(path)
        return cache[flag]
    return make
