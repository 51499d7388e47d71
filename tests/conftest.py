import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the C-ABI library on the device)")
    config.addinivalue_line("markers", "slow: long CPU test")


@pytest.fixture(scope="session")
def mech_dir(tmp_path_factory):
    d = os.environ.get("CK_MECH_DIR")
    if d:
        return d
    return str(tmp_path_factory.mktemp("mech"))


@pytest.fixture(scope="session")
def mech_path(mech_dir):
    from paper_1608_05794_amd import synth

    def get(name):
        return synth.mechanism_file(name, mech_dir)
    return get


@pytest.fixture(scope="session")
def oracle_mech(mech_path):
    from oracle import oracle as O
    cache = {}

    def get(name):
        if name not in cache:
            cache[name] = O.Mechanism(mech_path(name))
        return cache[name]
    return get
