import functools
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")


@functools.lru_cache(maxsize=None)
def _mech(name):
    from paper_2411_02640_amd import inputs as I
    spec = {"syn9": I.MECH_9, "syn53": I.MECH_53, "syn200": I.MECH_200, "syn100": I.MECH_100,
            "syn53x": I.MECH_53X, "syn53o": I.MECH_53O, "syn53q": I.MECH_53Q,
            "syn53xq": I.MECH_53XQ, "syn200q": I.MECH_200Q}[name]
    return I.make_mechanism(spec)


@pytest.fixture(scope="session")
def mech9():
    return _mech("syn9")


@pytest.fixture(scope="session")
def mech53():
    return _mech("syn53")


@pytest.fixture(scope="session")
def mech200():
    return _mech("syn200")


@pytest.fixture(scope="session")
def mech100():
    return _mech("syn100")


@pytest.fixture(scope="session")
def mech53x():
    return _mech("syn53x")


@pytest.fixture(scope="session")
def mech53o():
    return _mech("syn53o")


@pytest.fixture(scope="session")
def mech53q():
    return _mech("syn53q")


@pytest.fixture(scope="session")
def mech53xq():
    return _mech("syn53xq")


@pytest.fixture(scope="session")
def mech200q():
    return _mech("syn200q")


@pytest.fixture(scope="session")
def oracle_lib():
    from oracle import oracle as O
    O.lib()
    return O
