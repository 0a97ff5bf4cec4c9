import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: longer CPU test")


_CACHE = {}


def planet(name, **kw):
    """Cached seeded planets shared by the tests of one session."""
    import planetgen as pg
    key = (name, tuple(sorted(kw.items())))
    if key not in _CACHE:
        _CACHE[key] = getattr(pg, name)(**kw)
    return _CACHE[key]


def pencil(name, **kw):
    from oracle.assemble import Pencil
    key = ("pencil", name, tuple(sorted(kw.items())))
    if key not in _CACHE:
        _CACHE[key] = Pencil(planet(name, **kw))
    return _CACHE[key]
