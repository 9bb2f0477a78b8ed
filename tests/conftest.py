import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the C-ABI library)")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


_CACHE = {}


def built(name):
    """Session cache of small seeded H^2 representations used by several tests."""
    if name in _CACHE:
        return _CACHE[name]
    if name.endswith("_sym"):                 # couplings symmetrised (S_st = S_ts^T bit for bit)
        from h2gen.construct import symmetrize_couplings
        g, d = built(name[:-4])
        _CACHE[name] = (g, symmetrize_couplings(d))
        return _CACHE[name]
    import h2gen
    from h2gen.construct import build_h2
    from h2gen.geometry import box
    if name == "cube12":       # 0.5 wavelength cube, eps_r = 4, eps = 1e-4
        g = h2gen.cube(12, 0.5, 4.0)
        d = build_h2(g, eps=1e-4)
    elif name == "cube12_e3":
        g = h2gen.cube(12, 0.5, 4.0)
        d = build_h2(g, eps=1e-3)
    elif name == "cube8":      # all blocks near
        g = h2gen.cube(8, 0.5, (2.0, 6.0), seed=3)
        d = build_h2(g, eps=1e-4)
    elif name == "rod":        # 2-child splits, transfers on 2 levels
        g = box((64, 4, 4), 1.0 / 16, eps=(2.0, 6.0), seed=7)
        d = build_h2(g, eps=1e-4)
    elif name == "slab":       # 4-child splits
        g = box((32, 32, 4), 1.0 / 16, eps=(2.0, 6.0), seed=8)
        d = build_h2(g, eps=1e-4)
    elif name == "cube13":     # uneven leaves
        g = h2gen.cube(13, 13.0 / 16, (1.5, 8.0), seed=9)
        d = build_h2(g, eps=1e-4)
    elif name == "cube16":     # octree transfers
        g = h2gen.cube(16, 1.0, (2.0, 6.0), seed=2)
        d = build_h2(g, eps=1e-3)
    elif name == "box9":       # mixed leaf depths (9 -> 5+4 splits)
        g = box((9, 9, 9), 1.0 / 16, eps=(1.5, 8.0), seed=11)
        d = build_h2(g, eps=1e-4)
    else:
        raise KeyError(name)
    _CACHE[name] = (g, d)
    return g, d
