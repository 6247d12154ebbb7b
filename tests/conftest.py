import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the C ABI of the HIP library)")


@pytest.fixture(scope="session")
def det_barrel():
    from synth import barrel10
    return barrel10()


@pytest.fixture(scope="session")
def det_dense():
    from synth import barrel_endcap
    return barrel_endcap()


@pytest.fixture(scope="session")
def det_dense_vacuum():
    from synth import barrel_endcap
    return barrel_endcap(thick=0.0)


@pytest.fixture(scope="session")
def oracle_lib():
    import oracle
    oracle.build(force=not os.path.exists(oracle.LIB))
    return oracle


def double_matched(ev, meas_ids, seed_particle):
    """Paper section 3.1: the major particle contributes N of the track's Nt
    measurements and has Np measurements in total; matched if N > Nt/2 and
    N > Np/2 (and, here, it is the particle the seed came from)."""
    parts = ev.meas_particle[meas_ids]
    parts = parts[parts >= 0]
    if parts.size == 0:
        return False
    vals, cnt = np.unique(parts, return_counts=True)
    maj = vals[np.argmax(cnt)]
    N = cnt.max()
    return bool(N > len(meas_ids) / 2 and N > ev.particle_nhits[maj] / 2 and maj == seed_particle)


@pytest.fixture(scope="session")
def dense_table(det_dense):
    """The oracle's neighbour table of the whole barrel + endcap detector."""
    from oracle import learned as OL
    return OL.neighbour_table(det_dense.as_arrays())


@pytest.fixture(scope="session")
def golden_model():
    """Network parameters trained by the oracle alone on its own tracks
    (tests/golden/make_learned_model.py)."""
    return np.loadtxt(os.path.join(ROOT, "tests", "golden", "learned_model.txt"), dtype=np.float32)
