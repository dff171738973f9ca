"""Host logic of the exchange-path analysis (no GPU): path geometry, barrier and trap."""
import numpy as np
import pytest

from paper_2609_07842_amd import workloads as W


def test_path_geometry():
    from paper_2609_07842_amd import exchange as E
    p = W.vbc_params(f=3.0)
    x0, x1 = E.path_positions(p, 3, 0.0) - E.BOX / 2, E.path_positions(p, 3, 1.0) - E.BOX / 2
    m, d = 1.25, 2.5
    # centre, A at the well minimum, B beyond every range; spectators at the minimum on y
    assert np.allclose(x0[:3], [[0, 0, 0], [m, 0, 0], [-d, 0, 0]])
    assert np.allclose(x1[:3], [[0, 0, 0], [d, 0, 0], [-m, 0, 0]])
    assert np.allclose(x0[3:], [[0, m, 0], [0, -m, 0]]) and np.allclose(x0[3:], x1[3:])
    with pytest.raises(ValueError):
        E.path_positions(p, 6, 0.5)


def test_barrier_and_trap():
    from paper_2609_07842_amd.exchange import barrier_and_trap
    lam = np.linspace(0, 1, 21)
    hump = -1.0 + 0.5 * np.sin(np.pi * lam)
    assert barrier_and_trap(hump) == (pytest.approx(0.5), False)
    # a dip below the end points inside the path is a trap
    dip = -1.0 - 0.3 * np.sin(np.pi * lam)
    b, trap = barrier_and_trap(dip)
    assert b == pytest.approx(0.0) and trap
    # a dip between two humps that stays above the start is not a trap
    two = -1.0 + 0.4 * np.abs(np.sin(2 * np.pi * lam))
    assert barrier_and_trap(two) == (pytest.approx(0.4, abs=1e-3), False)
