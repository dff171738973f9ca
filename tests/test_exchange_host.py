"""Host logic of the exchange-landscape analysis (no GPU): geometry, minimax path, barrier
and trap."""
import numpy as np
import pytest

from paper_2609_07842_amd import workloads as W


def test_positions():
    from paper_2609_07842_amd import exchange as E
    p = W.vbc_params(f=3.0)
    x = E.positions(p, 3, 1.1, 2.3) - E.BOX / 2
    assert np.allclose(x, [[0, 0, 0], [1.1, 0, 0], [-2.3, 0, 0], [0, 1.25, 0], [0, -1.25, 0]])
    r = E.grid_radii(p, 11)
    assert r[0] == pytest.approx(0.9) and r[-1] == pytest.approx(2.5)
    with pytest.raises(ValueError):
        E.positions(p, 6, 1.0, 1.0)


def test_bottleneck_finds_the_pass():
    from paper_2609_07842_amd.exchange import bottleneck
    # two wells in opposite corners, a ridge of height 5 with a pass of height 2 at one cell
    U = np.zeros((9, 9))
    U[4, :] = 5.0
    U[4, 6] = 2.0
    U[0, 0] = U[8, 8] = -1.0
    assert bottleneck(U, (0, 0), (8, 8)) == 2.0
    U[4, 6] = 7.0  # no pass lower than the ridge
    assert bottleneck(U, (0, 0), (8, 8)) == 5.0
    # a diagonal step counts as a neighbour
    V = np.full((3, 3), 9.0)
    V[0, 0] = V[1, 1] = V[2, 2] = 0.0
    assert bottleneck(V, (0, 0), (2, 2)) == 0.0


def test_barrier_and_trap():
    from paper_2609_07842_amd.exchange import barrier_and_trap
    r = np.linspace(0.9, 2.5, 33)
    well = lambda q: -2.0 * np.exp(-((q - 1.25) / 0.15) ** 2)
    A, B = np.meshgrid(r, r, indexing="ij")
    # a bond only while the other particle is away: any exchange loses the whole well first
    U = np.where(B >= 1.8, well(A), 0.0) + np.where(A >= 1.8, well(B), 0.0)
    b, trap = barrier_and_trap(U, r)
    assert not trap and b == pytest.approx(-U.min(), abs=1e-4)  # up to the wells' tails
    # a channel through the double-bonded corner at half the depth: barrier 1
    U1 = np.minimum(U, -1.0 * ((A < 1.8) & (B < 1.8)))
    assert barrier_and_trap(U1, r) == (pytest.approx(1.0, abs=1e-9), False)
    # both bonded deep in the well, below one bond: a trap
    U2 = np.minimum(U, -3.0 * ((A < 1.35) & (B < 1.35)))
    assert barrier_and_trap(U2, r)[1]
    # lower only with the newcomer at the edge of the range: not a trap
    U3 = np.minimum(U, -2.005 * ((A > 1.2) & (A < 1.3) & (B > 1.45) & (B < 1.5)))
    assert not barrier_and_trap(U3, r)[1]


def test_trap_appears_when_suppression_comes_late():
    """With oracle energies: a negative shift delta lets an extra particle bind to a
    saturated centre (a trap); the exchange-tuned geometry has none."""
    import oracle
    from paper_2609_07842_amd import exchange as E

    def land(g, f):
        p = W.vbc_params(E_a=2.0, f=float(f), r_l=g[0], r_h=g[1], delta=g[2])
        r = E.grid_radii(p, 21)
        U = np.array([[oracle.evaluate(E.positions(p, f, a, b), E.BOX, p)["U"] for b in r] for a in r])
        return E.barrier_and_trap(U, r)

    assert land((1.29, 1.50, -0.6), 1)[1]
    assert not land((1.29, 1.50, 0.30), 1)[1] and not land((1.29, 1.50, 0.30), 3)[1]
