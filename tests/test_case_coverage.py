"""CPU checks that the GPU parity cases reach every lane split of the dU/dn pass: a brick's
window particles (those whose exact count lies within 1e-4 of a switching window) take
eight lanes each in one wave when there are at most 8, eight lanes each over the four
waves of the workgroup up to 32, and four lanes each beyond.  The window populations are
computed with the oracle's counts on the cases' own inputs and brick grid."""
import numpy as np
import pytest

import oracle
from paper_2609_07842_amd import workloads as W

MARGIN = 1e-4


def _window_per_brick(N, rho, f, seed):
    L = W.box_length(N, rho)
    p = W.vbc_params(E_a=5.0, f=f)
    x = W.uniform_positions(N, L, seed=seed)
    n = oracle.evaluate(x, L, p)["n"]
    win = (n > f - MARGIN) & (n < f + 1.0 + MARGIN)  # delta = 0: window (f, f + 1)
    # the library's grid: cells of at least the list radius r_h + buffer = 2.4, bricks of
    # min(4, nc - 2) cells per axis
    nc = int(np.floor(L / 2.4))
    while nc > 1 and L / nc < 2.4 * (1.0 + 1e-9):
        nc -= 1
    h, bd = L / nc, min(4, nc - 2)
    nb = -(-nc // bd)
    c = np.minimum(np.floor((x % L) / h).astype(int), nc - 1) // bd
    bid = c[:, 0] + nb * (c[:, 1] + nb * c[:, 2])
    return np.bincount(bid[win], minlength=nb ** 3)


@pytest.mark.parametrize("seed_off", [1, 2])
def test_parity_cases_reach_every_dudn_lane_split(seed_off):
    # the fp64 and fp32 parity tests draw positions with seed N + 1 and N + 2; each brick
    # takes the split its own window population selects
    cnt = np.concatenate([_window_per_brick(1500, 0.1, 2.0, 1500 + seed_off),
                          _window_per_brick(4000, 0.5, 6.0, 4000 + seed_off),
                          _window_per_brick(4000, 0.5, 10.0, 4000 + seed_off)])
    print(f"[coverage] window particles per brick: {sorted(cnt.tolist())}")
    assert np.any((cnt > 0) & (cnt <= 8))
    assert np.any((cnt > 8) & (cnt <= 32))
    assert np.any(cnt > 32)
