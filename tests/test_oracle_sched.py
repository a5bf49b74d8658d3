"""Pins of the scheduling oracle: LPT (Alg. 1, bound (13)) and modified Part_Schedule (Alg. 2, (14))."""
import numpy as np
import pytest

from oracle import sched


@pytest.mark.parametrize("P", [2, 3, 4])
def test_lpt_graham_tight_family(P):
    """Times 2P-1, 2P-1, 2P-2, 2P-2, ..., P+1, P+1, P, P, P reach the bound (13) exactly."""
    tau = []
    for v in range(2 * P - 1, P, -1):
        tau += [v, v]
    tau += [P, P, P]
    _, c_lpt = sched.lpt(tau, P)
    c_opt = sched.brute_force_opt(tau, P)
    assert c_opt == 3 * P
    assert c_lpt / c_opt == pytest.approx(sched.lpt_bound(P))


def test_lpt_within_bound_on_random_instances():
    rng = np.random.default_rng(0)
    for _ in range(60):
        P = int(rng.integers(2, 5))
        n = int(rng.integers(P + 1, 9))
        tau = list(rng.integers(1, 30, size=n).astype(float))
        C, c_lpt = sched.lpt(tau, P)
        assert sorted(sum(C, [])) == list(range(n))
        assert c_lpt <= sched.lpt_bound(P) * sched.brute_force_opt(tau, P) + 1e-12


def test_approximate_square_claim():
    """For P_i > 20 the next larger approximate square is within 20 % of P_i; the claim
    fails just below the cutoff (the reason for P_cutoff = 20)."""
    worst = max(sched.next_approx_square(p) / p for p in range(21, 5000))
    assert worst <= 0.2 + 1e-12
    assert any(sched.next_approx_square(p) / p > 0.2 for p in range(13, 21))


def _interposer_like(seed):
    """One task with 53 % of the estimated work and 128 tasks of 0.3-0.43 % (fan-out interposer)."""
    rng = np.random.default_rng(seed)
    small = rng.uniform(0.003, 0.0043, size=128)
    small *= 0.47 / small.sum()
    return np.concatenate([[0.53], small])


def test_part_schedule_invariants_and_bound():
    for seed in range(3):
        W = _interposer_like(seed)
        for P in (20, 40, 80, 160, 320):
            for modified in (True, False):
                Pi, C = sched.part_schedule(W, P, modified=modified)
                assert sum(p for p in Pi if p > 1) <= P
                lb = max(sched.ideal_length(W, P), max(W) / P)
                assert C <= sched.part_schedule_bound(P) * lb * 1.0000001
                if modified:
                    assert all(p <= 20 or sched.is_approx_square(p) for p in Pi)


def test_modified_vs_original_within_15_percent():
    """Modified and original Part_Schedule give schedule lengths (normalised by the ideal)
    that differ by less than 15 % on interposer-like task sets."""
    for seed in range(3):
        W = _interposer_like(seed)
        for P in (20, 50, 100, 200, 400, 800):
            _, cm = sched.part_schedule(W, P, modified=True)
            _, co = sched.part_schedule(W, P, modified=False)
            ideal = sched.ideal_length(W, P)
            assert abs(cm / ideal - co / ideal) / (co / ideal) < 0.15
