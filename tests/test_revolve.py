"""The binomial checkpointing schedule of the differentiable rollout
(adjoint.revolve_schedule, CPU only): every schedule reverses each step once,
last step first, from a state it holds, never holds more than the allowed
number of states, and re-runs exactly as many forward steps as the fewest
any schedule can: the minimum over all first splits found by exhaustive
search, and Griewank and Walther's closed form for binomial checkpointing
(r n - C(c + r, c + 1))."""
from functools import lru_cache

import pytest

from paper_2604_09984_amd.adjoint import revolve_cost, revolve_schedule


@lru_cache(None)
def fewest(n, c):
    """Exhaustive minimum: put the first kept state after m steps (m forward
    steps), reverse the tail with one state fewer, then the head with c."""
    if n <= 1:
        return 0
    if c <= 1:
        return sum(range(n))
    return min(m + fewest(n - m, c - 1) + fewest(m, c) for m in range(1, n))


def replay(n, c):
    held, peak, runs, reversed_ = {0}, 0, 0, []
    for act in revolve_schedule(n, c):
        if act[0] == "advance":
            _, a, m = act
            assert a in held and m > a and m not in held
            held.add(m)
            runs += m - a
        elif act[0] == "reverse":
            assert act[1] in held
            reversed_.append(act[1])
        else:
            assert act[1] in held and act[1] != 0
            held.remove(act[1])
        peak = max(peak, len(held) - 1)
    return peak, runs, reversed_


@pytest.mark.parametrize("c", [1, 2, 3, 4, 6])
def test_schedule_reverses_every_step_once_within_its_states(c):
    for n in range(0, 41):
        peak, runs, order = replay(n, c)
        assert order == list(range(n - 1, -1, -1))
        assert peak <= max(c, 1)
        assert runs == revolve_cost(n, c)


def test_cost_is_the_exhaustive_minimum():
    for c in range(1, 7):
        for n in range(1, 31):
            assert revolve_cost(n, c) == fewest(n, c), (n, c)


def test_cost_special_cases():
    for n in range(1, 30):
        assert revolve_cost(n, n - 1 if n > 2 else 2) == n - 1   # every state kept: one forward sweep
        assert revolve_cost(n, 1) == n * (n - 1) // 2            # one working state: re-run from the input
    # 20 steps with 3 kept states: r = 3 (C(6, 3) = 20), 3 * 20 - C(6, 4) = 45
    assert revolve_cost(20, 3) == 45
