"""Pins of the oracle's round-robin ordering (a cyclic parallel strategy in the
sense of Section 6.3, with a bye for odd n as in Section 6.3.2)."""
import itertools

import pytest


@pytest.mark.parametrize("n", [2, 3, 4, 7, 8, 64, 65, 300])
def test_round_robin_covers_each_pair_once(oracle, n):
    steps, pp, qq = oracle.round_robin(n)
    N = n + (n % 2)
    assert steps == N - 1
    seen = set()
    for s in range(steps):
        used = set()
        for p, q in zip(pp[s], qq[s]):
            if p < 0:
                assert n % 2 == 1
                continue
            assert 0 <= p < q < n
            assert p not in used and q not in used
            used.update((p, q))
            assert (p, q) not in seen
            seen.add((p, q))
        # a step holds floor(n/2) pairs
        assert len(used) == 2 * (n // 2)
    assert seen == set(itertools.combinations(range(n), 2))
