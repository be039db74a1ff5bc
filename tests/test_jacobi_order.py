"""Host check of the column hand-off rules of the register-resident Jacobi kernel.

The kernel (k_jacobi_oe) runs the odd-even ordering on N = c + (c mod 2) positions:
even steps pair (2k, 2k+1), odd steps (2k+1, 2k+2) with positions N-1 and 0 left
alone, and the two columns of a pair trade positions.  Group k holds its two
columns in registers as (first, second); after a step it hands one column on:

- after an even step: position 2k holds `second`, which goes to group k-1 (cyclic);
  `second` is replaced by the column coming from group k+1;
- after an odd step: position 2k+2 holds `first` (for the idle group H-1, whose pair
  did not trade, the two are swapped first), which goes to group k+1 (cyclic);
  `first` is replaced by the column coming from group k-1.

These tests replay those rules on column indices and check that every pair of
columns meets exactly once per sweep of N steps, over several sweeps, and that
the held columns stay a permutation.
"""
import itertools

import pytest


def _sweep(N, first, second):
    H = N // 2
    met = []
    for st in range(N):
        odd = st & 1
        for k in range(H):
            if not (odd and k == H - 1):
                met.append(frozenset((first[k], second[k])))
        if not odd:
            sent = list(second)
            second = [sent[(k + 1) % H] for k in range(H)]
        else:
            first, second = list(first), list(second)
            first[H - 1], second[H - 1] = second[H - 1], first[H - 1]  # the idle pair
            sent = list(first)
            first = [sent[(k - 1) % H] for k in range(H)]
    return met, first, second


@pytest.mark.parametrize("N", [2, 4, 6, 66, 98, 118, 128])
def test_every_pair_meets_once_per_sweep(N):
    H = N // 2
    first, second = [2 * k for k in range(H)], [2 * k + 1 for k in range(H)]
    everything = {frozenset(p) for p in itertools.combinations(range(N), 2)}
    for _ in range(3):
        met, first, second = _sweep(N, first, second)
        assert len(met) == len(everything) and set(met) == everything
        assert sorted(first + second) == list(range(N))


def test_all_even_widths_up_to_160():
    for N in range(2, 162, 2):
        H = N // 2
        first, second = [2 * k for k in range(H)], [2 * k + 1 for k in range(H)]
        met, _, _ = _sweep(N, first, second)
        assert len(set(met)) == N * (N - 1) // 2 == len(met), N
