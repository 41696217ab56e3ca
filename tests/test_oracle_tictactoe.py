"""Tic-Tac-Toe pins of the oracle (rules: App. C; end rules in order,
Sec. 3.3; random policy, Sec. 6).

Pins are facts of the game itself, found by exhaustive enumeration:
255168 complete games (131184 won by the first player, 77904 by the second,
46080 drawn), their split by length, 5478 reachable positions of which 958
are terminal, and the exact outcome law of uniform-random play
(737/1260, 121/420, 8/63; mean length 3203/420).
"""
from fractions import Fraction

import numpy as np
import pytest

from oracle import ref
from tests.oracle_util import apply_seq

TTT = ref.Game(ref.TICTACTOE, 3, 3)


def test_complete_games_by_length_and_winner():
    ref.set_checks(True)
    before = ref.check_failures()
    total, tab, trunc = ref.count_games(TTT, ref.init(TTT, 1), 9)
    assert total == 255168 and trunc == 0
    assert tab[:, 1].sum() == 131184
    assert tab[:, 2].sum() == 77904
    assert tab[:, 0].sum() == 46080
    assert list(tab.sum(1)) == [0, 0, 0, 0, 0, 1440, 5328, 47952, 72576, 127872]
    # a draw needs a full board
    assert tab[:9, 0].sum() == 0
    # the first player only wins on odd plies, the second on even plies
    assert tab[0::2, 1].sum() == 0 and tab[1::2, 2].sum() == 0
    assert ref.check_failures() == before


def _children(s):
    m = ref.legal_mask(TTT, s)[0]
    for a in np.flatnonzero(m):
        c = s.copy()
        ref.step(TTT, c, [a], want_mask=False)
        yield int(a), c


def test_reachable_positions():
    seen = {}
    stack = [ref.init(TTT, 1)]
    while stack:
        s = stack.pop()
        key = s.board.tobytes()
        if key in seen:
            continue
        seen[key] = int(s.status[0])
        if s.status[0] == ref.RUNNING:
            stack.extend(c for _, c in _children(s))
    assert len(seen) == 5478
    assert sum(1 for v in seen.values() if v != ref.RUNNING) == 958


def test_exact_random_play_law():
    memo = {}

    def law(s):
        key = s.board.tobytes()
        if key in memo:
            return memo[key]
        if s.status[0] != ref.RUNNING:
            w = int(s.winner[0])
            res = ({w: Fraction(1)}, Fraction(0))
        else:
            kids = list(_children(s))
            acc, length = {}, Fraction(0)
            for _, c in kids:
                sub, L = law(c)
                for k, v in sub.items():
                    acc[k] = acc.get(k, Fraction(0)) + v / len(kids)
                length += (L + 1) / len(kids)
            res = (acc, length)
        memo[key] = res
        return res

    dist, mean_len = law(ref.init(TTT, 1))
    assert dist[1] == Fraction(737, 1260)
    assert dist[2] == Fraction(121, 420)
    assert dist[0] == Fraction(8, 63)
    assert mean_len == Fraction(3203, 420)


def _chi2(counts, probs):
    n = sum(counts)
    return sum((c - n * float(p)) ** 2 / (n * float(p)) for c, p in zip(counts, probs))


def test_philox_playouts_follow_the_exact_law():
    # the 1024-env workload and a large sample; 2 dof: P(chi2 > 13.8) = 0.001
    probs = [Fraction(737, 1260), Fraction(121, 420), Fraction(8, 63)]
    for n, seed in ((1024, 1), (200000, 2)):
        s = ref.init(TTT, n)
        rew, term, stats = ref.playout(TTT, s, seed, 0, threads=8)
        assert term.all() and (s.status == ref.TERMINAL).all()
        counts = [int(stats[1]), int(stats[2]), int(stats[3])]
        assert sum(counts) == n
        assert stats[0] == int(s.ply.astype(np.int64).sum())
        assert _chi2(counts, probs) < 13.8, counts
        mean_len = stats[0] / n
        # sd of the length is < 1.2 plies
        assert abs(mean_len - 3203 / 420) < 6 * 1.2 / np.sqrt(n)


def test_known_games():
    # top row for player 1 at ply 5
    s, tr = apply_seq(TTT, [0, 3, 1, 4, 2])
    assert s.status[0] == ref.TERMINAL and s.winner[0] == 1 and tr[-1] == ((1, -1), 1)
    # anti-diagonal for player 2 at ply 6
    s, tr = apply_seq(TTT, [0, 2, 1, 4, 8, 6])
    assert s.winner[0] == 2 and tr[-1] == ((-1, 1), 1)
    # a draw: X O X / X O O / O X X
    s, tr = apply_seq(TTT, [0, 1, 2, 4, 3, 5, 7, 6, 8])
    assert s.status[0] == ref.TERMINAL and s.winner[0] == 0 and tr[-1] == ((0, 0), 1)
    assert s.ply[0] == 9 and s.last_action[0] == 8
