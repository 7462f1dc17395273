"""Host logic of the targeted Jacobi passes (lrr_diag_plan_rounds, no GPU).

After a check of the off-diagonal entries the solver marks the index-block
pairs that still need rotations; when few are marked it runs only rounds that
cover them.  Every round must be a perfect matching of the nb index blocks (the
tile updates of a round assume that every block belongs to exactly one pair),
and the rounds together must cover every marked pair: an off-diagonal mark
(p, q) needs p and q paired in some round, a mark inside block p needs p in
any pair (a pair solve sweeps inside both of its blocks)."""
import numpy as np
import pytest

from paper_1304_5583_amd import binding as B


def _check(need, rounds, pairs):
    nb = need.shape[0]
    together = set()
    for r in range(rounds):
        p, q = pairs[r, :, 0], pairs[r, :, 1]
        assert np.all(p < q) and np.all(q < nb)
        assert np.array_equal(np.sort(np.concatenate([p, q])), np.arange(nb)), "not a perfect matching"
        together |= set(zip(p.tolist(), q.tolist()))
    for p in range(nb):
        for q in range(p + 1, nb):
            if need[p, q]:
                assert (p, q) in together
    if rounds > 0:
        return
    assert not np.triu(need).any()


def test_nothing_marked_needs_no_round():
    r, _ = B.lrr_diag_plan_rounds(np.zeros((8, 8)), 7)
    assert r == 0


def test_single_pair_and_inner_marks():
    need = np.zeros((32, 32), dtype=np.int32)
    need[3, 17] = 1
    r, pairs = B.lrr_diag_plan_rounds(need, 15)
    assert r == 1 and (3, 17) in set(map(tuple, pairs[0].tolist()))
    _check(need, r, pairs)
    need = np.zeros((6, 6), dtype=np.int32)
    need[2, 2] = need[5, 5] = 1          # inside blocks 2 and 5 only
    r, pairs = B.lrr_diag_plan_rounds(need, 5)
    assert r == 1 and (2, 5) in set(map(tuple, pairs[0].tolist()))   # marked blocks go together
    _check(need, r, pairs)


def test_band_of_neighbours_needs_two_rounds():
    """(p, p + 1) for every p: the even and the odd neighbour pairs."""
    nb = 32
    need = np.zeros((nb, nb), dtype=np.int32)
    for p in range(nb - 1):
        need[p, p + 1] = 1
    r, pairs = B.lrr_diag_plan_rounds(need, 15)
    assert r == 2
    _check(need, r, pairs)


def test_cap_too_small_and_complete_graph():
    nb = 8
    need = np.triu(np.ones((nb, nb), dtype=np.int32))
    r, _ = B.lrr_diag_plan_rounds(need, 3)
    assert r == -1                       # 28 pairs, 4 per round: at least 7 rounds
    r, pairs = B.lrr_diag_plan_rounds(need, 20)
    assert nb - 1 <= r <= 20
    _check(need, r, pairs)


@pytest.mark.parametrize("seed", range(6))
def test_random_marks(seed):
    rng = np.random.default_rng(seed)
    for _ in range(50):
        nb = 2 * int(rng.integers(1, 40))
        dens = float(rng.choice([0.005, 0.02, 0.08, 0.3]))
        need = (rng.random((nb, nb)) < dens).astype(np.int32)
        r, pairs = B.lrr_diag_plan_rounds(need, nb - 1)
        if r < 0:
            continue
        _check(need, r, pairs)


def test_invalid_arguments():
    for nb in (1, 3, 7):
        with pytest.raises(B.LRRError) as e:
            B.lrr_diag_plan_rounds(np.zeros((nb, nb)), 2)
        assert e.value.status == B.LRR_EINVAL
    with pytest.raises(B.LRRError):
        B.lrr_diag_plan_rounds(np.zeros((4, 4)), -1)
