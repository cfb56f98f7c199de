"""The multicolour order: a symmetric permutation under which rows of one
colour share no stored entry, so updating them together is the same as the
sequential sweep of eqs (4)-(5) on P C P^T."""

import numpy as np
import pytest

import gen
import oracle


def _edges(m):
    rows = np.repeat(np.arange(m.n), np.diff(m.row_ptr))
    cols = m.col.astype(np.int64)
    off = rows != cols
    return rows[off], cols[off]


def _check_coloring(m, color, order, nc):
    r, c = _edges(m)
    assert not np.any(color[r] == color[c]), "same-colour edge"
    assert np.array_equal(np.sort(order), np.arange(m.n))
    assert np.all(np.diff(color[order]) >= 0), "colours not contiguous"
    for k in range(nc):
        rows_k = order[color[order] == k]
        assert np.all(np.diff(rows_k) > 0)
    assert color.min() == 0 and color.max() == nc - 1


@pytest.mark.parametrize("maker", [
    lambda: gen.random_dominant(200, seed=1000),
    lambda: gen.pedigree(3000, seed=5),
    lambda: gen.lattice(4, seed=3),
    lambda: gen.lattice(5, seed=3),
])
def test_coloring_valid(maker):
    m = maker()
    color, order, nc = oracle.greedy_color(m)
    _check_coloring(m, color, order, nc)


def test_coloring_is_greedy_first_fit():
    """Brute force on a small matrix: every row takes the smallest colour that
    no earlier neighbour (either direction) holds."""
    m = gen.random_dominant(60, seed=4)
    color, _, _ = oracle.greedy_color(m)
    A = gen.to_dense(m) != 0
    S = A | A.T
    for i in range(m.n):
        used = {int(color[j]) for j in range(i) if S[i, j]}
        c = 0
        while c in used:
            c += 1
        assert color[i] == c


def test_even_lattice_two_colours():
    m = gen.lattice(4, seed=1)
    color, order, nc = oracle.greedy_color(m)
    assert nc == 2
    L = 4
    site = np.arange(m.n)
    parity = sum((site // L ** mu) % L for mu in range(4)) % 2
    assert np.array_equal(color, parity)


def test_pedigree_few_colours():
    m = gen.pedigree(20000, seed=1001)
    _, _, nc = oracle.greedy_color(m)
    assert 3 <= nc <= 12
