"""Pins of the oracle's exhaustive disentangler sets (oracle/disentanglers.py), and the
library's own enumeration (gcamps_clifford_words, host code) checked against them.

Pins (none of them re-runs the oracle's own procedure):
* the counts §3 prints (20 for d = 2, 90 for d = 3; tests/golden/paper_counts.txt) and the closed
  forms |Sp(4, Z_d)| = d^4 (d^2 - 1)(d^4 - 1), |SL(2, Z_d)|^2 single-qudit Cliffords;
* each symplectic matrix against dense conjugation of the word's unitary;
* every generated matrix preserves the symplectic form; all classes have the same size;
* brute force: on random two-site tensors the best score over the exhaustive set equals the best
  over the whole Clifford group (the property the set exists for), and the score is constant on
  each class.
"""
import os

import numpy as np
import pytest

from oracle.clifford import word_matrix
from oracle.disentanglers import (all_cliffords, canonical_form, exhaustive_disentanglers, local_cliffords,
                                  symplectic)
from oracle.gcamps import renyi2
from oracle.weyl import site_matrix

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def paper_counts():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "paper_counts.txt")) if not l.startswith("#")]
    return {int(a): int(b) for a, b in rows}


def weyl_pair(d, v):
    return np.kron(site_matrix(d, v[0], v[1]), site_matrix(d, v[2], v[3]))


def is_multiple(a, b):
    """a = c b for a complex number c of modulus 1."""
    k = np.argmax(np.abs(b))
    c = a.flat[k] / b.flat[k]
    return abs(abs(c) - 1) < 1e-9 and np.allclose(a, c * b, atol=1e-9)


@pytest.mark.parametrize("d", [2, 3])
def test_counts(d):
    cl = all_cliffords(d)
    assert len(cl) == d ** 4 * (d * d - 1) * (d ** 4 - 1)
    assert len(local_cliffords(d)) == (d * (d * d - 1)) ** 2
    words = exhaustive_disentanglers(d)
    assert len(words) == paper_counts()[d] == d * d * (d * d + 1)
    assert words[0] == ()


@pytest.mark.parametrize("d", [2, 3])
def test_symplectic_matrix_against_dense_conjugation(d):
    rng = np.random.default_rng(11 + d)
    for _ in range(12):
        gens = tuple(int(g) for g in rng.integers(0, 6, size=rng.integers(1, 9)))
        u = word_matrix(d, gens, (0, 0, 0, 0))
        s = symplectic(d, gens)
        for c in range(4):
            e = np.zeros(4, np.int64)
            e[c] = 1
            img = u @ weyl_pair(d, e) @ u.conj().T
            assert is_multiple(img, weyl_pair(d, s[:, c]))


@pytest.mark.parametrize("d", [2, 3])
def test_symplectic_form_and_equal_classes(d):
    omega = np.array([[0, 1, 0, 0], [-1, 0, 0, 0], [0, 0, 0, 1], [0, 0, -1, 0]])
    cl = all_cliffords(d)
    local = np.stack(local_cliffords(d))
    sizes = {}
    for i, (_, s) in enumerate(cl):
        if i % 97 == 0 or d == 2:
            assert np.array_equal((s.T @ omega @ s) % d, omega % d)
        k = canonical_form(d, s, local)
        sizes[k] = sizes.get(k, 0) + 1
    assert len(sizes) == paper_counts()[d]
    assert set(sizes.values()) == {len(local)}


@pytest.mark.parametrize("d,chi,trials", [(2, 2, 3), (3, 1, 2)])
def test_exhaustive_set_is_optimal_by_brute_force(d, chi, trials):
    rng = np.random.default_rng(50 + d)
    cl = all_cliffords(d)
    mats = [word_matrix(d, w, (0, 0, 0, 0)) for w, _ in cl]
    best = set(exhaustive_disentanglers(d))
    local = np.stack(local_cliffords(d))
    for _ in range(trials):
        th = rng.normal(size=(chi, d, d, chi)) + 1j * rng.normal(size=(chi, d, d, chi))
        t = th.reshape(chi, d * d, chi)
        scores = np.array([renyi2(np.einsum("xy,ayb->axb", q, t).reshape(th.shape)) for q in mats])
        sub = np.array([scores[i] for i, (w, _) in enumerate(cl) if w in best])
        assert abs(sub.min() - scores.min()) < 1e-12
        # constant on classes: every member scores like its class's representative
        by_class = {}
        for i, (_, s) in enumerate(cl[:: 7 if d == 3 else 1]):
            k = canonical_form(d, s, local)
            by_class.setdefault(k, []).append(scores[i * (7 if d == 3 else 1)])
        for v in by_class.values():
            assert max(v) - min(v) < 1e-10


@pytest.mark.parametrize("d", [2, 3])
def test_library_enumeration_matches_oracle(d):
    """gcamps_clifford_words (host code, a different search) against the oracle's sets."""
    from paper_2511_06672_amd import gcamps as g
    local = np.stack(local_cliffords(d))
    mine = g.clifford_words(d, g.WORDS_DISENTANGLERS)
    assert mine[0].gens == () and all(w.weyl == (0, 0, 0, 0) for w in mine)
    keys = [canonical_form(d, symplectic(d, w.gens), local) for w in mine]
    want = {canonical_form(d, symplectic(d, w), local) for w in exhaustive_disentanglers(d)}
    assert len(keys) == len(set(keys)) == paper_counts()[d]
    assert set(keys) == want
    allw = g.clifford_words(d, g.WORDS_ALL)
    assert allw[0].gens == ()
    mats = {symplectic(d, w.gens).tobytes() for w in allw}
    assert len(allw) == len(mats) == len(all_cliffords(d))
