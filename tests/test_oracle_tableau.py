"""Pins of the oracle tableau (§2.2, §2.3, §2.3.1) against dense Clifford matrices."""
import numpy as np
import pytest

from oracle.gcamps import Config, Gcamps
from oracle.tableau import Tableau
from oracle.weyl import Weyl
from paper_2511_06672_amd.workload import SplitMix64, random_word


def random_clifford_state(d, n, seed, nwords=6, candidates=()):
    rng = SplitMix64(seed)
    g = Gcamps(d, n, Config(chi_max=64, cutoff=0.0), candidates)
    for _ in range(nwords):
        site = rng.below(n - 1)
        w = random_word(rng, d, 12)
        g.apply_clifford(site, w.gens, w.weyl)
    return g, rng


@pytest.mark.parametrize("d,n", [(2, 4), (3, 3)])
def test_rows_equal_dense_conjugates(d, n):
    """S_k = C Z_k C^dagger and D_k = C X_k C^dagger with C the dense product of the words
    (bit-exact phases: the dense matrices agree to rounding, not up to a phase)."""
    g, _ = random_clifford_state(d, n, 11 * d + n)
    C = g.dense_clifford()
    for k in range(n):
        zk = Weyl(d, np.zeros(n, int), np.eye(n, dtype=int)[k], 0).dense()
        xk = Weyl(d, np.eye(n, dtype=int)[k], np.zeros(n, int), 0).dense()
        assert np.allclose(g.tab.S(k).dense(), C @ zk @ C.conj().T, atol=1e-10)
        assert np.allclose(g.tab.D(k).dense(), C @ xk @ C.conj().T, atol=1e-10)


@pytest.mark.parametrize("d,n", [(2, 6), (3, 5), (5, 3)])
def test_symplectic_invariant_after_random_words(d, n):
    g, _ = random_clifford_state(d, n, 5 + d, nwords=25)
    assert g.tab.symplectic_ok()


@pytest.mark.parametrize("d,n", [(2, 4), (3, 3), (3, 6), (5, 3)])
def test_elimination_equals_closed_form_and_dense(d, n):
    g, rng = random_clifford_state(d, n, 101 + d + n, nwords=10)
    C = g.dense_clifford() if d ** n <= 729 else None
    for trial in range(6):
        x = np.array([rng.below(d) for _ in range(n)])
        z = np.array([rng.below(d) for _ in range(n)])
        p = rng.below(2 * d) if d == 2 else 2 * rng.below(d)
        W = Weyl(d, x, z, p)
        P, s, delta = g.tab.decompose(W)
        s2, delta2 = g.tab.decompose_closed_form(W)
        assert np.array_equal(s, s2) and np.array_equal(delta, delta2)
        if C is not None:
            assert np.allclose(P.dense(), C.conj().T @ W.dense() @ C, atol=1e-10)


@pytest.mark.parametrize("d,n", [(2, 4), (3, 3)])
def test_disentangler_update_is_right_multiplication(d, n):
    """C <- C Q^dagger: the updated rows equal the dense conjugates of the new C."""
    from oracle.clifford import word_matrix
    g, rng = random_clifford_state(d, n, 3 * d + n, nwords=5)
    C = g.dense_clifford()
    site = 1
    q = random_word(rng, d, 20)
    t = g.tab.copy()
    t.right_multiply_dagger(site, q.gens, q.weyl)
    Q = word_matrix(d, q.gens, q.weyl)
    full = np.kron(np.kron(np.eye(d ** site), Q), np.eye(d ** (n - site - 2)))
    Cn = C @ full.conj().T
    for k in range(n):
        zk = Weyl(d, np.zeros(n, int), np.eye(n, dtype=int)[k], 0).dense()
        xk = Weyl(d, np.eye(n, dtype=int)[k], np.zeros(n, int), 0).dense()
        assert np.allclose(t.S(k).dense(), Cn @ zk @ Cn.conj().T, atol=1e-10)
        assert np.allclose(t.D(k).dense(), Cn @ xk @ Cn.conj().T, atol=1e-10)
    assert t.symplectic_ok()


def test_non_prime_dimension_rejected():
    with pytest.raises(ValueError):
        Tableau(4, 3)


def test_planted_mistake_in_rules_is_caught():
    """A sign error planted in the P rule's phase breaks the dense comparison."""
    from oracle import clifford as cl
    d = 3
    w = Weyl(d, [2], [1], 0)
    x, z, p = w.x.reshape(1, 1).copy(), w.z.reshape(1, 1).copy(), np.array([0])
    cl.conj_P(d, x, z, p, 0)
    good = Weyl(d, x[0], z[0], int(p[0]))
    bad = Weyl(d, x[0], z[0], int(p[0]) - 2 * 2)      # phase off by omega^-2
    u = cl.P_matrix(d)
    ref = u @ w.dense() @ u.conj().T
    assert np.allclose(good.dense(), ref)
    assert not np.allclose(bad.dense(), ref)
