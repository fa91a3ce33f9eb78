"""Pins of the oracle's bond-dimension criterion (Config.criterion = "bond_dim").

* A maximally entangled qutrit pair (Schmidt rank 3) next to the word that undoes its
  preparation (SUM^-1, then F^3 = F^-1 on the first qutrit): that word leaves rank 1 and is
  chosen; the identity keeps rank 3.
* A product pair: no candidate goes below the identity's rank 1 (entangling ones raise it),
  so the identity stays.
* The paper's circuit (random Clifford layers, T on qudit 0) disentangled with the exhaustive
  set under the criterion in the exact regime: the state equals the dense simulation, and
  every accepted choice lowered the bond dimension of its split.
"""
import numpy as np

from oracle.clifford import word_matrix
from oracle.disentanglers import exhaustive_disentanglers
from oracle.gcamps import Config, Gcamps
from oracle.statevector import simulate
from paper_2511_06672_amd.workload import IDENTITY_WORD, Word, candidate_words, paper_circuit


def bare(d, cands):
    g = Gcamps(d, 2, Config(chi_max=d, cutoff=0.0, criterion="bond_dim"), cands)
    return g


def test_bell_pair_is_disentangled_by_the_inverse_preparation():
    d = 3
    bell = np.zeros((1, d, d, 1), complex)
    for j in range(d):
        bell[0, j, j, 0] = 1 / np.sqrt(d)
    undo = Word((5, 0, 0, 0), (0, 0, 0, 0))
    cands = [IDENTITY_WORD] + candidate_words(d, 8, 21)[1:] + [undo]
    g = bare(d, cands)
    r = g.ranks(bell)
    assert r[0] == 3 and r[-1] == 1
    rot = np.einsum("xy,ayb->axb", word_matrix(d, undo.gens, undo.weyl), bell.reshape(1, 9, 1))
    assert np.linalg.matrix_rank(rot.reshape(3, 3)) == 1
    c = g.select_bond_dim(bell)
    assert r[c] == 1


def test_product_pair_keeps_the_identity():
    d = 3
    prod = np.zeros((1, d, d, 1), complex)
    prod[0, 1, 2, 0] = 1.0
    g = bare(d, [IDENTITY_WORD] + candidate_words(d, 12, 22)[1:])
    r = g.ranks(prod)
    assert r[0] == 1 and r.min() == 1 and r.max() > 1      # entangling candidates raise it
    assert g.select_bond_dim(prod) == 0


def test_paper_circuit_exact_state_and_rank_decrease():
    d, n = 3, 5
    words = [Word(w, (0, 0, 0, 0)) for w in exhaustive_disentanglers(d)]
    c = paper_circuit(d, n, 4, 23)
    g = Gcamps(d, n, Config(chi_max=d ** 3, cutoff=0.0, criterion="bond_dim"), words)
    ranks_seen = []
    orig = g.select_bond_dim

    def spy(theta):
        ch = orig(theta)
        r = g.ranks(theta)
        ranks_seen.append((r[0], r[ch]))
        return ch

    g.select_bond_dim = spy
    for layer in c.layers:
        for b in layer.bricks:
            g.apply_clifford(b.site, b.word.gens, b.word.weyl)
        for ph in layer.phases:
            g.apply_phase_rotation(ph.site, ph.phi)
    psi, ref = g.statevector(), simulate(c)
    ov = np.vdot(psi, ref)
    assert np.max(np.abs(psi * (ov / abs(ov)) - ref)) < 1e-10
    assert ranks_seen and all(rc <= r0 for r0, rc in ranks_seen)
    assert any(rc < r0 for r0, rc in ranks_seen)            # the criterion did act
