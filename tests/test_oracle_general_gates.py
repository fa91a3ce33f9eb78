"""Pins of the oracle's general non-Clifford gates (Gcamps.apply_gate, weyl_expansion).

* The Weyl expansion reconstructs U (sum c W = U), and for a diagonal U it has only Z-type
  terms equal to the DFT closed form already pinned for phase gates.
* In the exact regime (no truncation) applying U through the tableau and the MPO gives the
  dense product U psi, for one- and two-site U, qubits and qutrits (the plain definition of a
  gate, checked on the oracle's own dense state before and after).
* A diagonal U through apply_gate gives the same state as apply_phase_rotation.
"""
import numpy as np
import pytest

from oracle.gcamps import Config, Gcamps, diagonal_coefficients, weyl_expansion
from oracle.weyl import site_matrix
from paper_2511_06672_amd.workload import brickwork_circuit


def random_unitary(rng, D):
    q, r = np.linalg.qr(rng.normal(size=(D, D)) + 1j * rng.normal(size=(D, D)))
    return q * (np.diag(r) / np.abs(np.diag(r)))


def dense_apply(psi, d, n, site, u):
    k = 1 if u.shape[0] == d else 2
    v = psi.reshape(d ** site, d ** k, d ** (n - site - k))
    return np.einsum("xy,ayb->axb", u, v).reshape(-1)


def aligned(a, b):
    ov = np.vdot(a, b)
    return float(np.max(np.abs(a * (ov / abs(ov)) - b)))


def prepared(d, n, seed, layers=6):
    c = brickwork_circuit(d, n, layers, layers, seed)
    g = Gcamps(d, n, Config(chi_max=d ** n, cutoff=0.0, auto_disentangle=False), [])
    for layer in c.layers:
        for b in layer.bricks:
            g.apply_clifford(b.site, b.word.gens, b.word.weyl)
        for ph in layer.phases:
            g.apply_phase_rotation(ph.site, ph.phi)
    return g


@pytest.mark.parametrize("d,k", [(2, 1), (2, 2), (3, 1), (3, 2)])
def test_weyl_expansion_reconstructs(d, k):
    rng = np.random.default_rng(10 * d + k)
    u = random_unitary(rng, d ** k)
    terms = weyl_expansion(d, k, u)
    assert len(terms) <= d ** (2 * k)
    back = np.zeros_like(u)
    for x, z, c in terms:
        w = np.ones((1, 1))
        for t in range(k):
            w = np.kron(w, site_matrix(d, x[t], z[t]))
        back += c * w
    assert np.allclose(back, u, atol=1e-12)


@pytest.mark.parametrize("d", [2, 3])
def test_diagonal_gate_expansion_is_the_dft(d):
    phi = np.array([0.0, 0.7, -1.3][:d])
    terms = weyl_expansion(d, 1, np.diag(np.exp(1j * phi)))
    assert all(x == (0,) for x, _, _ in terms)
    c = dict((z[0], cz) for _, z, cz in terms)
    want = diagonal_coefficients(d, phi)
    for b in range(d):
        assert abs(c.get(b, 0.0) - want[b]) < 1e-12


@pytest.mark.parametrize("d,n,site,k", [(2, 6, 2, 1), (2, 6, 3, 2), (3, 5, 1, 1), (3, 5, 2, 2)])
def test_apply_gate_equals_dense_product(d, n, site, k):
    rng = np.random.default_rng(100 + 10 * d + k)
    g = prepared(d, n, 70 + d)
    psi0 = g.statevector()
    u = random_unitary(rng, d ** k)
    g.apply_gate(site, u)
    assert aligned(g.statevector(), dense_apply(psi0, d, n, site, u)) < 1e-10
    # and a second one on top, elsewhere
    u2 = random_unitary(rng, d ** k)
    psi1 = g.statevector()
    g.apply_gate(n - k - 1, u2)
    assert aligned(g.statevector(), dense_apply(psi1, d, n, n - k - 1, u2)) < 1e-10


@pytest.mark.parametrize("d", [2, 3])
def test_diagonal_apply_gate_equals_phase_rotation(d):
    phi = [0.0, 0.4, -2.1][:d]
    a = prepared(d, 5, 80 + d)
    b = prepared(d, 5, 80 + d)
    a.apply_phase_rotation(2, phi)
    b.apply_gate(2, np.diag(np.exp(1j * np.array(phi))))
    assert aligned(a.statevector(), b.statevector()) < 1e-12
    assert a.mps.bond_dims() == b.mps.bond_dims()
