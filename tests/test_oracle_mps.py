"""Pins of the oracle MPS layer (§2.4): truncation rule, centre moves, MPO, coefficients."""
import numpy as np
import pytest

from oracle.gcamps import diagonal_coefficients
from oracle.mps import MPS, rtrunc
from oracle.weyl import Z_matrix


def random_mps(d, dims, seed):
    """Random normalised MPS with the given bond dims, centre on the last site."""
    rng = np.random.default_rng(seed)
    n = len(dims) + 1
    full = [1] + list(dims) + [1]
    ts = [rng.normal(size=(full[i], d, full[i + 1])) + 1j * rng.normal(size=(full[i], d, full[i + 1]))
          for i in range(n)]
    m = MPS(d, ts, 0)
    m.move_centre(n - 1)
    m.tensors[n - 1] /= np.linalg.norm(m.tensors[n - 1])
    return m


def test_rtrunc_special_cases():
    s = np.array([1.0, 0.5, 0.25, 1e-15])
    k, eps, f = rtrunc(s, 0.0, 10)
    assert k == 3 and not f                                  # rank floor drops 1e-15
    k, eps, f = rtrunc(s, 0.0, 2)
    assert k == 2 and np.isclose(eps, (0.25 ** 2 + 1e-30) / np.sum(s ** 2))
    w = s ** 2 / np.sum(s ** 2)
    k, eps, f = rtrunc(s, w[2] * 1.01, 10)                    # tail after 2 values <= cutoff
    assert k == 2 and np.isclose(eps, w[2] + w[3])
    # degenerate block cut by chi_max is dropped as a whole
    s = np.array([1.0, 0.5, 0.5, 0.5, 0.1])
    k, eps, f = rtrunc(s, 0.0, 2)
    assert k == 1 and not f
    # a block starting at index 0 keeps chi_max and is flagged
    s = np.ones(5)
    k, eps, f = rtrunc(s, 0.0, 3)
    assert k == 3 and f and np.isclose(eps, 0.4)


def test_centre_moves_preserve_state_and_orthonormality():
    d = 3
    m = random_mps(d, [3, 5, 4], 1)
    v0 = m.to_dense()
    for target in (0, 2, 1, 3):
        m.move_centre(target)
        assert np.allclose(m.to_dense(), v0)
        for i, t in enumerate(m.tensors):
            cl, _, cr = t.shape
            if i < target:
                a = t.reshape(cl * d, cr)
                assert np.allclose(a.conj().T @ a, np.eye(cr))
            elif i > target:
                a = t.reshape(cl, d * cr)
                assert np.allclose(a @ a.conj().T, np.eye(cl))


def test_svd_sweep_gives_schmidt_values():
    """After truncate_sweep_left without truncation the state is unchanged and each
    bond carries the Schmidt rank of the dense vector (library SVD as brute force)."""
    d = 2
    m = random_mps(d, [2, 4, 2], 3)
    v0 = m.to_dense()
    m.truncate_sweep_left(0, 3, 0.0, 100)
    assert np.allclose(m.to_dense(), v0)
    for cut in range(1, 4):
        sv = np.linalg.svd(v0.reshape(d ** cut, -1), compute_uv=False)
        assert m.bond_dims()[cut - 1] == int(np.sum(sv > 1e-13 * sv[0]))


def test_bond_renyi2_against_dense_cuts():
    """bond_renyi2 on an MPS in a random gauge (an invertible matrix and its inverse inserted on
    every bond) equals -ln sum p^2 from the singular values of the dense vector reshaped across
    each cut; a product state gives 0 everywhere and a maximally entangled pair ln d."""
    from oracle.mps import bond_renyi2
    rng = np.random.default_rng(11)
    d = 3
    m = random_mps(d, [3, 5, 4], 2)
    v0 = m.to_dense()
    ts = [t.copy() for t in m.tensors]
    for i in range(len(ts) - 1):
        k = ts[i].shape[2]
        x = rng.standard_normal((k, k)) + 1j * rng.standard_normal((k, k)) + 3 * np.eye(k)
        ts[i] = np.einsum("asb,bc->asc", ts[i], x)
        ts[i + 1] = np.einsum("cb,bsa->csa", np.linalg.inv(x), ts[i + 1])
    got = bond_renyi2(ts)
    for cut in range(1, 4):
        sv = np.linalg.svd(v0.reshape(d ** cut, -1), compute_uv=False)
        p = sv ** 2 / np.sum(sv ** 2)
        assert abs(got[cut - 1] + np.log(np.sum(p ** 2))) < 1e-12
    prod = [np.ones((1, d, 1), np.complex128) / np.sqrt(d) for _ in range(4)]
    assert np.allclose(bond_renyi2(prod), 0.0, atol=1e-14)
    # |00> + |11> + |22> on sites (1, 2) of a 4-site chain
    a = np.zeros((1, d, d), np.complex128)
    b = np.zeros((d, d, 1), np.complex128)
    for s in range(d):
        a[0, s, s] = 1 / np.sqrt(d)
        b[s, s, 0] = 1.0
    pair = [np.eye(1, d).reshape(1, d, 1).astype(np.complex128), a, b, np.eye(1, d).reshape(1, d, 1).astype(np.complex128)]
    assert np.allclose(bond_renyi2(pair), [0.0, np.log(d), 0.0], atol=1e-13)


def test_diagonal_coefficients_closed_form():
    for d in (2, 3, 5):
        rng = np.random.default_rng(d)
        phi = rng.uniform(0, 2 * np.pi, d)
        c = diagonal_coefficients(d, phi)
        # DFT closed form c_b = (1/d) sum_j e^{i phi_j} omega^{-bj}
        w = np.exp(2j * np.pi / d)
        dft = np.array([np.mean(np.exp(1j * phi) * w ** (-b * np.arange(d))) for b in range(d)])
        assert np.allclose(c, dft)
        assert np.isclose(np.sum(np.abs(c) ** 2), 1.0)       # unitary diag => sum |c_b|^2 = 1
        U = sum(c[b] * np.linalg.matrix_power(Z_matrix(d), b) for b in range(d))
        assert np.allclose(U, np.diag(np.exp(1j * phi)))


def test_qubit_t_gate_from_paper():
    """§2.3.2 prints T_2 = diag(1, e^{i pi/4}); its Z-decomposition is
    c = ((1 + e^{i pi/4})/2, (1 - e^{i pi/4})/2)."""
    import os
    line = [l for l in open(os.path.join(os.path.dirname(__file__), "golden", "t_gates.txt"))
            if not l.startswith("#")][0].split()
    d, phi = int(line[0]), [float(v) * np.pi for v in line[1:]]
    c = diagonal_coefficients(d, phi)
    e = np.exp(1j * np.pi / 4)
    assert np.allclose(c, [(1 + e) / 2, (1 - e) / 2])


def test_block_mpo_equals_dense_operator():
    d, n = 3, 4
    m = random_mps(d, [2, 3, 2], 9)
    rng = np.random.default_rng(4)
    ops = [[np.linalg.qr(rng.normal(size=(d, d)) + 1j * rng.normal(size=(d, d)))[0] for _ in range(3)]
           for _ in range(d)]
    coeff = rng.normal(size=d) + 1j * rng.normal(size=d)
    v0 = m.to_dense()
    m.apply_block_mpo(1, 3, ops, coeff)
    dense = sum(coeff[b] * np.kron(np.eye(d), np.kron(ops[b][0], np.kron(ops[b][1], ops[b][2])))
                for b in range(d))
    assert np.allclose(m.to_dense(), dense @ v0)
    assert m.bond_dims() == [2, 9, 6]
