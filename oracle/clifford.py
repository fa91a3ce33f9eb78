"""Qudit Clifford gates (§2.3) and their action on Weyl strings (Table 1).

Gate matrices, as defined in §2.3:
    H_d = F = d^{-1/2} sum_{ij} omega^{ij} |j><i|
    S_d = P = sum_j omega^{j(j-1)/2} |j><j|          (odd d)
            = sum_j tau^{j^2} |j><j|                  (even d)
    SUM_d |i, j> = |i, i + j mod d>

Conjugation rules U W U^dagger on the exponents (x, z) of the acted site(s) and
the tau-phase p.  They extend Table 1 (H: X->Z, Z->X^-1; S: X->tau XZ = Y, Z->Z;
SUM: X(x)I -> X(x)X, I(x)Z -> Z^-1(x)Z, others fixed) to arbitrary powers with the
phase tracked exactly:
    F:        (x, z, p) -> (-z, x, p - 2xz)
    P, odd d: (x, z, p) -> (x, z + x, p + x(x-1))
    P, even:  (x, z, p) -> (x, z + x, p + x^2)
    X^a Z^b:  (x, z, p) -> (x, z, p + 2(b x - a z))
    SUM a->b: x_b += x_a, z_a -= z_b            (p unchanged)
    SUM^-1:   x_b -= x_a, z_a += z_b            (p unchanged)
Each rule is pinned in the tests by dense conjugation of the matrices above.

A two-qudit *word* (gens, weyl) is the unitary U = (X^w0 Z^w1 (x) X^w2 Z^w3)
G_{L-1} ... G_1 G_0 on the ordered pair (a, b) = (site, site+1); generator codes
0..5 are F_a, F_b, P_a, P_b, SUM_{a->b}, SUM^{-1}_{a->b}.

Rules act in place on arrays of rows: ``x``, ``z`` of shape (rows, n) and ``p``
of shape (rows,), all int64.
"""
from __future__ import annotations

from typing import Sequence

import numpy as np

from .weyl import X_matrix, Z_matrix, Weyl, omega, tau


# ---------------------------------------------------------------- dense matrices

def F_matrix(d: int) -> np.ndarray:
    w = omega(d)
    m = np.zeros((d, d), dtype=np.complex128)
    for i in range(d):
        for j in range(d):
            m[j, i] = w ** (i * j)
    return m / np.sqrt(d)


def P_matrix(d: int) -> np.ndarray:
    if d % 2 == 1:
        return np.diag([omega(d) ** (j * (j - 1) // 2) for j in range(d)]).astype(np.complex128)
    return np.diag([tau(d) ** (j * j) for j in range(d)]).astype(np.complex128)


def SUM_matrix(d: int) -> np.ndarray:
    m = np.zeros((d * d, d * d), dtype=np.complex128)
    for i in range(d):
        for j in range(d):
            m[i * d + (i + j) % d, i * d + j] = 1.0
    return m


def generator_matrix(d: int, g: int) -> np.ndarray:
    """d^2 x d^2 matrix of generator code g on the ordered pair (a, b)."""
    I = np.eye(d, dtype=np.complex128)
    if g == 0:
        return np.kron(F_matrix(d), I)
    if g == 1:
        return np.kron(I, F_matrix(d))
    if g == 2:
        return np.kron(P_matrix(d), I)
    if g == 3:
        return np.kron(I, P_matrix(d))
    if g == 4:
        return SUM_matrix(d)
    if g == 5:
        return SUM_matrix(d).conj().T
    raise ValueError(g)


def weyl_shift_matrix(d: int, weyl: Sequence[int]) -> np.ndarray:
    def xz(a, b):
        return np.linalg.matrix_power(X_matrix(d), a % d) @ np.linalg.matrix_power(Z_matrix(d), b % d)
    return np.kron(xz(weyl[0], weyl[1]), xz(weyl[2], weyl[3]))


def word_matrix(d: int, gens: Sequence[int], weyl: Sequence[int]) -> np.ndarray:
    """U = Weyl * G_{L-1} ... G_0 as a d^2 x d^2 matrix (row index s_a * d + s_b)."""
    u = np.eye(d * d, dtype=np.complex128)
    for g in gens:
        u = generator_matrix(d, g) @ u
    return weyl_shift_matrix(d, weyl) @ u


# ---------------------------------------------------------------- conjugation rules

def conj_F(d, x, z, p, a, inverse=False):
    xa = x[:, a].copy()
    za = z[:, a].copy()
    if not inverse:          # (x, z, p) -> (-z, x, p - 2xz)
        x[:, a] = (-za) % d
        z[:, a] = xa % d
    else:                    # inverse map: (x, z, p) -> (z, -x, p - 2xz)
        x[:, a] = za % d
        z[:, a] = (-xa) % d
    p[:] = (p - 2 * xa * za) % (2 * d)


def conj_P(d, x, z, p, a, inverse=False):
    xa = x[:, a]
    sgn = -1 if inverse else 1
    z[:, a] = (z[:, a] + sgn * xa) % d
    if d % 2 == 1:
        p[:] = (p + sgn * xa * (xa - 1)) % (2 * d)
    else:
        p[:] = (p + sgn * xa * xa) % (2 * d)


def conj_SUM(d, x, z, p, a, b, inverse=False):
    sgn = -1 if inverse else 1
    x[:, b] = (x[:, b] + sgn * x[:, a]) % d
    z[:, a] = (z[:, a] - sgn * z[:, b]) % d


def conj_weyl(d, x, z, p, a, alpha, beta, inverse=False):
    sgn = -1 if inverse else 1
    p[:] = (p + sgn * 2 * (beta * x[:, a] - alpha * z[:, a])) % (2 * d)


def _apply_gen(d, x, z, p, g, a, b, inverse):
    if g == 0:
        conj_F(d, x, z, p, a, inverse)
    elif g == 1:
        conj_F(d, x, z, p, b, inverse)
    elif g == 2:
        conj_P(d, x, z, p, a, inverse)
    elif g == 3:
        conj_P(d, x, z, p, b, inverse)
    elif g == 4:
        conj_SUM(d, x, z, p, a, b, inverse)
    elif g == 5:
        conj_SUM(d, x, z, p, a, b, not inverse)
    else:
        raise ValueError(g)


def conj_word(d, x, z, p, a, gens, weyl):
    """Rows <- U rows U^dagger for the word U acting on (a, a+1)."""
    b = a + 1
    for g in gens:
        _apply_gen(d, x, z, p, g, a, b, False)
    conj_weyl(d, x, z, p, a, weyl[0], weyl[1])
    conj_weyl(d, x, z, p, b, weyl[2], weyl[3])


def conj_word_inverse(d, x, z, p, a, gens, weyl):
    """Rows <- U^dagger rows U (the inverse conjugation, rules undone in reverse)."""
    b = a + 1
    conj_weyl(d, x, z, p, b, weyl[2], weyl[3], inverse=True)
    conj_weyl(d, x, z, p, a, weyl[0], weyl[1], inverse=True)
    for g in reversed(list(gens)):
        _apply_gen(d, x, z, p, g, a, b, True)


def conj_weyl_string(w: Weyl, a: int, gens, weyl, inverse=False) -> Weyl:
    """U W U^dagger (or U^dagger W U) for one Weyl string."""
    x = w.x.reshape(1, -1).copy()
    z = w.z.reshape(1, -1).copy()
    p = np.array([w.p], dtype=np.int64)
    if inverse:
        conj_word_inverse(w.d, x, z, p, a, gens, weyl)
    else:
        conj_word(w.d, x, z, p, a, gens, weyl)
    return Weyl(w.d, x[0], z[0], int(p[0]))
