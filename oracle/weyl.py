"""Generalised Pauli (Weyl) operators for qudits of dimension d (§2.3).

Definitions taken from §2.3: omega = exp(2 pi i / d), X|j> = |j+1 mod d>,
Z|j> = omega^j |j>, so that X Z = omega^{-1} Z X.  For even d the paper introduces
tau = omega^{1/2}; we use tau = exp(i pi / d) for every d and store every phase
as a power of tau in Z_{2d}.

A Weyl string on n qudits is W(x, z, p) = tau^p (X^{x_0} Z^{z_0}) (x) ... (x)
(X^{x_{n-1}} Z^{z_{n-1}}) with x, z in Z_d^n (site 0 is the most significant
tensor factor everywhere in this package).

Product rule (derived from Z X = omega X Z, one commutation per site):
    W(x,z,p) W(x',z',p') = W(x+x', z+z', p+p'+2<z,x'>)
Power rule (induction on the product rule):
    W(x,z,p)^b = W(bx, bz, bp + 2<x,z> b(b-1)/2)
Commutation: W(r) W(r') = omega^{lam(r,r')} W(r') W(r), lam = <z,x'> - <x,z'>.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


def tau(d: int) -> complex:
    return np.exp(1j * np.pi / d)


def omega(d: int) -> complex:
    return np.exp(2j * np.pi / d)


def X_matrix(d: int) -> np.ndarray:
    """X|j> = |j+1 mod d> (§2.3)."""
    m = np.zeros((d, d), dtype=np.complex128)
    for j in range(d):
        m[(j + 1) % d, j] = 1.0
    return m


def Z_matrix(d: int) -> np.ndarray:
    """Z|j> = omega^j |j> (§2.3)."""
    return np.diag([omega(d) ** j for j in range(d)]).astype(np.complex128)


def site_matrix(d: int, x: int, z: int) -> np.ndarray:
    """X^x Z^z as a dense d x d matrix."""
    return np.linalg.matrix_power(X_matrix(d), x % d) @ np.linalg.matrix_power(Z_matrix(d), z % d)


@dataclass
class Weyl:
    """W(x, z, p) = tau^p prod_i X_i^{x_i} Z_i^{z_i}; x, z mod d, p mod 2d."""
    d: int
    x: np.ndarray
    z: np.ndarray
    p: int

    def __post_init__(self):
        self.x = np.asarray(self.x, dtype=np.int64) % self.d
        self.z = np.asarray(self.z, dtype=np.int64) % self.d
        self.p = int(self.p) % (2 * self.d)

    @property
    def n(self) -> int:
        return len(self.x)

    @staticmethod
    def identity(d: int, n: int) -> "Weyl":
        return Weyl(d, np.zeros(n, np.int64), np.zeros(n, np.int64), 0)

    def copy(self) -> "Weyl":
        return Weyl(self.d, self.x.copy(), self.z.copy(), self.p)

    def key(self):
        return (tuple(int(v) for v in self.x), tuple(int(v) for v in self.z), self.p)

    def __eq__(self, other) -> bool:  # type: ignore[override]
        return isinstance(other, Weyl) and self.d == other.d and self.key() == other.key()

    def __mul__(self, other: "Weyl") -> "Weyl":
        """Operator product self * other (product rule above)."""
        d = self.d
        cross = int(np.dot(self.z, other.x))
        return Weyl(d, self.x + other.x, self.z + other.z, self.p + other.p + 2 * cross)

    def power(self, b: int) -> "Weyl":
        """self^b for b >= 0 (power rule above)."""
        d = self.d
        b = int(b)
        xz = int(np.dot(self.x, self.z))
        return Weyl(d, b * self.x, b * self.z, b * self.p + 2 * xz * (b * (b - 1) // 2))

    def dense(self) -> np.ndarray:
        """Dense d^n x d^n matrix (small n only)."""
        m = np.array([[1.0 + 0j]])
        for xi, zi in zip(self.x, self.z):
            m = np.kron(m, site_matrix(self.d, int(xi), int(zi)))
        return (tau(self.d) ** self.p) * m


def lam(a: Weyl, b: Weyl) -> int:
    """Symplectic form lam(a, b) = <z_a, x_b> - <x_a, z_b> mod d."""
    return int(np.dot(a.z, b.x) - np.dot(a.x, b.z)) % a.d
