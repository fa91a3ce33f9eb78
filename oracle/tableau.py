"""Z_d stabilizer tableau of the Clifford C in psi = C|MPS> (§2.2, §2.3, §2.3.1).

Layout (the paper leaves the column order open; this is the reading used
throughout): 2n rows, rows 0..n-1 are the stabilizers S_k = C Z_k C^dagger, rows
n..2n-1 the destabilizers D_k = C X_k C^dagger; each row is a Weyl string with
exponents x_0..x_{n-1} | z_0..z_{n-1} and a phase p in Z_{2d} (powers of tau).
The exported integer matrix is [2n][2n+1] = x | z | p.

Initial state C = I: S_k = Z_k, D_k = X_k, all phases zero.

* A Clifford gate G updates C <- G C, i.e. every row R -> G R G^dagger (top loop
  of Fig. 1, rules of Table 1 in ``clifford``).
* A disentangler Q updates C <- C Q^dagger (§3): for every Pauli P on the pair,
  C Q^dagger P Q C^dagger is the product of old rows given by the exponents of
  Q^dagger P Q.
* ``decompose`` expresses C^dagger W C for a Weyl target W: the exponents of the
  tableau rows are found by Gaussian elimination over the field Z_d (§2.3.1, so d
  must be prime) and the phase by multiplying the rows out explicitly, as §2.3.1
  describes.  ``decompose_closed_form`` is an independent derivation used as a
  cross-check: with the symplectic relations lam(D_j, S_k) = -delta_jk the
  exponents are delta_j = -lam(W, S_j), s_j = lam(W, D_j).
"""
from __future__ import annotations

from typing import Sequence, Tuple

import numpy as np

from .clifford import conj_word, conj_word_inverse
from .weyl import Weyl, lam


def _is_prime(d: int) -> bool:
    return d >= 2 and all(d % k for k in range(2, int(d ** 0.5) + 1))


class Tableau:
    def __init__(self, d: int, n: int):
        if not _is_prime(d):
            raise ValueError("the tableau decomposition needs a field: d must be prime")
        self.d, self.n = d, n
        self.x = np.zeros((2 * n, n), dtype=np.int64)
        self.z = np.zeros((2 * n, n), dtype=np.int64)
        self.p = np.zeros(2 * n, dtype=np.int64)
        for k in range(n):
            self.z[k, k] = 1          # S_k = Z_k
            self.x[n + k, k] = 1      # D_k = X_k

    def copy(self) -> "Tableau":
        t = Tableau.__new__(Tableau)
        t.d, t.n = self.d, self.n
        t.x, t.z, t.p = self.x.copy(), self.z.copy(), self.p.copy()
        return t

    def row(self, i: int) -> Weyl:
        return Weyl(self.d, self.x[i], self.z[i], int(self.p[i]))

    def S(self, k: int) -> Weyl:
        return self.row(k)

    def D(self, k: int) -> Weyl:
        return self.row(self.n + k)

    def set_row(self, i: int, w: Weyl):
        self.x[i], self.z[i], self.p[i] = w.x, w.z, w.p

    def export(self) -> np.ndarray:
        """[2n][2n+1] int matrix x | z | p."""
        return np.concatenate([self.x, self.z, self.p[:, None]], axis=1).astype(np.int64)

    # ------------------------------------------------------------ Clifford updates
    def apply_word(self, site: int, gens: Sequence[int], weyl: Sequence[int]):
        """C <- U C for the word U on (site, site+1): rows R -> U R U^dagger."""
        conj_word(self.d, self.x, self.z, self.p, site, gens, weyl)

    def right_multiply_dagger(self, site: int, gens: Sequence[int], weyl: Sequence[int]):
        """C <- C Q^dagger for the word Q on (site, site+1) (disentangler update, §3).

        For P in {Z_a, Z_b, X_a, X_b}: new row(P) = C (Q^dagger P Q) C^dagger.  Writing
        Q^dagger P Q = tau^q X_a^{x1} Z_a^{z1} X_b^{x2} Z_b^{z2}, this is the ordered product
        tau^q D_a^{x1} S_a^{z1} D_b^{x2} S_b^{z2} of the old rows.
        """
        n, d = self.n, self.d
        a, b = site, site + 1
        old = {"Sa": self.S(a), "Sb": self.S(b), "Da": self.D(a), "Db": self.D(b)}
        new_rows = {}
        for key, (site_p, kind) in {"Sa": (a, "Z"), "Sb": (b, "Z"),
                                    "Da": (a, "X"), "Db": (b, "X")}.items():
            x = np.zeros((1, n), np.int64)
            z = np.zeros((1, n), np.int64)
            p = np.zeros(1, np.int64)
            if kind == "Z":
                z[0, site_p] = 1
            else:
                x[0, site_p] = 1
            conj_word_inverse(d, x, z, p, a, gens, weyl)
            # Q^dagger P Q = tau^p X_a^{x[a]} Z_a^{z[a]} X_b^{x[b]} Z_b^{z[b]}
            acc = Weyl(d, np.zeros(n, np.int64), np.zeros(n, np.int64), int(p[0]))
            acc = acc * old["Da"].power(int(x[0, a]))
            acc = acc * old["Sa"].power(int(z[0, a]))
            acc = acc * old["Db"].power(int(x[0, b]))
            acc = acc * old["Sb"].power(int(z[0, b]))
            new_rows[key] = acc
        self.set_row(a, new_rows["Sa"])
        self.set_row(b, new_rows["Sb"])
        self.set_row(n + a, new_rows["Da"])
        self.set_row(n + b, new_rows["Db"])

    # ------------------------------------------------------------ decomposition
    def _solve_mod_d(self, target: Weyl) -> np.ndarray:
        """Gaussian elimination over Z_d: find y = [s; delta] with
        sum_j s_j vec(S_j) + delta_j vec(D_j) = vec(target)   (§2.3.1)."""
        d, n = self.d, self.n
        # columns of M are the vectors (x | z) of the 2n rows, in the order S_0..S_{n-1}, D_0..
        M = np.concatenate([self.x, self.z], axis=1).T % d           # (2n, 2n)
        rhs = np.concatenate([target.x, target.z]) % d
        A = np.concatenate([M, rhs[:, None]], axis=1).astype(np.int64)
        rows, cols = 2 * n, 2 * n
        piv_cols = []
        r = 0
        for c in range(cols):
            pr = None
            for i in range(r, rows):
                if A[i, c] % d:
                    pr = i
                    break
            if pr is None:
                continue
            A[[r, pr]] = A[[pr, r]]
            inv = pow(int(A[r, c]), d - 2, d)          # Fermat inverse, d prime
            A[r] = (A[r] * inv) % d
            for i in range(rows):
                if i != r and A[i, c] % d:
                    A[i] = (A[i] - A[i, c] * A[r]) % d
            piv_cols.append(c)
            r += 1
        if r != cols:
            raise ArithmeticError("tableau rows are not independent")
        y = np.zeros(cols, np.int64)
        for i, c in enumerate(piv_cols):
            y[c] = A[i, cols] % d
        return y

    def decompose(self, target: Weyl) -> Tuple[Weyl, np.ndarray, np.ndarray]:
        """C^dagger W C for the Weyl string W = target (bottom loop, §2.3.1, §3).

        Returns (P, s, delta): P = W(delta, s, p_W + 2<s, delta> - q) where the
        explicitly multiplied product prod_j S_j^{s_j} D_j^{delta_j} = tau^q W(t).
        """
        d, n = self.d, self.n
        y = self._solve_mod_d(target)
        s, delta = y[:n], y[n:]
        prod = Weyl.identity(d, n)
        for j in range(n):
            prod = prod * self.S(j).power(int(s[j]))
            prod = prod * self.D(j).power(int(delta[j]))
        if not (np.array_equal(prod.x, target.x % d) and np.array_equal(prod.z, target.z % d)):
            raise ArithmeticError("elimination result does not reproduce the target")
        q = prod.p
        # C^dagger S_j C = Z_j and C^dagger D_j C = X_j, so C^dagger prod C is the ordered
        # product of Z_j^{s_j} X_j^{delta_j} = omega^{s_j delta_j} X_j^{delta_j} Z_j^{s_j}.
        sd = int(np.dot(s, delta))
        P = Weyl(d, delta, s, target.p - q + 2 * sd)
        return P, s, delta

    def decompose_closed_form(self, target: Weyl) -> Tuple[np.ndarray, np.ndarray]:
        """Exponents from the symplectic relations (cross-check of the elimination)."""
        n = self.n
        delta = np.array([(-lam(target, self.S(j))) % self.d for j in range(n)], np.int64)
        s = np.array([lam(target, self.D(j)) % self.d for j in range(n)], np.int64)
        return s, delta

    def symplectic_ok(self) -> bool:
        """lam(S_j,S_k) = lam(D_j,D_k) = 0 and lam(D_j,S_k) = -delta_jk (mod d)."""
        n, d = self.n, self.d
        for j in range(n):
            for k in range(n):
                if lam(self.S(j), self.S(k)) != 0 or lam(self.D(j), self.D(k)) != 0:
                    return False
                if lam(self.D(j), self.S(k)) != ((-1 if j == k else 0) % d):
                    return False
        return True
