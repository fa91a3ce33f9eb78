"""Matrix product states (§2.4, Eq. (MPS)) for the oracle.

psi(s_0..s_{n-1}) = A^(0)_{s_0} A^(1)_{s_1} ... A^(n-1)_{s_{n-1}}, each site tensor
stored as a complex128 array of shape (chi_left, d, chi_right), site 0 the most
significant digit of the dense index.  ``centre`` is the orthogonality centre:
sites left of it are left-orthonormal, sites right of it right-orthonormal.

Truncation rule (the paper only says a fixed number of singular values is kept;
this is the reading used everywhere, R-TRUNC):
  w_j = sigma_j^2 / sum sigma^2 (sigma sorted descending)
  k_cut   = smallest k >= 1 with sum_{j >= k} w_j <= cutoff   (0-based tail)
  k_floor = #{j : sigma_j > 1e-13 sigma_0}                    (numerical rank)
  k       = min(k_cut, k_floor, chi_max)
  degeneracy guard: if the cut is not a rank-floor cut and sigma_k >=
  sigma_{k-1} (1 - 1e-10), k is lowered to the first index of that near-degenerate
  block; if the block starts at index 0, k is kept and the cut is flagged.
  eps = sum_{j >= k} w_j;  kept values are renormalised to unit 2-norm and the
  fidelity estimate is multiplied by (1 - eps).
"""
from __future__ import annotations

from typing import List, Tuple

import numpy as np

RANK_FLOOR = 1e-13
DEGENERACY = 1e-10


def svd(a: np.ndarray):
    """Thin SVD (LAPACK).  The divide-and-conquer driver occasionally fails to converge; the
    QR-iteration driver then computes the same decomposition."""
    try:
        return np.linalg.svd(a, full_matrices=False)
    except np.linalg.LinAlgError:
        import scipy.linalg
        return scipy.linalg.svd(a, full_matrices=False, lapack_driver="gesvd")


def rtrunc(sigma: np.ndarray, cutoff: float, chi_max: int,
           floor: float = RANK_FLOOR, degen: float = DEGENERACY) -> Tuple[int, float, bool]:
    """Apply R-TRUNC to singular values ``sigma`` (descending).  Returns (k, eps, flagged)."""
    sigma = np.asarray(sigma, dtype=np.float64)
    q = len(sigma)
    if q == 0 or sigma[0] <= 0.0:
        raise ArithmeticError("zero tensor cannot be truncated")
    w = sigma ** 2 / np.sum(sigma ** 2)
    tail = np.zeros(q + 1)
    for j in range(q - 1, -1, -1):          # tail[k] = sum_{j >= k} w_j
        tail[j] = tail[j + 1] + w[j]
    k_cut = q
    for k in range(1, q + 1):
        if tail[k] <= cutoff:
            k_cut = k
            break
    k_floor = int(np.sum(sigma > floor * sigma[0]))
    k = max(1, min(k_cut, k_floor, chi_max))
    flagged = False
    if k < q and sigma[k] > floor * sigma[0] and sigma[k] >= sigma[k - 1] * (1.0 - degen):
        j = k - 1
        while j > 0 and sigma[j] >= sigma[j - 1] * (1.0 - degen):
            j -= 1
        if j == 0:
            flagged = True
        else:
            k = j
    return k, float(tail[k]), flagged


def bond_renyi2(tensors: List[np.ndarray]) -> List[float]:
    """Renyi-2 entropy S2 = -ln(sum_k lambda_k^2) across every bond of the chain, with lambda_k the
    squared Schmidt coefficients of the cut normalised to sum 1 (Sec. 3: the entanglement
    measure the disentangler minimises, here evaluated on the committed state).  Works in any
    gauge: QR steps make every site left-orthonormal, then SVDs from the right read off each
    bond's Schmidt coefficients (the right part being right-orthonormal by then)."""
    ts = [np.array(t, dtype=np.complex128) for t in tensors]
    n = len(ts)
    for i in range(n - 1):
        cl, d, cr = ts[i].shape
        q, r = np.linalg.qr(ts[i].reshape(cl * d, cr))
        ts[i] = q.reshape(cl, d, q.shape[1])
        ts[i + 1] = np.einsum("ab,bsc->asc", r, ts[i + 1])
    out = [0.0] * (n - 1)
    for i in range(n - 1, 0, -1):
        cl, d, cr = ts[i].shape
        u, s, vh = np.linalg.svd(ts[i].reshape(cl, d * cr), full_matrices=False)
        lam = s ** 2 / np.sum(s ** 2)
        out[i - 1] = float(-np.log(np.sum(lam ** 2)))
        ts[i] = vh.reshape(len(s), d, cr)
        ts[i - 1] = np.einsum("asb,bc->asc", ts[i - 1], u * s[None, :])
    return out


class MPS:
    def __init__(self, d: int, tensors: List[np.ndarray], centre: int = 0):
        self.d = d
        self.tensors = tensors
        self.centre = centre

    @staticmethod
    def product_zero(d: int, n: int) -> "MPS":
        ts = []
        for _ in range(n):
            a = np.zeros((1, d, 1), dtype=np.complex128)
            a[0, 0, 0] = 1.0
            ts.append(a)
        return MPS(d, ts, 0)

    @property
    def n(self) -> int:
        return len(self.tensors)

    def copy(self) -> "MPS":
        return MPS(self.d, [t.copy() for t in self.tensors], self.centre)

    def bond_dims(self) -> List[int]:
        return [t.shape[2] for t in self.tensors[:-1]]

    def to_dense(self) -> np.ndarray:
        v = self.tensors[0].reshape(self.d, -1)
        for t in self.tensors[1:]:
            v = v @ t.reshape(t.shape[0], -1)
            v = v.reshape(-1, t.shape[2])
        return v.reshape(-1)

    def norm(self) -> float:
        return float(np.linalg.norm(self.tensors[self.centre]))

    # ----------------------------------------------------------- exact centre moves
    def _shift_right(self, i: int):
        a = self.tensors[i]
        cl, d, cr = a.shape
        q, r = np.linalg.qr(a.reshape(cl * d, cr))
        self.tensors[i] = q.reshape(cl, d, q.shape[1])
        nxt = self.tensors[i + 1]
        self.tensors[i + 1] = np.einsum("ab,bsc->asc", r, nxt)

    def _shift_left(self, i: int):
        a = self.tensors[i]
        cl, d, cr = a.shape
        # A = R^dagger Q^dagger from the QR of A^dagger
        q, r = np.linalg.qr(a.reshape(cl, d * cr).conj().T)
        self.tensors[i] = q.conj().T.reshape(q.shape[1], d, cr)
        prv = self.tensors[i - 1]
        self.tensors[i - 1] = np.einsum("asb,bc->asc", prv, r.conj().T)

    def move_centre(self, target: int):
        while self.centre < target:
            self._shift_right(self.centre)
            self.centre += 1
        while self.centre > target:
            self._shift_left(self.centre)
            self.centre -= 1

    # ----------------------------------------------------------- two-site tensor
    def theta(self, i: int) -> np.ndarray:
        """Two-site tensor of sites (i, i+1), shape (chi_l, d, d, chi_r)."""
        return np.einsum("asm,mtb->astb", self.tensors[i], self.tensors[i + 1])

    def split(self, i: int, theta: np.ndarray, cutoff: float, chi_max: int,
              move_right: bool, force_k: int | None = None) -> Tuple[float, bool, int]:
        """SVD-split theta back into sites (i, i+1) with R-TRUNC.

        Returns (eps, flagged, kept).  The centre ends on i+1 (move_right) or i.
        ``force_k`` replaces the rule's rank (frozen-decision replay); eps is then the
        discarded weight of that rank.
        """
        cl, d, _, cr = theta.shape
        u, s, vh = svd(theta.reshape(cl * d, d * cr))
        k, eps, flagged = rtrunc(s, cutoff, chi_max)
        if force_k is not None:
            k, flagged = int(force_k), False
            eps = float(np.sum(s[k:] ** 2) / np.sum(s ** 2))
        sk = s[:k] / np.linalg.norm(s[:k])
        u, vh = u[:, :k], vh[:k, :]
        if move_right:
            self.tensors[i] = u.reshape(cl, d, k)
            self.tensors[i + 1] = (sk[:, None] * vh).reshape(k, d, cr)
            self.centre = i + 1
        else:
            self.tensors[i] = (u * sk[None, :]).reshape(cl, d, k)
            self.tensors[i + 1] = vh.reshape(k, d, cr)
            self.centre = i
        return eps, flagged, k

    def truncate_sweep_left(self, l: int, r: int, cutoff: float, chi_max: int,
                            force_ks: List[int] | None = None
                            ) -> Tuple[List[float], List[bool]]:
        """Compression after an operator on [l, r]: QR left-to-right over [l, r-1], then
        SVD right-to-left for i = r..l+1 with R-TRUNC; the centre ends on l.
        ``force_ks`` (one rank per split, in order) replaces the rule's ranks."""
        self.move_centre(l)
        for i in range(l, r):
            self._shift_right(i)
        self.centre = r
        epss, flags = [], []
        self.last_ks = []
        for t, i in enumerate(range(r, l, -1)):
            a = self.tensors[i]
            cl, d, cr = a.shape
            u, s, vh = svd(a.reshape(cl, d * cr))
            k, eps, flagged = rtrunc(s, cutoff, chi_max)
            if force_ks is not None:
                k, flagged = int(force_ks[t]), False
                eps = float(np.sum(s[k:] ** 2) / np.sum(s ** 2))
            sk = s[:k] / np.linalg.norm(s[:k])
            self.tensors[i] = vh[:k].reshape(k, d, cr)
            self.tensors[i - 1] = np.einsum("asb,bc->asc", self.tensors[i - 1],
                                            u[:, :k] * sk[None, :])
            self.centre = i - 1
            epss.append(eps)
            flags.append(flagged)
            self.last_ks.append(k)
        return epss, flags

    # ----------------------------------------------------------- operators
    def apply_two_site(self, i: int, u: np.ndarray):
        """Contract a d^2 x d^2 operator into sites (i, i+1) without splitting (returns theta)."""
        th = self.theta(i)
        cl, d, _, cr = th.shape
        return np.einsum("xy,ayb->axb", u, th.reshape(cl, d * d, cr)).reshape(cl, d, d, cr)

    def apply_site_operator(self, i: int, o: np.ndarray):
        self.tensors[i] = np.einsum("st,atb->asb", o, self.tensors[i])

    def apply_block_mpo(self, l: int, r: int, ops: List[List[np.ndarray]], coeff: np.ndarray):
        """Apply sum_b coeff[b] (x)_{i=l..r} ops[b][i-l] as a bond-D MPO (D = len(coeff)).

        The MPO is block diagonal in b: site l carries the coefficient and opens the b
        index on its right bond, interior sites are block diagonal, site r closes it.
        Bond dimensions on [l, r-1] grow by the factor D (§2.4, operators acting on
        several sites).
        """
        D = len(coeff)
        if l == r:
            o = sum(coeff[b] * ops[b][0] for b in range(D))
            self.apply_site_operator(l, o)
            return
        for i in range(l, r + 1):
            a = self.tensors[i]
            cl, d, cr = a.shape
            blocks = [np.einsum("st,atb->asb", ops[b][i - l], a) for b in range(D)]
            if i == l:
                out = np.zeros((cl, d, D * cr), dtype=np.complex128)
                for b in range(D):
                    out[:, :, b * cr:(b + 1) * cr] = coeff[b] * blocks[b]
            elif i == r:
                out = np.zeros((D * cl, d, cr), dtype=np.complex128)
                for b in range(D):
                    out[b * cl:(b + 1) * cl, :, :] = blocks[b]
            else:
                out = np.zeros((D * cl, d, D * cr), dtype=np.complex128)
                for b in range(D):
                    out[b * cl:(b + 1) * cl, :, b * cr:(b + 1) * cr] = blocks[b]
            self.tensors[i] = out

    def expectation_product(self, ops: List[np.ndarray]) -> complex:
        """<MPS| (x)_i ops[i] |MPS> by left-to-right transfer matrices
        E' = sum_{a b s t} E[a, b] conj(A[a, s, c]) O[s, t] A[b, t, d], contracted one operand at a
        time (chi^3 d work per site)."""
        e = np.ones((1, 1), dtype=np.complex128)
        for a, o in zip(self.tensors, ops):
            x = np.einsum("ab,btd->atd", e, a)          # E A
            x = np.einsum("st,atd->asd", o, x)          # O on the physical index
            e = np.einsum("asc,asd->cd", a.conj(), x)   # conj(A) closes a and s
        return complex(e[0, 0])
