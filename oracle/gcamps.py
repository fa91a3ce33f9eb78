"""GCAMPS state psi = C|MPS> (§3, Fig. 1), plain FP64 reference.

Top loop: a Clifford word updates only the tableau of C.

Bottom loop for a diagonal phase gate U = diag(e^{i phi_j}) on site k:
  (a) decompose U = sum_b c_b Z_k^b by solving the d x d linear system
      sum_b c_b omega^{bj} = e^{i phi_j} (§3: the decomposition is found by a
      linear solve; for a diagonal gate this is a DFT),
  (b) commute through C: C^dagger U C = sum_b c_b P^b with P = C^dagger Z_k C from
      the tableau decomposition (§2.3.1),
  (c) apply sum_b c_b P^b to the MPS as a bond-d MPO on the support [l, r] of P and
      compress (centre -> l, QR l..r-1, SVD r..l+1 with R-TRUNC, renormalise),
  (d) disentangle (§3): sweeps over all n-1 bonds, alternating left-to-right and
      right-to-left.  At each bond the two-site tensor Theta is rotated by every
      candidate Q_c, scored by the Renyi-2 entropy of the cut between the two
      sites, S2_c = -ln(sum |rho_c|^2 / (tr rho_c)^2), rho_c = M_c M_c^dagger with
      M_c the (chi_l d) x (d chi_r) matrix of Q_c Theta; the selected c* is the
      lowest index with S2_c <= min_c S2_c + tie_tol.  If c* != 0, Theta <- Q Theta
      and C <- C Q^dagger.  Theta is then SVD-split with R-TRUNC.  Sweeping stops
      after a sweep that keeps the identity everywhere or after max_sweeps.
      (The paper gives the idea of reducing entanglement with two-qudit Cliffords
      and an exhaustive search; the entropy measure, tie rule and sweep schedule are
      this package's readings of it.  Parity of the truncated regime is "parity
      unpinned": it is fixed only by these rules.)

Observables (§3): <psi|W|psi> = <MPS|C^dagger W C|MPS> by transfer matrices;
Re<W> is the expectation of the Hermitian O = (W + W^dagger)/2.

Dense amplitudes: the oracle records every Clifford it applies to C, so it can
rebuild C as a dense product and return psi with its true global phase.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Sequence, Tuple

import numpy as np

from .clifford import word_matrix
from .mps import MPS, rtrunc
from .mps import svd as mps_svd
from .tableau import Tableau
from .weyl import Weyl, omega, site_matrix, tau


def diagonal_coefficients(d: int, phi: Sequence[float]) -> np.ndarray:
    """c_b with diag(e^{i phi}) = sum_b c_b Z^b, by a linear solve (step (a))."""
    V = np.array([[omega(d) ** (b * j) for b in range(d)] for j in range(d)])
    return np.linalg.solve(V, np.exp(1j * np.asarray(phi, dtype=np.float64)))


def weyl_expansion(d: int, k: int, u: np.ndarray, drop: float = 1e-14):
    """U = sum_{x,z} c_xz W_xz on k sites, W_xz = (x)_t X^{x_t} Z^{z_t} (§2.3: the d^{2k} Weyl
    operators are orthogonal, Tr(W^dagger W') = d^k delta), so c_xz = Tr(W_xz^dagger U) / d^k.
    Returns [(x, z, c)] for |c| > drop * max|c|, x and z tuples over the k sites."""
    from itertools import product
    terms = []
    for x in product(range(d), repeat=k):
        for z in product(range(d), repeat=k):
            w = np.ones((1, 1))
            for t in range(k):
                w = np.kron(w, site_matrix(d, x[t], z[t]))
            terms.append((x, z, np.trace(w.conj().T @ u) / d ** k))
    cmax = max(abs(c) for _, _, c in terms)
    return [t for t in terms if abs(t[2]) > drop * cmax]


def renyi2(theta: np.ndarray) -> float:
    """S2 across the middle cut of a two-site tensor (chi_l, d, d, chi_r), direct definition."""
    cl, d, _, cr = theta.shape
    m = theta.reshape(cl * d, d * cr)
    rho = m @ m.conj().T if m.shape[0] <= m.shape[1] else m.conj().T @ m
    tr = np.real(np.trace(rho))
    return float(-np.log(np.sum(np.abs(rho) ** 2) / tr ** 2))


def renyi2_replica(theta: np.ndarray, q: np.ndarray) -> float:
    """Same score via the replica identity (independent formula, tests only):
    purity * |Theta|^4 = sum_{xyzw} W_xyzw V_xyzw(Q) with
    F_(a x),(a' y) = sum_b Theta_axb conj(Theta_a'yb),  W_xyzw = sum_{a a'} F_(ax),(a'y) F_(a'z),(aw),
    V_xyzw = sum Q_(s1 s2),x conj(Q_(s1' s2),y) Q_(s1' t2),z conj(Q_(s1 t2),w)."""
    cl, d, _, cr = theta.shape
    t = theta.reshape(cl, d * d, cr)
    F = np.einsum("axb,cyb->axcy", t, t.conj())
    W = np.einsum("axcy,czaw->xyzw", F, F)
    qq = q.reshape(d, d, d * d)
    V = np.einsum("pqx,rqy,rtz,ptw->xyzw", qq, qq.conj(), qq, qq.conj())
    nrm2 = np.real(np.sum(np.abs(theta) ** 2))
    purity = np.real(np.sum(W * V)) / nrm2 ** 2
    return float(-np.log(purity))


@dataclass
class Config:
    chi_max: int
    cutoff: float
    tie_tol: float = 1e-10
    max_sweeps: int = 2
    auto_disentangle: bool = True
    criterion: str = "renyi2"   # or "bond_dim": the bond-dimension criterion (§4)


@dataclass
class ChoiceEntry:
    gate: int
    sweep: int
    bond: int
    choice: int


class Gcamps:
    def __init__(self, d: int, n: int, cfg: Config, candidates: Sequence = (), frozen=None):
        """``frozen`` = (choices, ranks) replays a recorded run: the disentangler takes the
        recorded choices in order (no scoring) and every truncating split keeps the
        recorded rank.  The rank log lists the kept rank of every truncating split
        (compression splits, then disentangler splits, in execution order)."""
        self.d, self.n, self.cfg = d, n, cfg
        self.rank_log: List[int] = []
        self._frozen_choices = list(frozen[0]) if frozen is not None else None
        self._frozen_ranks = list(frozen[1]) if frozen is not None else None
        self.tab = Tableau(d, n)
        self.mps = MPS.product_zero(d, n)
        self.f_est = 1.0
        self.eps_log: List[float] = []      # discarded weight of every truncation, in order
        self.choice_log: List[ChoiceEntry] = []
        self.gate_count = 0
        self.flags = 0                      # number of degenerate cuts (parity unpinned)
        self.record: List[Tuple[str, int, tuple, tuple]] = []
        self.candidates = list(candidates)
        self._cand_mats = [word_matrix(d, w.gens, w.weyl) for w in self.candidates]
        self.last_support: Tuple[int, int] = (-1, -1)
        # Bookkeeping for the reverse-mode derivative (oracle/adjoint.py), no arithmetic:
        # every step that changes the state of the MPS, in execution order --
        #   ("mpo", l, r, ops, phi, phase)  sum_b c_b(phi) phase[b] (x)_{i=l..r} ops[b][i-l]
        #   ("cut", c, k)                   truncating split across the cut after site c-1,
        #                                   k values kept, renormalised
        #   ("q", i, Q)                     disentangler unitary on sites (i, i+1)
        # Exact centre moves leave the state unchanged and are not listed.
        self.steps: List[tuple] = []

    # ------------------------------------------------------------------ top loop
    def apply_clifford(self, site: int, gens: Sequence[int], weyl: Sequence[int]):
        self.tab.apply_word(site, gens, weyl)
        self.record.append(("G", site, tuple(gens), tuple(weyl)))

    # ------------------------------------------------------------------ bottom loop
    def apply_phase_rotation(self, site: int, phi: Sequence[float]):
        d, n = self.d, self.n
        c = diagonal_coefficients(d, phi)
        zk = Weyl(d, np.zeros(n, np.int64), np.eye(n, dtype=np.int64)[site], 0)
        P, _, _ = self.tab.decompose(zk)
        sup = [i for i in range(n) if P.x[i] or P.z[i]]
        l, r = sup[0], sup[-1]
        self.last_support = (l, r)
        powers = [P.power(b) for b in range(d)]
        coeff = np.array([c[b] * tau(d) ** powers[b].p for b in range(d)])
        ops = [[site_matrix(d, int(powers[b].x[i]), int(powers[b].z[i])) for i in range(l, r + 1)]
               for b in range(d)]
        self.steps.append(("mpo", l, r, ops, tuple(float(v) for v in phi),
                           np.array([tau(d) ** powers[b].p for b in range(d)])))
        self.mps.move_centre(l)
        self.mps.apply_block_mpo(l, r, ops, coeff)
        if r > l:
            force = None
            if self._frozen_ranks is not None:
                force = [self._frozen_ranks.pop(0) for _ in range(r - l)]
            epss, flags = self.mps.truncate_sweep_left(l, r, self.cfg.cutoff, self.cfg.chi_max,
                                                       force_ks=force)
            self.rank_log.extend(self.mps.last_ks)
            self.steps.extend(("cut", i, k) for i, k in zip(range(r, l, -1), self.mps.last_ks))
            for e in epss:
                self.f_est *= (1.0 - e)
                self.eps_log.append(float(e))
            self.flags += sum(flags)
        self.gate_count += 1
        if self.cfg.auto_disentangle and self.candidates:
            self.disentangle()

    def apply_gate(self, site: int, u: np.ndarray):
        """A general gate U on sites site..site+k-1 (the bottom loop for a non-diagonal or
        two-site unitary): every Weyl term of U is commuted through C by elimination (§2.3.1),
        the sum is applied as a block MPO with one block per term, then compressed (§2.4) and
        disentangled (§3)."""
        d, n = self.d, self.n
        k = 1 if u.shape[0] == d else 2
        terms = weyl_expansion(d, k, u)
        Ps, coeff = [], []
        for x, z, c in terms:
            xs = np.zeros(n, np.int64)
            zs = np.zeros(n, np.int64)
            xs[site:site + k] = x
            zs[site:site + k] = z
            P, _, _ = self.tab.decompose(Weyl(d, xs, zs, 0))
            Ps.append(P)
            coeff.append(c * tau(d) ** P.p)
        sup = [i for i in range(n) if any(P.x[i] or P.z[i] for P in Ps)]
        l, r = (sup[0], sup[-1]) if sup else (site, site)
        self.last_support = (l, r)
        ops = [[site_matrix(d, int(P.x[i]), int(P.z[i])) for i in range(l, r + 1)] for P in Ps]
        self.mps.move_centre(l)
        self.mps.apply_block_mpo(l, r, ops, np.array(coeff))
        if r > l:
            epss, flags = self.mps.truncate_sweep_left(l, r, self.cfg.cutoff, self.cfg.chi_max)
            self.rank_log.extend(self.mps.last_ks)
            for e in epss:
                self.f_est *= (1.0 - e)
                self.eps_log.append(float(e))
            self.flags += sum(flags)
        self.gate_count += 1
        if self.cfg.auto_disentangle and self.candidates:
            self.disentangle()

    def scores(self, theta: np.ndarray) -> np.ndarray:
        cl, d, _, cr = theta.shape
        out = np.empty(len(self._cand_mats))
        for c, q in enumerate(self._cand_mats):
            th = np.einsum("xy,ayb->axb", q, theta.reshape(cl, d * d, cr)).reshape(cl, d, d, cr)
            out[c] = renyi2(th)
        return out

    def select(self, s2: np.ndarray) -> int:
        lim = np.min(s2) + self.cfg.tie_tol
        return int(np.nonzero(s2 <= lim)[0][0])

    def ranks(self, theta: np.ndarray) -> np.ndarray:
        """Bond dimension each candidate leaves: the split's truncation rule applied to the
        singular values of the rotated two-site tensor."""
        cl, d, _, cr = theta.shape
        out = np.empty(len(self._cand_mats), dtype=np.int64)
        for c, q in enumerate(self._cand_mats):
            m = np.einsum("xy,ayb->axb", q, theta.reshape(cl, d * d, cr)).reshape(cl * d, d * cr)
            _, s, _ = mps_svd(m)
            out[c] = rtrunc(s, self.cfg.cutoff, self.cfg.chi_max)[0]
        return out

    def select_bond_dim(self, theta: np.ndarray) -> int:
        """Bond-dimension criterion: keep the identity unless a candidate leaves a smaller bond
        dimension; among the candidates of the smallest one, the rule of `select` on their S2."""
        r = self.ranks(theta)
        if r.min() >= r[0]:
            return 0
        s2 = self.scores(theta)
        best = np.nonzero(r == r.min())[0]
        lim = np.min(s2[best]) + self.cfg.tie_tol
        return int(best[np.nonzero(s2[best] <= lim)[0][0]])

    def disentangle(self) -> Tuple[int, int]:
        """Sweeps of the disentangler; returns (sweeps run, bonds changed)."""
        n = self.n
        sweeps, changed_total = 0, 0
        for sweep in range(self.cfg.max_sweeps):
            sweeps += 1
            changed = 0
            left_to_right = (sweep % 2 == 0)
            bonds = range(n - 1) if left_to_right else range(n - 2, -1, -1)
            for i in bonds:
                self.mps.move_centre(i if left_to_right else i + 1)
                th = self.mps.theta(i)
                if self._frozen_choices is not None:
                    c = self._frozen_choices.pop(0)
                elif self.cfg.criterion == "bond_dim":
                    c = self.select_bond_dim(th)
                else:
                    c = self.select(self.scores(th))
                self.choice_log.append(ChoiceEntry(self.gate_count - 1, sweep, i, c))
                if c != 0:
                    w = self.candidates[c]
                    cl, d, _, cr = th.shape
                    th = np.einsum("xy,ayb->axb", self._cand_mats[c],
                                   th.reshape(cl, d * d, cr)).reshape(cl, d, d, cr)
                    self.tab.right_multiply_dagger(i, w.gens, w.weyl)
                    self.record.append(("Q", i, tuple(w.gens), tuple(w.weyl)))
                    self.steps.append(("q", i, self._cand_mats[c]))
                    changed += 1
                force = self._frozen_ranks.pop(0) if self._frozen_ranks is not None else None
                eps, flagged, kept = self.mps.split(i, th, self.cfg.cutoff, self.cfg.chi_max,
                                                    move_right=left_to_right, force_k=force)
                self.rank_log.append(kept)
                self.steps.append(("cut", i + 1, kept))
                self.f_est *= (1.0 - eps)
                self.eps_log.append(float(eps))
                self.flags += int(flagged)
            changed_total += changed
            if changed == 0:
                break
        return sweeps, changed_total

    # ------------------------------------------------------------------ observables
    def expectation(self, x: Sequence[int], z: Sequence[int], p: int = 0) -> complex:
        d = self.d
        W = Weyl(d, np.asarray(x), np.asarray(z), p)
        P, _, _ = self.tab.decompose(W)
        ops = [site_matrix(d, int(P.x[i]), int(P.z[i])) for i in range(self.n)]
        return complex(tau(d) ** P.p * self.mps.expectation_product(ops))

    def loss_sum_z(self) -> float:
        """Re sum_j <Z_j>, i.e. sum_j <(Z_j + Z_j^dagger)/2> (§3 observables)."""
        tot = 0.0
        for j in range(self.n):
            z = np.zeros(self.n, np.int64)
            z[j] = 1
            tot += self.expectation(np.zeros(self.n, np.int64), z, 0).real
        return tot

    def statevector(self) -> np.ndarray:
        """Dense psi = C|MPS> with C rebuilt from the recorded Cliffords (true phase)."""
        d, n = self.d, self.n
        v = self.mps.to_dense()
        gates = [r for r in self.record if r[0] == "G"]
        dis = [r for r in self.record if r[0] == "Q"]
        # C = (G_last ... G_first)(Q_first^dagger ... Q_last^dagger)
        for _, site, gens, weyl in reversed(dis):
            v = apply_dense_two_site(v, d, n, site, word_matrix(d, gens, weyl).conj().T)
        for _, site, gens, weyl in gates:
            v = apply_dense_two_site(v, d, n, site, word_matrix(d, gens, weyl))
        return v

    def dense_clifford(self) -> np.ndarray:
        """Dense matrix of C (very small n only)."""
        d, n = self.d, self.n
        D = d ** n
        cols = [self._apply_C(np.eye(D, dtype=np.complex128)[:, j]) for j in range(D)]
        return np.stack(cols, axis=1)

    def _apply_C(self, v):
        d, n = self.d, self.n
        for _, site, gens, weyl in reversed([r for r in self.record if r[0] == "Q"]):
            v = apply_dense_two_site(v, d, n, site, word_matrix(d, gens, weyl).conj().T)
        for _, site, gens, weyl in [r for r in self.record if r[0] == "G"]:
            v = apply_dense_two_site(v, d, n, site, word_matrix(d, gens, weyl))
        return v


def apply_dense_two_site(v: np.ndarray, d: int, n: int, site: int, u: np.ndarray) -> np.ndarray:
    t = v.reshape(d ** site, d * d, d ** (n - site - 2))
    return np.einsum("xy,ayb->axb", u, t).reshape(-1)


def run_circuit(circuit, candidates, cfg: Config, record_states: bool = False,
                phases_override=None, frozen=None) -> Gcamps:
    """Run a workload circuit (bricks, then phase gates, then general gates, layer by layer).
    ``phases_override[param]`` replaces the angles of parametrised gates."""
    g = Gcamps(circuit.d, circuit.n, cfg, candidates, frozen=frozen)
    for layer in circuit.layers:
        for b in layer.bricks:
            g.apply_clifford(b.site, b.word.gens, b.word.weyl)
        for ph in layer.phases:
            phi = ph.phi
            if phases_override is not None and ph.param >= 0:
                phi = phases_override[ph.param]
            g.apply_phase_rotation(ph.site, phi)
        for gg in layer.gates:
            D = circuit.d ** gg.k
            g.apply_gate(gg.site, np.array(gg.u, dtype=complex).reshape(D, D))
    return g
