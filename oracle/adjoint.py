"""Reverse-mode derivative of the frozen GCAMPS forward pass (oracle).

Test infrastructure only: the library never imports this module.

The loss is L(theta) = Re sum_j <psi|Z_j|psi> (the observables of §3) with every discrete
decision frozen at theta0: the disentangler choices and the kept rank of every truncating
split (as in oracle/gradient.py).  With the decisions fixed, the bottom loop of §3 is a
composition of three kinds of steps acting on the MPS state |MPS> (psi = C|MPS>, and the
Clifford frame C depends on the decisions only, not on theta):

* the commuted gate sum_b c_b(phi) P^b (§3, step (b) of oracle/gcamps.py): a linear map whose
  coefficients c_b depend on the gate's angles phi;
* a disentangler commit Q on sites (i, i+1) (§3): a fixed unitary;
* a truncating split across a cut (§2.4): with the MPS in canonical form around the cut, the
  split's SVD is the Schmidt decomposition of the whole state across that cut, so keeping k
  values and renormalising maps the state to P v / |P v|, P the projector onto its top-k left
  Schmidt vectors.  Exact centre moves leave the state unchanged.

This module replays that composition on the dense vector of |MPS> (small n only), keeps
every intermediate vector, and runs the chain rule backwards.  Conventions: for a real loss,
g_v = dL/d(conj v) (so dL = 2 Re <g_v, dv>).

* linear step v' = O v:          g_v = O^dagger g_v',  dL/dphi_j = 2 Re <g_v', (dO/dphi_j) v>;
* renormalisation v' = y / |y|:  g_y = (g_v' - Re<g_v', y> y / |y|^2) / |y|;
* projection y = P(M) M, M the state reshaped across the cut (left block x right block),
  A = M M^dagger = U diag(lam) U^dagger (full basis, lam padded with zeros), K the kept
  indices:  dP = U (G o U^dagger dA U) U^dagger with G_ab = 1 / (lam_a - lam_b) when exactly
  one of a, b is kept (the first-order change of the kept eigenvectors; pairs inside K
  cancel), so g_M = P Gy + (D + D^dagger) M with Gy = g_y as a matrix,
  D = U (G o U^dagger (Gy M^dagger) U) U^dagger.
  The kept ranks are those of the recorded run, where the degeneracy guard keeps the cut off
  every near-degenerate group, so every such lam_a - lam_b is nonzero.

Pins (tests/test_oracle_adjoint.py): without truncation the result equals the dense
derivative of the circuit (oracle/gradient.py ``dense_gradient``); with truncation it equals
Richardson-extrapolated central differences of the oracle's own frozen replay.
"""
from __future__ import annotations

from typing import List, Sequence

import numpy as np

from .gcamps import Config, run_circuit
from .gradient import angles, n_param_gates
from .statevector import apply_one_site, apply_two_site
from .weyl import omega, site_matrix, tau


def _apply_string(v: np.ndarray, d: int, n: int, l: int, ops: Sequence[np.ndarray], adjoint: bool = False):
    for t, o in enumerate(ops):
        v = apply_one_site(v, d, n, l + t, o.conj().T if adjoint else o)
    return v


def _coefficients(d: int, phi: Sequence[float]):
    """c(phi) = V^-1 e^{i phi} with V_jb = omega^{bj} (diag(e^{i phi}) = sum_b c_b Z^b), and
    dc/dphi_j = V^-1 (i e^{i phi_j} e_j) as the columns of a d x d matrix."""
    V = np.array([[omega(d) ** (b * j) for b in range(d)] for j in range(d)])
    Vinv = np.linalg.inv(V)
    e = np.exp(1j * np.asarray(phi, dtype=np.float64))
    return Vinv @ e, Vinv * (1j * e)[None, :]


def _loss_vector(st, v: np.ndarray) -> np.ndarray:
    """H v with H = sum_j (W_j + W_j^dagger)/2, W_j = C^dagger Z_j C as a Weyl string of the
    final tableau (§3 observables)."""
    from .weyl import Weyl
    d, n = st.d, st.n
    out = np.zeros_like(v)
    for j in range(n):
        z = np.zeros(n, np.int64)
        z[j] = 1
        P, _, _ = st.tab.decompose(Weyl(d, np.zeros(n, np.int64), z, 0))
        ops = [site_matrix(d, int(P.x[i]), int(P.z[i])) for i in range(n)]
        ph = tau(d) ** P.p
        wv = ph * _apply_string(v, d, n, 0, ops)
        wdv = np.conj(ph) * _apply_string(v, d, n, 0, ops, adjoint=True)
        out += 0.5 * (wv + wdv)
    return out


def _cut_matrix(v: np.ndarray, d: int, n: int, c: int):
    """The state across the cut after site c - 1 as a matrix with no more rows than
    columns: (left block x right block), transposed when the left block is larger (the
    projector onto the top-k left Schmidt vectors of M equals, transposed, the one onto the
    top-k left singular vectors of M^T, so either side gives the same step)."""
    M = v.reshape(d ** c, d ** (n - c))
    return (M.T, True) if M.shape[0] > M.shape[1] else (M, False)


def _cut_basis(M: np.ndarray):
    U, s, _ = np.linalg.svd(M, full_matrices=True)
    lam = np.zeros(M.shape[0])
    lam[:len(s)] = s ** 2
    return U, lam


def frozen_adjoint(circuit, candidates, cfg: Config, theta, frozen):
    """(loss, dL/dtheta) of the frozen GCAMPS forward pass at theta, reverse mode on the
    dense vector of the MPS.  ``frozen`` = (choices, ranks) from oracle.gradient.record."""
    d, n = circuit.d, circuit.n
    if any(L.gates for L in circuit.layers):
        raise ValueError("general gates are not differentiated")
    ng = n_param_gates(circuit)
    phis = angles(theta, d, ng)
    st = run_circuit(circuit, candidates, cfg, phases_override=phis, frozen=frozen)
    params = [ph.param for L in circuit.layers for ph in L.phases]
    # forward replay of the logged steps on the dense vector
    v = np.zeros(d ** n, dtype=np.complex128)
    v[0] = 1.0
    tape: List[tuple] = []
    gate = 0
    for step in st.steps:
        kind = step[0]
        if kind == "mpo":
            _, l, r, ops, phi, phase = step
            c, dc = _coefficients(d, phi)
            terms = [_apply_string(v, d, n, l, ops[b]) for b in range(d)]
            tape.append(("mpo", l, ops, c * phase, dc * phase[:, None], terms, params[gate]))
            v = sum(c[b] * phase[b] * terms[b] for b in range(d))
            gate += 1
        elif kind == "q":
            _, i, Q = step
            tape.append(("q", i, Q))
            v = apply_two_site(v, d, n, i, Q)
        else:
            _, cut, k = step
            M, tr = _cut_matrix(v, d, n, cut)
            U, lam = _cut_basis(M)
            Uk = U[:, :k]
            y = Uk @ (Uk.conj().T @ M)
            ny = np.linalg.norm(y)
            tape.append(("cut", tr, k, M, U, lam, y, ny))
            v = ((y.T if tr else y) / ny).reshape(-1)
    hv = _loss_vector(st, v)
    loss = float(np.real(np.vdot(v, hv)))
    # reverse sweep
    grad = np.zeros(len(theta))
    g = hv                                   # dL/d(conj v) of L = <v|H|v>
    for rec in reversed(tape):
        kind = rec[0]
        if kind == "mpo":
            _, l, ops, coeff, dcoeff, terms, p = rec
            if p >= 0:
                for j in range(1, d):
                    dv = sum(dcoeff[b, j] * terms[b] for b in range(d))
                    grad[(d - 1) * p + j - 1] += 2.0 * np.real(np.vdot(g, dv))
            g = sum(np.conj(coeff[b]) * _apply_string(g, d, n, l, ops[b], adjoint=True) for b in range(d))
        elif kind == "q":
            _, i, Q = rec
            g = apply_two_site(g, d, n, i, Q.conj().T)
        else:
            _, tr, k, M, U, lam, y, ny = rec
            gv = g.reshape(M.shape[::-1]).T if tr else g.reshape(M.shape)
            gy = (gv - np.real(np.vdot(gv, y)) * y / ny ** 2) / ny
            a = M.shape[0]
            kept = np.zeros(a, dtype=bool)
            kept[:k] = True
            G = np.zeros((a, a))
            diff = lam[:, None] - lam[None, :]
            mask = kept[:, None] ^ kept[None, :]
            G[mask] = 1.0 / np.abs(diff[mask])
            Uk = U[:, :k]
            CU = U.conj().T @ (gy @ M.conj().T) @ U
            D = U @ (G * CU) @ U.conj().T
            gM = Uk @ (Uk.conj().T @ gy) + (D + D.conj().T) @ M
            g = (gM.T if tr else gM).reshape(-1)
    return loss, grad, st, v
