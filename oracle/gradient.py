"""Gradient of the observable loss with respect to phase-gate angles (oracle).

Test infrastructure only: the library never imports this module.

Loss (the observables of §3 on a parametrised circuit): L(theta) = Re sum_j <psi|Z_j|psi>,
equal to sum_j <(Z_j + Z_j^dagger)/2>.  Parametrised gates are diag(e^{i phi_0}, ...,
e^{i phi_{d-1}}) with phi = (0, theta[(d-1)g], ..., theta[(d-1)g + d-2]) for gate g
(``PhaseGate.param``): diagonal phase gates as in §2.3.2 with free angles.

The derivative is taken with the method's discrete decisions frozen (disentangler choices
and kept ranks of every truncating split, recorded at theta0): the GCAMPS forward pass is
then a smooth function of theta and its derivative is well defined.  Three definitions:

* ``dense_gradient``: the exact derivative of the dense circuit state (§2.1), obtained by
  differentiating one phase gate at a time, d/dphi_j diag(e^{i phi}) = i |j><j| diag(e^{i phi}).
  Equals the GCAMPS derivative whenever nothing is truncated.
* ``fd_gradient``: central differences of the frozen GCAMPS replay (error O(h^2) plus
  rounding / h), optionally Richardson-extrapolated (O(h^4)).
* ``replay_loss``: the frozen GCAMPS forward pass itself.
"""
from __future__ import annotations

from typing import List, Sequence, Tuple

import numpy as np

from .clifford import word_matrix
from .gcamps import Config, run_circuit
from .statevector import apply_one_site, apply_two_site


def angles(theta: Sequence[float], d: int, ngates: int) -> List[Tuple[float, ...]]:
    th = np.asarray(theta, dtype=np.float64)
    return [(0.0,) + tuple(th[(d - 1) * g:(d - 1) * (g + 1)]) for g in range(ngates)]


def n_param_gates(circuit) -> int:
    """Number of parameter blocks: one past the largest parameter index in the circuit."""
    return 1 + max((ph.param for L in circuit.layers for ph in L.phases), default=-1)


# ------------------------------------------------------------------ dense definition
def _dense_state(circuit, phis, deriv=None) -> np.ndarray:
    """Dense state; with deriv = (g, j) the phase gate of parameter g is replaced by its
    derivative with respect to phi_j."""
    d, n = circuit.d, circuit.n
    v = np.zeros(d ** n, dtype=np.complex128)
    v[0] = 1.0
    for layer in circuit.layers:
        for b in layer.bricks:
            v = apply_two_site(v, d, n, b.site, word_matrix(d, b.word.gens, b.word.weyl))
        for ph in layer.phases:
            phi = phis[ph.param] if ph.param >= 0 else ph.phi
            diag = np.exp(1j * np.asarray(phi, dtype=np.float64))
            if deriv is not None and ph.param == deriv[0]:
                dd = np.zeros(d, dtype=np.complex128)
                dd[deriv[1]] = 1j * diag[deriv[1]]
                diag = dd
            v = apply_one_site(v, d, n, ph.site, np.diag(diag))
    return v


def _z_sum_hermitian(v: np.ndarray, d: int, n: int) -> np.ndarray:
    """H v with H = sum_j (Z_j + Z_j^dagger)/2, Z = diag(omega^k)."""
    omega = np.exp(2j * np.pi / d)
    zr = np.real(omega ** np.arange(d))          # (Z + Z^dagger)/2 is diag(cos(2 pi k/d))
    out = np.zeros_like(v)
    for j in range(n):
        out += apply_one_site(v, d, n, j, np.diag(zr.astype(np.complex128)))
    return out


def dense_loss(circuit, theta) -> float:
    phis = angles(theta, circuit.d, n_param_gates(circuit))
    v = _dense_state(circuit, phis)
    return float(np.real(np.vdot(v, _z_sum_hermitian(v, circuit.d, circuit.n))))


def dense_gradient(circuit, theta) -> np.ndarray:
    """dL/dtheta = 2 Re <d psi|H|psi> for each parameter (exact, one gate at a time)."""
    d, n = circuit.d, circuit.n
    ng = n_param_gates(circuit)
    phis = angles(theta, d, ng)
    v = _dense_state(circuit, phis)
    hv = _z_sum_hermitian(v, d, n)
    g = np.zeros((d - 1) * ng)
    for gi in range(ng):
        for j in range(1, d):
            dv = _dense_state(circuit, phis, deriv=(gi, j))
            g[(d - 1) * gi + j - 1] = 2.0 * np.real(np.vdot(dv, hv))
    return g


# ------------------------------------------------------------------ GCAMPS definition
def record(circuit, candidates, cfg: Config, theta):
    """Forward pass at theta; returns (state, frozen decisions)."""
    phis = angles(theta, circuit.d, n_param_gates(circuit))
    st = run_circuit(circuit, candidates, cfg, phases_override=phis)
    frozen = ([e.choice for e in st.choice_log], list(st.rank_log))
    return st, frozen


def replay_loss(circuit, candidates, cfg: Config, theta, frozen) -> float:
    phis = angles(theta, circuit.d, n_param_gates(circuit))
    st = run_circuit(circuit, candidates, cfg, phases_override=phis, frozen=frozen)
    return st.loss_sum_z()


def fd_gradient(circuit, candidates, cfg: Config, theta, frozen, h: float = 1e-6,
                params: Sequence[int] | None = None, richardson: bool = False) -> np.ndarray:
    """Central differences D(h) = (L(theta + h e_k) - L(theta - h e_k)) / 2h of the frozen
    replay (error O(h^2)); with ``richardson`` the extrapolation (4 D(h) - D(2h)) / 3, whose
    error is O(h^4)."""
    theta = np.asarray(theta, dtype=np.float64)
    idx = range(len(theta)) if params is None else params
    g = np.full(len(theta), np.nan)

    def central(k, step):
        tp, tm = theta.copy(), theta.copy()
        tp[k] += step
        tm[k] -= step
        return (replay_loss(circuit, candidates, cfg, tp, frozen)
                - replay_loss(circuit, candidates, cfg, tm, frozen)) / (2.0 * step)

    for k in idx:
        g[k] = central(k, h)
        if richardson:
            g[k] = (4.0 * g[k] - central(k, 2.0 * h)) / 3.0
    return g
