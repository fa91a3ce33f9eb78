"""Dense state-vector simulator (§2.1): psi = U_circuit |0...0>, d^n amplitudes.

Brute-force reference for small n: every Clifford word is applied as its dense
d^2 x d^2 matrix and every phase gate as a diagonal d x d matrix.  Site 0 is the
most significant digit of the amplitude index.
"""
from __future__ import annotations

import numpy as np

from .clifford import word_matrix


def apply_one_site(v: np.ndarray, d: int, n: int, site: int, u: np.ndarray) -> np.ndarray:
    t = v.reshape(d ** site, d, d ** (n - site - 1))
    return np.einsum("xy,ayb->axb", u, t).reshape(-1)


def apply_two_site(v: np.ndarray, d: int, n: int, site: int, u: np.ndarray) -> np.ndarray:
    t = v.reshape(d ** site, d * d, d ** (n - site - 2))
    return np.einsum("xy,ayb->axb", u, t).reshape(-1)


def simulate(circuit, phases_override=None) -> np.ndarray:
    """Dense final state of a workload circuit.  ``phases_override`` maps a
    parametrised gate index to its angles (used for gradient checks)."""
    d, n = circuit.d, circuit.n
    v = np.zeros(d ** n, dtype=np.complex128)
    v[0] = 1.0
    for layer in circuit.layers:
        for b in layer.bricks:
            v = apply_two_site(v, d, n, b.site, word_matrix(d, b.word.gens, b.word.weyl))
        for ph in layer.phases:
            phi = ph.phi
            if phases_override is not None and ph.param >= 0:
                phi = phases_override[ph.param]
            v = apply_one_site(v, d, n, ph.site, np.diag(np.exp(1j * np.asarray(phi))))
    return v


def align_global_phase(v: np.ndarray, ref: np.ndarray) -> np.ndarray:
    """Multiply v by the unit phase that maximises Re <ref|v> (fix the C phase)."""
    ov = np.vdot(v, ref)
    if abs(ov) == 0:
        return v
    return v * (ov / abs(ov))
