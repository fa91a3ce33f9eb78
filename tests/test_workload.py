"""The seeded workload generator: Haar-random unitaries and general-gate circuits.

Pins of ``haar_unitary`` against what the Haar measure fixes: unitarity; E|u_ij|^2 = 1/D and
E|u_ij|^4 = 2/(D(D+1)) (the second moment separates Haar from, e.g., random permutations with
random phases, whose E|u|^4 is 1/D); E u_ij = 0; the same draw on every call with one seed.
"""
import math

import numpy as np
import pytest

from paper_2511_06672_amd.workload import (SplitMix64, general_circuit, haar_unitary, substream,
                                           workload)


@pytest.mark.parametrize("D", [2, 3, 4, 9])
def test_haar_unitary_is_unitary(D):
    rng = SplitMix64(11 + D)
    for _ in range(5):
        u = np.array(haar_unitary(rng, D)).reshape(D, D)
        assert np.max(np.abs(u.conj().T @ u - np.eye(D))) < 1e-14


@pytest.mark.parametrize("D", [3, 4])
def test_haar_unitary_moments(D):
    rng = SplitMix64(2024 + D)
    draws = 3000
    a2 = a4 = 0.0
    mean = 0j
    for _ in range(draws):
        u = np.array(haar_unitary(rng, D)).reshape(D, D)
        e = np.abs(u) ** 2
        a2 += e.mean()
        a4 += (e ** 2).mean()
        mean += u.mean()
    a2, a4, mean = a2 / draws, a4 / draws, mean / draws
    assert abs(a2 - 1.0 / D) < 1e-12           # rows of a unitary: exact
    want4 = 2.0 / (D * (D + 1))
    assert abs(a4 - want4) < 0.05 * want4       # several standard errors at 3000 draws
    assert abs(mean) < 0.02


def test_haar_unitary_is_deterministic():
    a = haar_unitary(substream(5, 6), 9)
    b = haar_unitary(substream(5, 6), 9)
    assert a == b


def test_general_circuit_shape():
    c = general_circuit(3, 10, 7, 2, 42)
    assert len(c.layers) == 7 and c.n_general_gates == 7 and c.n_phase_gates == 0
    for L, layer in enumerate(c.layers):
        assert [b.site for b in layer.bricks] == list(range(L % 2, 9, 2))
        (gg,) = layer.gates
        assert gg.k == 2 and 0 <= gg.site <= 8 and len(gg.u) == 81
    # the bricks are those of the plain brickwork generator with the same seed
    from paper_2511_06672_amd.workload import brickwork_circuit
    b = brickwork_circuit(3, 10, 7, 0, 42)
    assert [[x.word for x in L.bricks] for L in b.layers] == [[x.word for x in L.bricks] for L in c.layers]


def test_general_workloads():
    for name, d, k, cset in [("general_d3_n24", 3, 1, "listed"), ("general_d2_n24", 2, 2, "all_sp4")]:
        wl = workload(name)
        assert wl.circuit.d == d and wl.circuit.n == 24 and wl.circuit.n_general_gates == 24
        assert all(g.k == k for L in wl.circuit.layers for g in L.gates)
        assert wl.chi_max == 64 and wl.candidate_set == cset
        assert wl.chi_max * d ** (2 * k) <= 4096     # the library's bond capacity
    assert not math.isnan(workload("general_d3_n24").circuit.layers[0].gates[0].u[0].real)
