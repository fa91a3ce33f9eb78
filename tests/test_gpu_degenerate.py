"""Degenerate and extreme inputs of the bottom loop, against the oracle and the dense state:
the shortest chain (n = 2), a circuit with no non-Clifford gate, phase gates whose value is the
identity or a Clifford (a single Weyl term, so no bond grows), an empty Clifford layer through
the C ABI, disentangling switched off (max_sweeps = 0), and the state vector at its size limit
(d^n = 2^16).  Bars as in the other parity tests: choices, bond dimensions and tableau bit-exact,
F_est relative 1e-9, amplitudes 1e-10 after aligning the global phase."""
import ctypes as C
import math
import sys

import numpy as np
import pytest

from oracle.gcamps import Config, Gcamps
from oracle.statevector import simulate
from paper_2511_06672_amd.workload import Circuit, Layer, PhaseGate, brickwork_circuit, candidate_words

pytestmark = pytest.mark.gpu
F_TOL = 1e-9


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def g():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2511_06672_amd import gcamps
    gcamps.lib()
    return gcamps


def aligned(a, b):
    ov = np.vdot(a, b)
    return float(np.max(np.abs(a * (ov / abs(ov)) - b)))


def run_both(g, c, cands, chi_max, cutoff, max_sweeps=2):
    st = g.State(g.make_config(c.d, c.n, chi_max, cutoff, max_sweeps=max_sweeps, max_candidates=max(1, len(cands))))
    if cands:
        st.set_candset(g.CandSet(c.d, cands))
    g.run_circuit(st, c)
    orc = Gcamps(c.d, c.n, Config(chi_max=chi_max, cutoff=cutoff, max_sweeps=max_sweeps), cands)
    for layer in c.layers:
        for b in layer.bricks:
            orc.apply_clifford(b.site, b.word.gens, b.word.weyl)
        for ph in layer.phases:
            orc.apply_phase_rotation(ph.site, ph.phi)
    return st, orc


def same(st, orc):
    log = st.choice_log()
    want = np.array([[e.gate, e.sweep, e.bond, e.choice] for e in orc.choice_log]).reshape(-1, 4)
    assert np.array_equal(log, want)
    assert st.bond_dims() == orc.mps.bond_dims()
    assert np.array_equal(st.tableau(), orc.tab.export())
    assert abs(st.fidelity() - orc.f_est) <= F_TOL * orc.f_est


@pytest.mark.parametrize("d", [2, 3])
def test_two_site_chain(g, d):
    say(f"two-site chain d={d}")
    c = brickwork_circuit(d, 2, 12, 12, seed=500 + d)
    st, orc = run_both(g, c, candidate_words(d, 24, 500 + d), d, 0.0)
    same(st, orc)
    assert aligned(st.statevector(), simulate(c)) < 1e-10


def test_clifford_only_circuit(g):
    say("Clifford-only circuit d=3 n=6")
    c = brickwork_circuit(3, 6, 10, 0, seed=510)
    assert c.n_phase_gates == 0
    st, orc = run_both(g, c, candidate_words(3, 16, 510), 27, 0.0)
    same(st, orc)
    assert st.bond_dims() == [1] * 5 and st.fidelity() == 1.0 and len(st.choice_log()) == 0
    assert aligned(st.statevector(), simulate(c)) < 1e-10


@pytest.mark.parametrize("d", [2, 3])
def test_identity_and_clifford_valued_phases(g, d):
    """diag(1, ..., 1) is the identity and diag(omega^j) = Z a single Weyl term: neither grows a
    bond or needs disentangling; the state equals the dense product."""
    say(f"identity and Z-valued phase gates d={d}")
    base = brickwork_circuit(d, 5, 6, 0, seed=520 + d)
    ident = tuple(0.0 for _ in range(d))
    zgate = tuple(2 * math.pi * j / d for j in range(d))
    layers = []
    for li, layer in enumerate(base.layers):
        layers.append(Layer(layer.bricks, [PhaseGate(li % 5, ident), PhaseGate((li + 2) % 5, zgate)]))
    c = Circuit(d, 5, layers)
    st, orc = run_both(g, c, candidate_words(d, 16, 520 + d), d ** 2, 0.0)
    same(st, orc)
    assert st.bond_dims() == [1] * 4 and st.fidelity() == 1.0
    assert aligned(st.statevector(), simulate(c)) < 1e-10


def test_empty_layer_and_no_disentangling(g):
    say("empty Clifford layer through the C ABI; max_sweeps = 0")
    c = brickwork_circuit(3, 5, 8, 6, seed=530, one_per_layer=False)
    st, orc = run_both(g, c, candidate_words(3, 16, 530), 81, 0.0, max_sweeps=0)
    same(st, orc)
    assert len(st.choice_log()) == 0
    before = st.statevector()
    sites = (C.c_int32 * 1)(0)
    words = (g.CWord * 1)()
    assert g.lib().gcamps_apply_clifford_layer(st.handle, sites, words, 0) == 0
    assert np.array_equal(st.statevector(), before)
    assert aligned(before, simulate(c)) < 1e-10


def test_statevector_at_its_size_limit(g):
    say("state vector at d^n = 2^16 (qubits, n = 16)")
    c = brickwork_circuit(2, 16, 10, 6, seed=540)
    st, orc = run_both(g, c, candidate_words(2, 16, 540), 256, 0.0)
    same(st, orc)
    assert aligned(st.statevector(), simulate(c)) < 1e-10
