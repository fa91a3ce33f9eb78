"""General non-Clifford gates (gcamps_apply_gate) against the oracle's Gcamps.apply_gate.

Bars as in the other parity tests: amplitudes 1e-10 after aligning the global phase in the
exact regime; with truncation and disentangling, choices, bond dimensions and tableau
bit-exact and F_est relative 1e-9.
"""
import sys

import numpy as np
import pytest

from oracle.gcamps import Config, Gcamps
from paper_2511_06672_amd.workload import brickwork_circuit, candidate_words

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


def random_unitary(rng, D):
    q, r = np.linalg.qr(rng.normal(size=(D, D)) + 1j * rng.normal(size=(D, D)))
    return q * (np.diag(r) / np.abs(np.diag(r)))


def aligned(a, b):
    ov = np.vdot(a, b)
    return float(np.max(np.abs(a * (ov / abs(ov)) - b)))


def both(g, d, n, chi_max, cutoff, cands, auto, seed, layers, gate_every, k):
    """The same circuit on the GPU and in the oracle: brickwork layers with T gates, and a
    random k-site unitary after every `gate_every`-th layer."""
    rng = np.random.default_rng(seed)
    c = brickwork_circuit(d, n, layers, layers, seed)
    st = g.State(g.make_config(d, n, chi_max, cutoff, auto_disentangle=auto, max_candidates=max(1, len(cands)),
                               max_gate_terms=d ** (2 * k)))
    if cands:
        st.set_candset(g.CandSet(d, cands))
    orc = Gcamps(d, n, Config(chi_max=chi_max, cutoff=cutoff, auto_disentangle=auto), cands)
    for li, layer in enumerate(c.layers):
        if layer.bricks:
            st.apply_clifford_layer([b.site for b in layer.bricks], [b.word for b in layer.bricks])
            for b in layer.bricks:
                orc.apply_clifford(b.site, b.word.gens, b.word.weyl)
        for ph in layer.phases:
            st.apply_phase_rotation(ph.site, ph.phi)
            orc.apply_phase_rotation(ph.site, ph.phi)
        if li % gate_every == gate_every - 1:
            u = random_unitary(rng, d ** k)
            site = int(rng.integers(0, n - k + 1))
            st.apply_gate(site, u)
            orc.apply_gate(site, u)
    return st, orc


@pytest.mark.parametrize("d,n,k", [(2, 6, 1), (2, 6, 2), (3, 5, 1), (3, 5, 2)])
def test_general_gates_exact_regime(g, d, n, k):
    say(f"general gates exact regime d={d} n={n} k={k}")
    st, orc = both(g, d, n, d ** (n // 2), 0.0, [], False, 300 + 10 * d + k, 8, 2, k)
    assert st.bond_dims() == orc.mps.bond_dims()
    assert np.array_equal(st.tableau(), orc.tab.export())
    assert aligned(st.statevector(), orc.statevector()) < 1e-10


@pytest.mark.parametrize("d,n,chi_max,layers", [(2, 10, 8, 12), (3, 6, 9, 9)])
def test_general_two_site_gates_with_disentangling(g, d, n, chi_max, layers):
    cands = candidate_words(d, 32, 310 + d)
    say(f"general two-site gates with truncation and disentangling d={d} n={n} chi_max={chi_max}")
    st, orc = both(g, d, n, chi_max, 1e-10, cands, True, 320 + d, layers, 3, 2)
    log = st.choice_log()
    want = np.array([[e.gate, e.sweep, e.bond, e.choice] for e in orc.choice_log]).reshape(-1, 4)
    assert np.array_equal(log, want)
    assert st.bond_dims() == orc.mps.bond_dims()
    assert np.array_equal(st.tableau(), orc.tab.export())
    assert abs(st.fidelity() - orc.f_est) <= F_TOL * orc.f_est
    assert orc.f_est < 1.0                                   # truncation happened
    assert aligned(st.statevector(), orc.statevector()) < 1e-9


def test_diagonal_gate_matches_phase_rotation_and_errors(g):
    d, n = 3, 6
    say("diagonal apply_gate vs phase rotation; error paths")
    phi = [0.0, 0.4, -2.1]
    c = brickwork_circuit(d, n, 4, 4, 330)
    sts = []
    for use_gate in (False, True):
        st = g.State(g.make_config(d, n, 27, 0.0, auto_disentangle=False))
        for layer in c.layers:
            st.apply_clifford_layer([b.site for b in layer.bricks], [b.word for b in layer.bricks])
            if use_gate:
                st.apply_gate(2, np.diag(np.exp(1j * np.array(phi))))
            else:
                st.apply_phase_rotation(2, phi)
        sts.append(st)
    assert sts[0].bond_dims() == sts[1].bond_dims()
    assert aligned(sts[0].statevector(), sts[1].statevector()) < 1e-12
    st = sts[0]
    with pytest.raises(g.GcampsError) as e:
        st.apply_gate(1, np.ones((3, 3)))                    # not unitary
    assert e.value.code == -1
    rng = np.random.default_rng(5)
    with pytest.raises(g.GcampsError) as e:
        st.apply_gate(1, random_unitary(rng, 9))             # 81 terms > max_gate_terms (d)
    assert e.value.code == -4
    with pytest.raises(g.GcampsError):
        st.apply_gate(n - 1, random_unitary(rng, 9))         # second site beyond the chain
