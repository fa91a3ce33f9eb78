"""GPU parity: the HIP path through the C ABI against the CPU oracle on seeded inputs.

Bars: tableaux, choice logs and bond dimensions bit-exact; amplitudes within 1e-10
after aligning the global phase (the tableau fixes C only up to a phase).  The
fidelity estimate F = prod(1 - eps) is compared to F_TOL relative: the GPU takes the
discarded weights eps from Gram eigen-decompositions whose eigenvalues carry an
absolute error of order m * 2^-52 * lambda_max each, so over T truncations with up to
m discarded values F can move by about T * m^2 * 1e-16 (1e-9 covers T = 1000, m = 100).
"""
import sys

F_TOL = 1e-9

import numpy as np
import pytest

from oracle.gcamps import Config, Gcamps
from oracle.statevector import simulate
from oracle.weyl import Weyl
from paper_2511_06672_amd.workload import (SplitMix64, brickwork_circuit, candidate_words,
                                           random_word, t_gate_phases, workload)

pytestmark = pytest.mark.gpu


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


def aligned_error(psi, ref):
    ov = np.vdot(psi, ref)
    return float(np.max(np.abs(psi * (ov / abs(ov)) - ref)))


def run_pair(g, circuit, cands, chi_max, cutoff, prec=0, auto=True, max_sweeps=2, near_tie=1e-3,
             max_candidates=None):
    cfg = g.make_config(circuit.d, circuit.n, chi_max, cutoff, score_prec=prec, near_tie=near_tie,
                        max_sweeps=max_sweeps, auto_disentangle=auto,
                        max_candidates=max_candidates or max(1, len(cands)))
    st = g.State(cfg)
    if cands:
        st.set_candset(g.CandSet(circuit.d, cands))
    orc = Gcamps(circuit.d, circuit.n, Config(chi_max=chi_max, cutoff=cutoff, max_sweeps=max_sweeps,
                                              auto_disentangle=auto), cands)
    for li, layer in enumerate(circuit.layers):
        if layer.bricks:
            st.apply_clifford_layer([b.site for b in layer.bricks], [b.word for b in layer.bricks])
            for b in layer.bricks:
                orc.apply_clifford(b.site, b.word.gens, b.word.weyl)
        for ph in layer.phases:
            st.apply_phase_rotation(ph.site, ph.phi)
            orc.apply_phase_rotation(ph.site, ph.phi)
    return st, orc


def oracle_log(orc):
    return np.array([[e.gate, e.sweep, e.bond, e.choice] for e in orc.choice_log], dtype=np.int64).reshape(-1, 4)


@pytest.mark.parametrize("d,n", [(2, 8), (3, 8), (3, 33), (2, 70)])
def test_tableau_layers_bit_exact(g, d, n):
    say(f"tableau layers d={d} n={n}")
    c = brickwork_circuit(d, n, 12, 0, seed=300 + d + n)
    st, orc = run_pair(g, c, [], 4, 0.0, auto=False)
    assert np.array_equal(st.tableau(), orc.tab.export())


def test_single_clifford_calls_and_expectations(g):
    d, n = 3, 6
    say("expectations on a Clifford state")
    rng = SplitMix64(41)
    st, orc = run_pair(g, brickwork_circuit(d, n, 3, 0, seed=41), [], 4, 0.0, auto=False)
    for _ in range(10):
        w = random_word(rng, d, 20)
        s = rng.below(n - 1)
        st.apply_clifford(s, w)
        orc.apply_clifford(s, w.gens, w.weyl)
    assert np.array_equal(st.tableau(), orc.tab.export())
    for _ in range(6):
        x = [rng.below(d) for _ in range(n)]
        z = [rng.below(d) for _ in range(n)]
        p = 2 * rng.below(d)
        assert abs(st.expectation(x, z, p) - orc.expectation(x, z, p)) < 1e-12


@pytest.mark.parametrize("d", [2, 3])
def test_phase_gates_without_disentangling(g, d):
    """Commute + MPO + compression only: state, bond dims and tableau equal the oracle's."""
    n = 6
    say(f"phase gates, no disentangling, d={d}")
    c = brickwork_circuit(d, n, 8, 5, seed=60 + d, one_per_layer=False)
    st, orc = run_pair(g, c, [], 64, 0.0, auto=False)
    assert st.bond_dims() == orc.mps.bond_dims()
    assert np.array_equal(st.tableau(), orc.tab.export())
    err = aligned_error(st.statevector(), orc.statevector())
    assert err < 1e-10, err
    assert aligned_error(st.statevector(), simulate(c)) < 1e-10


def test_exact_workload_parity(g):
    """qutrits n=8, 20 layers, 8 T gates, 512 candidates, no truncation (exact regime)."""
    wl = workload("exact_d3_n8")
    say("exact workload FP64 scoring")
    st, orc = run_pair(g, wl.circuit, wl.candidates, wl.chi_max, wl.cutoff)
    log = st.choice_log()
    assert np.array_equal(log, oracle_log(orc))
    assert np.array_equal(st.tableau(), orc.tab.export())
    assert st.bond_dims() == orc.mps.bond_dims()
    assert abs(st.fidelity() - orc.f_est) <= 1e-12
    psi = st.statevector()
    ref = simulate(wl.circuit)
    assert aligned_error(psi, ref) < 1e-10
    assert abs(np.linalg.norm(psi) - 1.0) < 1e-12


def test_exact_workload_fp32_scoring_same_choices(g):
    wl = workload("exact_d3_n8")
    say("exact workload FP32 scoring with FP64 window re-score")
    st, orc = run_pair(g, wl.circuit, wl.candidates, wl.chi_max, wl.cutoff, prec=1, near_tie=1e-3)
    assert np.array_equal(st.choice_log(), oracle_log(orc))
    assert np.array_equal(st.tableau(), orc.tab.export())
    assert aligned_error(st.statevector(), simulate(wl.circuit)) < 1e-10


@pytest.mark.parametrize("d,n", [(5, 4), (7, 3)])
@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32_scored"])
def test_larger_prime_d_exact_regime(g, d, n, prec):
    """d = 5 and 7 (tableau LUTs of 625 and 2401 entries, MPO bond d, d^2 x d^2 disentanglers):
    choices and tableau bit-exact against the oracle, the state against the dense simulation."""
    say(f"exact regime d={d} n={n} prec={prec}")
    c = brickwork_circuit(d, n, 8, 6, seed=600 + d, parametrised=True, one_per_layer=False)
    cands = candidate_words(d, 24, 600 + d)
    st, orc = run_pair(g, c, cands, d ** (n // 2), 0.0, prec=prec, near_tie=1e-4)
    assert np.array_equal(st.choice_log(), oracle_log(orc))
    assert np.array_equal(st.tableau(), orc.tab.export())
    assert aligned_error(st.statevector(), simulate(c)) < 1e-10


@pytest.mark.parametrize("d,n", [(5, 8), (7, 6)])
def test_larger_prime_d_truncated(g, d, n):
    """d = 5 and 7 with chi_max = d and cutoff 1e-10: truncation, choices, bonds, tableau and
    F_est against the oracle."""
    say(f"truncated regime d={d} n={n} chi_max={d}")
    c = brickwork_circuit(d, n, 10, 8, seed=610 + d, parametrised=True, one_per_layer=False)
    cands = candidate_words(d, 24, 610 + d)
    st, orc = run_pair(g, c, cands, d, 1e-10, near_tie=1e-4)
    assert orc.f_est < 1.0
    assert np.array_equal(st.choice_log(), oracle_log(orc))
    assert st.bond_dims() == orc.mps.bond_dims()
    assert np.array_equal(st.tableau(), orc.tab.export())
    assert abs(st.fidelity() - orc.f_est) <= F_TOL * orc.f_est


def test_truncated_regime_parity(g):
    """chi_max and cutoff active: choices, dims, tableau and F_est follow the oracle."""
    d, n = 3, 10
    say("truncated regime n=10 chi_max=9")
    c = brickwork_circuit(d, n, 16, 16, seed=77)
    cands = candidate_words(d, 96, 77)
    st, orc = run_pair(g, c, cands, 9, 1e-10)
    assert np.array_equal(st.choice_log(), oracle_log(orc))
    assert st.bond_dims() == orc.mps.bond_dims()
    assert np.array_equal(st.tableau(), orc.tab.export())
    assert abs(st.fidelity() - orc.f_est) <= F_TOL * orc.f_est
    assert aligned_error(st.statevector(), orc.statevector()) < 1e-9


def test_truncated_regime_large_bonds(g):
    """chi_max = 27 with many T gates: block-Jacobi splits, the centre-only split when the
    identity is kept, and truncation, all against the oracle."""
    d, n = 3, 10
    say("truncated regime n=10 chi_max=27")
    c = brickwork_circuit(d, n, 20, 20, seed=78)
    cands = candidate_words(d, 64, 78)
    st, orc = run_pair(g, c, cands, 27, 1e-10)
    assert st.stats()["centre_splits"] > 0
    assert np.array_equal(st.choice_log(), oracle_log(orc))
    assert st.bond_dims() == orc.mps.bond_dims()
    assert np.array_equal(st.tableau(), orc.tab.export())
    assert abs(st.fidelity() - orc.f_est) <= F_TOL * orc.f_est
    assert aligned_error(st.statevector(), orc.statevector()) < 1e-9


def test_large_matrices_block_paths(g):
    """Saturated bonds (chi up to 81 on n=8): block-Jacobi factorisations (m > 96) and the
    tiled MFMA scoring kernel, checked against the dense state and the oracle's choices."""
    d, n = 3, 8
    say("large matrices: saturating phase gates without disentangling")
    c = brickwork_circuit(d, n, 12, 12, seed=91)
    st, orc = run_pair(g, c, [], 81, 0.0, auto=False, max_candidates=64)
    assert max(st.bond_dims()) >= 27
    assert st.bond_dims() == orc.mps.bond_dims()
    assert aligned_error(st.statevector(), simulate(c)) < 1e-10
    cands = candidate_words(d, 48, 91)
    say("large matrices: one disentangling call, FP64 then FP32 scoring")
    cs = g.CandSet(d, cands)
    orc.candidates = list(cands)
    from oracle.clifford import word_matrix
    orc._cand_mats = [word_matrix(d, w.gens, w.weyl) for w in cands]
    st.disentangle(cs)
    orc.disentangle()
    assert np.array_equal(st.choice_log(), oracle_log(orc))
    assert np.array_equal(st.tableau(), orc.tab.export())
    assert st.bond_dims() == orc.mps.bond_dims()
    assert aligned_error(st.statevector(), orc.statevector()) < 1e-10


def test_bf16_scoring_same_choices(g):
    """Split-BF16 scoring (matrices above 96 rows) with the FP64 window re-score picks exactly
    the oracle's disentanglers on saturated bonds (n = 10, bonds up to 243, m up to 243)."""
    d, n = 3, 10
    say("split-BF16 scoring on saturated bonds")
    c = brickwork_circuit(d, n, 12, 12, seed=93)
    cands = candidate_words(d, 48, 94)
    st, orc = run_pair(g, c, [], 243, 0.0, prec=2, auto=False, max_candidates=48, near_tie=1e-4)
    assert max(st.bond_dims()) == 243
    cs = g.CandSet(d, cands)
    orc.candidates = list(cands)
    from oracle.clifford import word_matrix
    orc._cand_mats = [word_matrix(d, w.gens, w.weyl) for w in cands]
    st.disentangle(cs)
    orc.disentangle()
    assert st.stats()["tiled_launches"] > 0          # the BF16 Gram kernel ran
    assert np.array_equal(st.choice_log(), oracle_log(orc))
    assert np.array_equal(st.tableau(), orc.tab.export())
    assert st.bond_dims() == orc.mps.bond_dims()
    assert aligned_error(st.statevector(), orc.statevector()) < 1e-10


def test_error_paths(g):
    say("error paths")
    st = g.State(g.make_config(3, 4, 9, 0.0))
    with pytest.raises(g.GcampsError):
        st.apply_phase_rotation(7, [0.0, 0.1, 0.2])
    from paper_2511_06672_amd.workload import Word
    with pytest.raises(g.GcampsError):
        st.apply_clifford_layer([0, 1], [Word((0,), (0, 0, 0, 0)), Word((1,), (0, 0, 0, 0))])
    with pytest.raises(g.GcampsError):
        st.disentangle()                       # no candidate set attached
    assert st.bond_dims() == [1, 1, 1]
