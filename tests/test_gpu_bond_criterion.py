"""The bond-dimension criterion (GCAMPS_CRITERION_BOND_DIM) on the paper's own workload
(N = 12 qudits, N layers of a random Clifford followed by T on qudit 0, the exhaustive
disentangler set; and 1.5 N layers, past the transition), against the oracle given the same words: choices, bond dimensions and tableau
bit-exact, F_est relative 1e-9; in the exact regime of a smaller copy, the state against the
dense simulation (1e-10 after aligning the global phase)."""
import sys

import numpy as np
import pytest

from oracle.gcamps import Config, Gcamps
from oracle.statevector import simulate
from paper_2511_06672_amd.workload import brickwork_circuit, workload

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


def run_both(g, name, n, layers=None):
    wl = workload(name, n=n, layers=layers)
    c = wl.circuit
    words = g.clifford_words(c.d, g.WORDS_DISENTANGLERS)
    st = g.State(g.make_config(c.d, c.n, wl.chi_max, wl.cutoff, criterion=g.CRITERION_BOND_DIM,
                               max_candidates=len(words)))
    st.set_candset(g.CandSet(c.d, words))
    orc = Gcamps(c.d, c.n, Config(chi_max=wl.chi_max, cutoff=wl.cutoff, criterion="bond_dim"), words)
    for layer in c.layers:
        if layer.bricks:
            st.apply_clifford_layer([b.site for b in layer.bricks], [b.word for b in layer.bricks])
            for b in layer.bricks:
                orc.apply_clifford(b.site, b.word.gens, b.word.weyl)
        for ph in layer.phases:
            st.apply_phase_rotation(ph.site, ph.phi)
            orc.apply_phase_rotation(ph.site, ph.phi)
    return c, st, orc


@pytest.mark.parametrize("name,n,layers", [("paper_d3_n12", 12, None), ("paper_d2_n12", 12, None),
                                           ("paper_d3_n12", 6, None), ("paper_d2_n12", 8, None),
                                           ("paper_d2_n12", 12, 18), ("paper_d3_n12", 8, 12)])
def test_paper_workload_bond_dimension_criterion(g, name, n, layers):
    """N layers (the onset of the transition), and 1.5 N layers past it, where two-site matrices
    outgrow the batched per-candidate SVD and every candidate goes through the split's own
    factorisation."""
    say(f"bond-dimension criterion {name} n={n} layers={layers or n}")
    c, st, orc = run_both(g, name, n, layers)
    log = st.choice_log()
    want = np.array([[e.gate, e.sweep, e.bond, e.choice] for e in orc.choice_log]).reshape(-1, 4)
    assert np.array_equal(log, want)
    assert np.any(log[:, 3] != 0)
    assert st.bond_dims() == orc.mps.bond_dims()
    assert np.array_equal(st.tableau(), orc.tab.export())
    assert abs(st.fidelity() - orc.f_est) <= F_TOL * orc.f_est
    if c.d ** c.n <= 2 ** 16:
        psi, ref = st.statevector(), simulate(c)
        ov = np.vdot(psi, ref)
        assert np.max(np.abs(psi * (ov / abs(ov)) - ref)) < 1e-10


def test_bond_dimension_criterion_on_large_bonds_and_configuration(g):
    """Bonds whose two-site matrices exceed the batched SVD's size (smaller side > 32) on a
    brickwork circuit, disentangled under the criterion: choices, bonds and tableau equal the
    oracle's; the criterion needs FP64 scores."""
    from oracle.gcamps import Config, Gcamps
    d, n = 3, 8
    say("bond-dimension criterion on large bonds")
    c = brickwork_circuit(d, n, 10, 10, seed=91)
    words = g.clifford_words(d, g.WORDS_DISENTANGLERS)
    st = g.State(g.make_config(d, n, 81, 0.0, auto_disentangle=False, criterion=g.CRITERION_BOND_DIM,
                               max_candidates=90))
    orc = Gcamps(d, n, Config(chi_max=81, cutoff=0.0, criterion="bond_dim", auto_disentangle=False), words)
    for layer in c.layers:
        st.apply_clifford_layer([b.site for b in layer.bricks], [b.word for b in layer.bricks])
        for b in layer.bricks:
            orc.apply_clifford(b.site, b.word.gens, b.word.weyl)
        for ph in layer.phases:
            st.apply_phase_rotation(ph.site, ph.phi)
            orc.apply_phase_rotation(ph.site, ph.phi)
    dims = [1] + st.bond_dims() + [1]
    assert any(min(dims[i] * d, d * dims[i + 2]) > 32 for i in range(n - 1))
    st.disentangle(g.CandSet(d, words))
    orc.disentangle()
    log = st.choice_log()
    want = np.array([[e.gate, e.sweep, e.bond, e.choice] for e in orc.choice_log]).reshape(-1, 4)
    assert np.array_equal(log, want)
    assert st.bond_dims() == orc.mps.bond_dims()
    assert np.array_equal(st.tableau(), orc.tab.export())
    with pytest.raises(g.GcampsError) as e:
        g.State(g.make_config(d, n, 27, 0.0, score_prec=g.SCORE_FP32, criterion=g.CRITERION_BOND_DIM))
    assert e.value.code == -1


def test_paper_workload_past_the_transition_against_stored_reference(g):
    """Qutrits, N = 12, 1.5 N = 18 layers: bonds reach 3^6 = 729, so nearly every bond's
    candidates go through the split's own factorisation.  Expected values: the oracle's run in
    tests/golden/paper_d3_n12_l18_oracle.json (make_paper_reference.py, oracle only), with the
    oracle's own enumeration of the 90 unique disentanglers as the candidate list on both sides.
    Choices, bonds and tableau per gate bit-exact, F_est 1e-9, final <Z_j> 1e-8."""
    import hashlib
    import json
    import os
    from oracle.disentanglers import exhaustive_disentanglers
    from paper_2511_06672_amd.workload import Word
    path = os.path.join(os.path.dirname(__file__), "golden", "paper_d3_n12_l18_oracle.json")
    ref = json.load(open(path))
    wl = workload("paper_d3_n12", n=12, layers=ref["layers"])
    c = wl.circuit
    words = [Word(tuple(w), (0, 0, 0, 0)) for w in exhaustive_disentanglers(c.d)]
    assert len(words) == ref["candidates"] == 90
    say(f"paper workload past the transition: d=3 n=12 layers={ref['layers']}")
    st = g.State(g.make_config(c.d, c.n, wl.chi_max, wl.cutoff, criterion=g.CRITERION_BOND_DIM,
                               max_candidates=len(words)))
    st.set_candset(g.CandSet(c.d, words))
    gi, prev = 0, 0
    for layer in c.layers:
        if layer.bricks:
            st.apply_clifford_layer([b.site for b in layer.bricks], [b.word for b in layer.bricks])
        for ph in layer.phases:
            st.apply_phase_rotation(ph.site, ph.phi)
            r = ref["gates"][gi]
            log = st.choice_log()
            mine, prev = log[prev:], len(log)
            assert [list(map(int, x[1:])) for x in mine] == r["choices"], f"choices differ at gate {gi}"
            assert st.bond_dims() == r["bond_dims"], f"bond dims differ at gate {gi}"
            dig = hashlib.sha256(np.ascontiguousarray(st.tableau(), dtype="<i8").tobytes()).hexdigest()[:16]
            assert dig == r["tableau_sha256"], f"tableau differs at gate {gi}"
            assert abs(st.fidelity() - r["f_est"]) <= F_TOL * r["f_est"], f"fidelity differs at gate {gi}"
            gi += 1
    assert gi == ref["gates_done"]
    assert max(st.bond_dims()) == 729
    n = c.n
    got = np.array([[v.real, v.imag] for v in
                    (st.expectation([0] * n, [1 if k == j else 0 for k in range(n)]) for j in range(n))])
    assert np.max(np.abs(got - np.array(ref["final_z_expectations"]))) <= 1e-8
    assert np.array_equal(st.tableau(), np.array(ref["final_tableau"]))
