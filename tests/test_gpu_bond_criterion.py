"""The bond-dimension criterion (GCAMPS_CRITERION_BOND_DIM) on the paper's own workload
(N = 12 qudits, N layers of a random Clifford followed by T on qudit 0, the exhaustive
disentangler set), against the oracle given the same words: choices, bond dimensions and tableau
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


def run_both(g, name, n):
    wl = workload(name, n=n)
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


@pytest.mark.parametrize("name,n", [("paper_d3_n12", 12), ("paper_d2_n12", 12), ("paper_d3_n12", 6),
                                    ("paper_d2_n12", 8)])
def test_paper_workload_bond_dimension_criterion(g, name, n):
    say(f"bond-dimension criterion {name} n={n}")
    c, st, orc = run_both(g, name, n)
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


def test_bond_dimension_criterion_limits(g):
    """Two-site matrices beyond the per-candidate SVD's size give EUNSUPPORTED; the criterion
    needs FP64 scores."""
    d, n = 3, 8
    say("bond-dimension criterion: size limit and configuration check")
    c = brickwork_circuit(d, n, 10, 10, seed=91)
    st = g.State(g.make_config(d, n, 81, 0.0, auto_disentangle=False, criterion=g.CRITERION_BOND_DIM,
                               max_candidates=90))
    for layer in c.layers:
        st.apply_clifford_layer([b.site for b in layer.bricks], [b.word for b in layer.bricks])
        for ph in layer.phases:
            st.apply_phase_rotation(ph.site, ph.phi)
    dims = [1] + st.bond_dims() + [1]
    assert any(min(dims[i] * d, d * dims[i + 2]) > 32 for i in range(n - 1))
    with pytest.raises(g.GcampsError) as e:
        st.disentangle(g.CandSet(d, g.clifford_words(d, g.WORDS_DISENTANGLERS)))
    assert e.value.code == -2
    with pytest.raises(g.GcampsError) as e:
        g.State(g.make_config(d, n, 27, 0.0, score_prec=g.SCORE_FP32, criterion=g.CRITERION_BOND_DIM))
    assert e.value.code == -1
