"""Replica-tensor scoring (GCAMPS_SCORE_REPLICA) against the oracle.

* Scores: every candidate's S2 at every bond of saturated states (both cuts: chi_l < chi_r
  takes the left table, chi_l > chi_r the right one; bonds with m <= 96 go to the direct FP64
  kernel), element by element against the oracle's direct definition on the same two-site
  tensor, and against the library's own FP64 mode.
  Tolerance 1e-9 absolute in S2 (= relative in the purity): the pair sum adds up to
  X^2/2 * d^8 FP64 products (X <= 243 here), whose rounding stays orders of magnitude below;
  the near-tie window (>= 1e-6) is far wider, so the FP64 re-score sees every near tie.
* Choices: one disentangling call on saturated bonds picks exactly the oracle's candidates.
"""
import sys

import numpy as np
import pytest

from oracle.clifford import word_matrix
from oracle.gcamps import Config, Gcamps, renyi2
from paper_2511_06672_amd.workload import brickwork_circuit, candidate_words

pytestmark = pytest.mark.gpu

S2_TOL = 1e-9


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


def saturated_state(g, d, n, chi_max, prec, seed, ncand, layers):
    c = brickwork_circuit(d, n, layers, layers, seed=seed)
    st = g.State(g.make_config(d, n, chi_max, 0.0, score_prec=prec, auto_disentangle=False,
                               max_candidates=ncand))
    for layer in c.layers:
        if layer.bricks:
            st.apply_clifford_layer([b.site for b in layer.bricks], [b.word for b in layer.bricks])
        for ph in layer.phases:
            st.apply_phase_rotation(ph.site, ph.phi)
    return c, st


def oracle_scores(d, theta, mats):
    cl, _, _, cr = theta.shape
    t = theta.reshape(cl, d * d, cr)
    return np.array([renyi2(np.einsum("xy,ayb->axb", q, t).reshape(theta.shape)) for q in mats])


@pytest.mark.parametrize("d,n,chi_max,layers", [(3, 11, 243, 14), (2, 15, 128, 30)])
def test_replica_scores_match_oracle(g, d, n, chi_max, layers):
    """Bonds saturate (3^min(j, n-j), 2^min(j, n-j) capped at chi_max): the bonds next to the
    middle have chi_l != chi_r with m > 96 on both sides."""
    ncand = 40
    cands = candidate_words(d, ncand, 401 + d)
    mats = [word_matrix(d, w.gens, w.weyl) for w in cands]
    say(f"replica scores d={d} n={n} chi_max={chi_max}")
    _, st = saturated_state(g, d, n, chi_max, g.SCORE_REPLICA, 400 + d, ncand, layers)
    _, ref = saturated_state(g, d, n, chi_max, g.SCORE_FP64, 400 + d, ncand, layers)
    dims = [1] + st.bond_dims() + [1]
    assert dims == [1] + ref.bond_dims() + [1]
    cs = g.CandSet(d, cands)
    st.set_candset(cs)
    ref.set_candset(cs)
    cuts = set()
    for i in range(n - 1):
        cl, cr = dims[i], dims[i + 2]
        say(f"  bond {i}: chi_l={cl} chi_r={cr}")
        s_rep = st.score_bond(i)
        s_64 = ref.score_bond(i)
        a, b = st.site(i), st.site(i + 1)
        theta = np.tensordot(a, b, axes=([2], [0]))           # (chi_l, d, d, chi_r)
        assert theta.shape == (cl, d, d, cr)
        s_orc = oracle_scores(d, theta, mats)
        assert np.max(np.abs(s_rep - s_orc)) < S2_TOL, (i, np.max(np.abs(s_rep - s_orc)))
        assert np.max(np.abs(s_rep - s_64)) < S2_TOL
        if min(cl * d, d * cr) > 96:
            cuts.add("left" if cl <= cr else "right")
    assert cuts == {"left", "right"}                          # both tables were exercised


def test_replica_choices_match_oracle(g):
    """One disentangling call on saturated qutrit bonds (n = 10, chi up to 243, m up to 243)."""
    d, n = 3, 10
    cands = candidate_words(d, 48, 404)
    say("replica scoring: disentangling call on saturated bonds")
    c = brickwork_circuit(d, n, 12, 12, seed=93)
    st = g.State(g.make_config(d, n, 243, 0.0, score_prec=g.SCORE_REPLICA, near_tie=1e-4,
                               auto_disentangle=False, max_candidates=48))
    orc = Gcamps(d, n, Config(chi_max=243, cutoff=0.0, auto_disentangle=False), [])
    for layer in c.layers:
        if layer.bricks:
            st.apply_clifford_layer([b.site for b in layer.bricks], [b.word for b in layer.bricks])
            for b in layer.bricks:
                orc.apply_clifford(b.site, b.word.gens, b.word.weyl)
        for ph in layer.phases:
            st.apply_phase_rotation(ph.site, ph.phi)
            orc.apply_phase_rotation(ph.site, ph.phi)
    assert max(st.bond_dims()) == 243
    orc.candidates = list(cands)
    orc._cand_mats = [word_matrix(d, w.gens, w.weyl) for w in cands]
    st.disentangle(g.CandSet(d, cands))
    orc.disentangle()
    log = st.choice_log()
    want = np.array([[e.gate, e.sweep, e.bond, e.choice] for e in orc.choice_log]).reshape(-1, 4)
    assert np.array_equal(log, want)
    assert np.any(log[:, 3] != 0)                             # some non-identity choice
    assert np.array_equal(st.tableau(), orc.tab.export())
    assert st.bond_dims() == orc.mps.bond_dims()
    ov = np.vdot(st.statevector(), orc.statevector())
    assert abs(abs(ov) - 1.0) < 1e-10
