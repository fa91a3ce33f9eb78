"""Pins of the oracle's reverse-mode derivative of the frozen GCAMPS forward pass
(oracle/adjoint.py), against definitions that do not share its arithmetic:

* without truncation the frozen forward pass is the circuit itself, so the reverse sweep must
  give the dense derivative of the circuit state (oracle/gradient.py, one gate differentiated at
  a time); this also exercises the projection term of every exact split, whose kept ranks equal
  the Schmidt ranks (the (1 - P) dM term of a rank-deficient cut);
* with truncation it must give the derivative of the oracle's own frozen replay, measured by
  Richardson-extrapolated central differences (error O(h^4)).

A dropped renormalisation, a dropped or mis-signed projector-derivative term, or a wrong
coefficient derivative each fails one of these (the truncated case moves the loss derivative
by far more than the tolerance when any of them is removed)."""
import numpy as np

from oracle.adjoint import frozen_adjoint
from oracle.gcamps import Config
from oracle.gradient import dense_gradient, dense_loss, fd_gradient, record
from paper_2511_06672_amd.workload import brickwork_circuit, candidate_words, workload
from test_oracle_gradient import theta_of


def test_adjoint_equals_the_dense_derivative_without_truncation():
    c = brickwork_circuit(3, 6, 12, 4, 702, one_per_layer=False, parametrised=True)
    th = theta_of(c)
    cands = candidate_words(3, 24, 702)
    cfg = Config(chi_max=27, cutoff=0.0)
    st, frozen = record(c, cands, cfg, th)
    loss, g, st2, v = frozen_adjoint(c, cands, cfg, th, frozen)
    assert np.max(np.abs(v - st2.mps.to_dense())) < 1e-12     # the dense replay is the MPS
    assert abs(loss - dense_loss(c, th)) < 1e-12
    gd = dense_gradient(c, th)
    assert np.max(np.abs(gd)) > 1e-2
    assert np.max(np.abs(g - gd)) <= 1e-12 * max(1.0, np.max(np.abs(gd)))


def test_adjoint_equals_finite_differences_of_the_truncated_replay():
    c = workload("grad_d3_n24", n=6).circuit
    th = theta_of(c)
    cands = candidate_words(3, 24, 704)
    cfg = Config(chi_max=4, cutoff=1e-10)
    st, frozen = record(c, cands, cfg, th)
    assert st.f_est < 0.99                                      # truncation happened
    loss, g, st2, v = frozen_adjoint(c, cands, cfg, th, frozen)
    assert loss == st2.loss_sum_z() or abs(loss - st2.loss_sum_z()) < 1e-13
    sel = list(range(0, len(th), max(1, len(th) // 8)))
    fd = fd_gradient(c, cands, cfg, th, frozen, h=1e-5, params=sel, richardson=True)
    scale = np.max(np.abs(g))
    assert scale > 1e-3
    assert np.max(np.abs(g[sel] - fd[sel])) <= 1e-7 * scale
