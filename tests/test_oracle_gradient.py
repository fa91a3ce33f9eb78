"""Pins of the oracle's loss gradient (oracle/gradient.py): a hand-derived closed form,
finite differences of the dense loss, agreement of the frozen GCAMPS replay with the dense
derivative when nothing is truncated, and consistency of the replay itself."""
import math

import numpy as np

from oracle.gcamps import Config
from oracle.gradient import dense_gradient, dense_loss, fd_gradient, record, replay_loss
from paper_2511_06672_amd.workload import (Brick, Circuit, Layer, PhaseGate, Word, brickwork_circuit,
                                           candidate_words)


def theta_of(circuit):
    out = []
    for L in circuit.layers:
        for ph in sorted(L.phases, key=lambda p: p.param):
            if ph.param >= 0:
                out.append((ph.param, ph.phi[1:]))
    out.sort()
    return np.array([x for _, phi in out for x in phi])


def test_dense_loss_and_gradient_closed_form():
    # F on qutrit 0, diag(1, e^{i t1}, e^{i t2}), F again:  <Z_0> = <phi|F^dag Z F|phi> with
    # F^dag Z F a cyclic shift, so Re<Z_0> = (cos t1 + cos t2 + cos(t1 - t2))/3 and <Z_1> = 1.
    f_a = Word((0,), (0, 0, 0, 0))
    t1, t2 = 0.7, -1.9
    c = Circuit(3, 2, [Layer([Brick(0, f_a)], [PhaseGate(0, (0.0, t1, t2), 0)]), Layer([Brick(0, f_a)], [])])
    theta = np.array([t1, t2])
    want = (math.cos(t1) + math.cos(t2) + math.cos(t1 - t2)) / 3.0 + 1.0
    assert abs(dense_loss(c, theta) - want) < 1e-14
    g = dense_gradient(c, theta)
    want_g = np.array([-math.sin(t1) - math.sin(t1 - t2), -math.sin(t2) + math.sin(t1 - t2)]) / 3.0
    assert np.max(np.abs(g - want_g)) < 1e-14


def test_dense_gradient_matches_dense_finite_differences():
    from paper_2511_06672_amd.workload import workload
    c = workload("grad_d3_n24", n=4).circuit
    th = theta_of(c)
    g = dense_gradient(c, th)
    assert np.max(np.abs(g)) > 1e-2
    h = 1e-5
    fd = np.array([(dense_loss(c, th + h * e) - dense_loss(c, th - h * e)) / (2 * h) for e in np.eye(len(th))])
    assert np.max(np.abs(g - fd)) < 1e-8 * max(1.0, np.max(np.abs(g)))


def test_frozen_replay_gradient_equals_dense_gradient_without_truncation():
    c = brickwork_circuit(3, 6, 12, 4, 702, one_per_layer=False, parametrised=True)
    th = theta_of(c)
    cands = candidate_words(3, 24, 702)
    cfg = Config(chi_max=27, cutoff=0.0)
    st, frozen = record(c, cands, cfg, th)
    assert abs(st.loss_sum_z() - dense_loss(c, th)) < 1e-10
    assert replay_loss(c, cands, cfg, th, frozen) == st.loss_sum_z()
    g = dense_gradient(c, th)
    assert np.max(np.abs(g)) > 1e-2                        # a loss that depends on theta
    fd = fd_gradient(c, cands, cfg, th, frozen, h=1e-5)
    assert np.max(np.abs(fd - g)) <= 1e-7 * np.max(np.abs(g))


def test_frozen_replay_in_the_truncated_regime_is_smooth():
    """With decisions frozen, the truncated forward pass is smooth: central differences
    converge at the O(h^2) rate (halving h divides their change by about four)."""
    from paper_2511_06672_amd.workload import workload
    c = workload("grad_d3_n24", n=8).circuit
    th = theta_of(c)
    cands = candidate_words(3, 24, 703)
    cfg = Config(chi_max=9, cutoff=1e-10)
    st, frozen = record(c, cands, cfg, th)
    assert st.f_est < 0.999                       # truncation happened
    assert replay_loss(c, cands, cfg, th, frozen) == st.loss_sum_z()
    sel = [0, 3, 7, 10]
    g = [fd_gradient(c, cands, cfg, th, frozen, h=h, params=sel)[sel] for h in (1e-4, 5e-5, 2.5e-5)]
    assert np.max(np.abs(g[2])) > 1e-3            # a loss that depends on theta
    e1, e2 = np.abs(g[0] - g[1]), np.abs(g[1] - g[2])
    assert np.all(e2 <= 0.3 * e1 + 1e-9)
