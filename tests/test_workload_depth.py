"""The paper's workload stands in a deep brickwork circuit for each layer's random n-qudit Clifford
(n sublayers of random two-qudit words).  Check on the oracle that the stand-in is deep enough:
doubling it to 2n sublayers leaves the bond-dimension trajectory under the bond-dimension
criterion unchanged within its seed-to-seed spread (qubits, N = 6, twelve layers, 24 circuits per
depth; the exact regime, chi_max = 2^3).  Per layer, the mean of log2 chi over the circuits of
each depth may differ by at most three standard errors of the difference plus 0.05; the first
layer where chi exceeds 1 likewise."""
import numpy as np

from oracle.disentanglers import exhaustive_disentanglers
from oracle.gcamps import Config, Gcamps
from paper_2511_06672_amd.workload import Word, paper_circuit


def trajectory(d, n, layers, seed, depth):
    words = [Word(w, (0, 0, 0, 0)) for w in exhaustive_disentanglers(d)]
    c = paper_circuit(d, n, layers, seed, depth=depth)
    g = Gcamps(d, n, Config(chi_max=d ** (n // 2), cutoff=0.0, criterion="bond_dim"), words)
    out = []
    for layer in c.layers:
        for b in layer.bricks:
            g.apply_clifford(b.site, b.word.gens, b.word.weyl)
        for ph in layer.phases:
            g.apply_phase_rotation(ph.site, ph.phi)
            out.append(max(g.mps.bond_dims()))
    return out


def test_clifford_depth_does_not_change_the_bond_trajectory():
    d, n, layers, count = 2, 6, 12, 24
    runs = {depth: np.log2(np.array([trajectory(d, n, layers, 7000 + 100 * depth + s, depth)
                                     for s in range(count)]))
            for depth in (n, 2 * n)}
    a, b = runs[n], runs[2 * n]
    se = np.sqrt(a.var(0) / count + b.var(0) / count)
    assert np.all(np.abs(a.mean(0) - b.mean(0)) <= 3 * se + 0.05)
    assert a[:, -1].mean() > 1.5 and a[:, 0].max() == 0.0     # the run does cross the transition
    fa = np.array([np.argmax(r > 0) if (r > 0).any() else layers for r in a])
    fb = np.array([np.argmax(r > 0) if (r > 0).any() else layers for r in b])
    assert abs(fa.mean() - fb.mean()) <= 3 * np.sqrt(fa.var() / count + fb.var() / count) + 0.05
