"""gcamps_amplitude through the C ABI against the dense state-vector oracle (§3: psi = C|MPS>).

In the exact regime (no truncation beyond the rank floor) the state the library holds equals
the dense product of the circuit's gates up to one global phase, which the tableau leaves
undefined.  The phase is fixed once from the largest reference amplitude; every sampled
amplitude must then agree within 1e-10.  The amplitude call builds the dense state inside the
ctx's own workspace, so it must also equal the corresponding entry of gcamps_statevector bit
for bit.  Cases: the exact qutrit workload (3^8 = 6561 amplitudes, 512 candidates) and the
largest dense size the call accepts (2^16: sixteen qubits; 3^10 = 59049 for qutrits), plus the
refusal one site beyond it.
"""
import sys

import numpy as np
import pytest

from oracle.statevector import simulate
from paper_2511_06672_amd.workload import SplitMix64, brickwork_circuit, candidate_words, workload

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


def digits_of(y, d, n):
    out = []
    for _ in range(n):
        out.append(y % d)
        y //= d
    return out[::-1]


def sample_indices(ref, count, seed):
    """The largest amplitude, the next largest ones and seeded uniform indices."""
    order = np.argsort(-np.abs(ref))
    rng = SplitMix64(seed)
    picks = [int(i) for i in order[:8]] + [int(rng.below(ref.size)) for _ in range(count)]
    return picks


def check_amplitudes(g, st, ref, d, n, seed):
    picks = sample_indices(ref, 40, seed)
    amps = np.array([st.amplitude(digits_of(y, d, n)) for y in picks])
    y0 = picks[0]
    phase = (ref[y0] / amps[0]) / abs(ref[y0] / amps[0])
    err = float(np.max(np.abs(amps * phase - ref[picks])))
    assert err <= 1e-10, f"amplitude error {err:.3e}"
    full = st.statevector()
    assert np.array_equal(amps, full[picks]), "amplitude differs from the state vector entry"
    return err


def test_amplitude_exact_qutrit_workload(g):
    wl = workload("exact_d3_n8")
    c = wl.circuit
    say(f"amplitude exact_d3_n8 n={c.n} d={c.d} chi_max={wl.chi_max} cands={len(wl.candidates)}")
    st = g.State(g.make_config(c.d, c.n, wl.chi_max, wl.cutoff, max_candidates=len(wl.candidates)))
    st.set_candset(g.CandSet(c.d, wl.candidates))
    g.run_circuit(st, c)
    ref = simulate(c)
    check_amplitudes(g, st, ref, c.d, c.n, 11)


@pytest.mark.parametrize("d,n,layers,nt", [(2, 16, 12, 10), (3, 10, 8, 6)])
def test_amplitude_at_the_dense_limit(g, d, n, layers, nt):
    assert d ** n <= 1 << 16
    c = brickwork_circuit(d, n, layers, nt, seed=4100 + d, one_per_layer=False)
    cands = candidate_words(d, 32, 4100 + d)
    chi = d ** (n // 2)
    say(f"amplitude at the dense limit d={d} n={n} D={d ** n} chi_max={chi}")
    st = g.State(g.make_config(d, n, chi, 0.0, max_candidates=len(cands)))
    st.set_candset(g.CandSet(d, cands))
    g.run_circuit(st, c)
    ref = simulate(c)
    check_amplitudes(g, st, ref, d, n, 13 + d)


def test_amplitude_refused_beyond_the_dense_limit(g):
    say("amplitude refused at 2^17")
    st = g.State(g.make_config(2, 17, 4, 0.0))
    with pytest.raises(g.GcampsError) as e:
        st.amplitude([0] * 17)
    assert e.value.code == -2
    with pytest.raises(g.GcampsError) as e:
        st.amplitude([0] * 16 + [2])  # digit out of range is checked before the size? either is an error
    assert e.value.code in (-1, -2)
