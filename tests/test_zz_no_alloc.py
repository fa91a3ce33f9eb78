"""gcamps_statevector_static (no allocation, static device scratch) against gcamps_statevector
(caller scratch) through the C ABI: bit-identical dense states on two calls in a row, the second
on a smaller state, then the refusal above the static size."""
import sys

import numpy as np
import pytest

from paper_2511_06672_amd.workload import brickwork_circuit, candidate_words

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


def state_of(g, d, n, layers, nt, seed):
    c = brickwork_circuit(d, n, layers, nt, seed=seed, one_per_layer=False)
    cands = candidate_words(d, 24, seed)
    st = g.State(g.make_config(d, n, d ** (n // 2), 0.0, max_candidates=len(cands)))
    st.set_candset(g.CandSet(d, cands))
    g.run_circuit(st, c)
    return st


def test_static_statevector_equals_the_scratch_variant_twice(g):
    for d, n, layers, nt, seed in [(3, 10, 8, 6, 71), (3, 6, 6, 4, 72)]:   # 59049, then 729 amplitudes
        say(f"static statevector d={d} n={n} D={d ** n}")
        st = state_of(g, d, n, layers, nt, seed)
        ref = st.statevector()
        got = st.statevector_static()
        assert got.shape == ref.shape
        assert np.array_equal(got, ref)
        assert abs(np.linalg.norm(got) - 1.0) < 1e-10


def test_static_statevector_refuses_above_its_size(g):
    say("static statevector refused at 3^11")
    st = g.State(g.make_config(3, 11, 4, 0.0))
    with pytest.raises(g.GcampsError) as e:
        st.statevector_static()
    assert e.value.code == -2
