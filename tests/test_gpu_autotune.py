"""Launch-parameter tuner: the rotated-matrix generator's candidates per thread (1, 2, 4 or 8) is
picked per (precision, d, chi_l, chi_r) by timing every choice on the first full-set chunk of a
bond; the choice changes only the speed, so every score must be bit-identical with tuning on or
off.  The picks persist in a JSON file (GCAMPS_TUNE_FILE) that later runs read back; an entry
naming a choice the call does not offer is timed again.

Checked on a saturated qubit state (chi = 128, 128 candidates, FP32 and split-BF16 scoring): bit
equality of every candidate's S2, the file's entry (the choice is the fastest of its four
timings), the cache hit on the next call, a hand-written entry being used, and an invalid one
being re-timed.  The decisions are read from the tuner's trace on stderr.
"""
import json
import sys

import numpy as np
import pytest

from paper_2511_06672_amd.workload import brickwork_circuit, candidate_words

pytestmark = pytest.mark.gpu
CHOICES = [1, 2, 4, 8]


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


def saturated(g, prec):
    d, n, chi, layers, ncand = 2, 15, 128, 30, 128
    c = brickwork_circuit(d, n, layers, layers, seed=602)
    st = g.State(g.make_config(d, n, chi, 0.0, score_prec=prec, auto_disentangle=False, max_candidates=ncand))
    for layer in c.layers:
        if layer.bricks:
            st.apply_clifford_layer([b.site for b in layer.bricks], [b.word for b in layer.bricks])
        for ph in layer.phases:
            st.apply_phase_rotation(ph.site, ph.phi)
    st.set_candset(g.CandSet(d, candidate_words(d, ncand, 612)))
    dims = [1] + st.bond_dims() + [1]
    i = int(np.argmax([dims[j] * dims[j + 2] for j in range(n - 1)]))
    return st, i, dims[i], dims[i + 2]


def entries(path, prec, cl, cr):
    with open(path) as f:
        data = json.load(f)
    return [e for e in data["entries"]
            if e["knob"] == "gen_cpt" and e["prec"] == prec and e["d"] == 2 and e["shape"] == [cl, cr]]


def decisions(err, cl, cr):
    tag = f"knob=gen_cpt prec="
    return [l for l in err.splitlines() if l.startswith("gcamps-tune") and tag in l and f"shape={cl}x{cr}" in l]


@pytest.mark.parametrize("prec_name", ["fp32", "bf16"])
def test_tuned_generator_is_bit_identical_and_cached(g, prec_name, tmp_path, monkeypatch, capfd):
    prec = g.SCORE_FP32 if prec_name == "fp32" else g.SCORE_BF16
    st, i, cl, cr = saturated(g, prec)
    say(f"autotune {prec_name}: bond {i}, chi_l={cl}, chi_r={cr}")
    assert min(cl * 2, 2 * cr) > 96  # the tiled path, where the generator runs
    monkeypatch.setenv("GCAMPS_AUTOTUNE", "0")
    off = st.score_bond(i)
    path = tmp_path / "tune.json"
    monkeypatch.setenv("GCAMPS_AUTOTUNE", "1")
    monkeypatch.setenv("GCAMPS_TUNE_FILE", str(path))
    monkeypatch.setenv("GCAMPS_TRACE_TUNE", "1")
    capfd.readouterr()
    on = st.score_bond(i)
    assert np.array_equal(on, off)
    ent = entries(path, prec, cl, cr)
    assert len(ent) == 1
    e = ent[0]
    assert e["choice"] in CHOICES and len(e["us"]) == len(CHOICES)
    assert e["choice"] == CHOICES[int(np.argmin(e["us"]))]
    err = capfd.readouterr().err
    assert any("source=timed" in l and f"choice={e['choice']}" in l for l in decisions(err, cl, cr)), err
    again = st.score_bond(i)
    assert np.array_equal(again, off)
    err = capfd.readouterr().err
    assert any("source=cache" in l for l in decisions(err, cl, cr)), err
    say(f"  timed {e['us']} us -> {e['choice']} candidates per thread")


def test_cache_file_entries_are_used_and_invalid_ones_retimed(g, tmp_path, monkeypatch, capfd):
    prec = g.SCORE_FP32
    st, i, cl, cr = saturated(g, prec)
    monkeypatch.setenv("GCAMPS_AUTOTUNE", "0")
    off = st.score_bond(i)
    monkeypatch.setenv("GCAMPS_AUTOTUNE", "1")
    monkeypatch.setenv("GCAMPS_TRACE_TUNE", "1")
    for choice, source in ((2, "cache"), (3, "timed")):
        path = tmp_path / f"tune_{choice}.json"
        path.write_text('{"entries": [\n'
                        f'  {{"knob": "gen_cpt", "prec": {prec}, "d": 2, "shape": [{cl}, {cr}], '
                        f'"choice": {choice}, "us": []}}\n'
                        ']}\n')
        monkeypatch.setenv("GCAMPS_TUNE_FILE", str(path))
        capfd.readouterr()
        s = st.score_bond(i)
        assert np.array_equal(s, off)
        dec = decisions(capfd.readouterr().err, cl, cr)
        assert any(f"source={source}" in l for l in dec), dec
        if source == "cache":
            assert any(f"choice={choice} source=cache" in l for l in dec), dec
        else:  # re-timed and written back with a valid choice
            ent = entries(path, prec, cl, cr)
            assert len(ent) == 1 and ent[0]["choice"] in CHOICES and len(ent[0]["us"]) == len(CHOICES)
