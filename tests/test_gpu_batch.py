"""Batched independent circuits (gcamps_batch_run) against the single-state path and the oracle.

Every circuit of a batch must give exactly what it gives alone through gcamps_init and the
single-state calls (same kernels, so bit-identical), and what the oracle gives: the same
disentangler choices and bond dimensions, the fidelity estimate within F_TOL and <Z_j>
within Z_TOL.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

F_TOL = 1e-9     # relative, fidelity estimate (same derivation as the single-state parity tests)
Z_TOL = 1e-8     # absolute, <Z_j> of a unit-norm state after a few hundred FP64 factorisations


def small_batch(count=6, seed=3100):
    from paper_2511_06672_amd.workload import batch_workload
    return batch_workload(count=count, seed=seed, n_range=(4, 8), t_range=(2, 6), chi_max=27,
                          cutoff=1e-10, n_candidates=48, name="batch_small")


def configs(g, bw, precs):
    return [g.make_config(3, c.n, bw.chi_max, bw.cutoff, score_prec=p, near_tie=1e-4,
                          max_candidates=len(bw.candidates))
            for c, p in zip(bw.circuits, precs)]


def single_state(g, c, cfg, cs):
    st = g.State(cfg)
    st.set_candset(cs)
    g.run_circuit(st, c)
    z = []
    for j in range(c.n):
        zz = [0] * c.n
        zz[j] = 1
        z.append(st.expectation([0] * c.n, zz, 0))
    return st, np.array(z)


def test_batch_matches_single_state_and_oracle():
    import torch
    from oracle.gcamps import Config, run_circuit
    from paper_2511_06672_amd import gcamps as g
    assert torch.cuda.is_available()
    bw = small_batch()
    precs = [i % 2 for i in range(len(bw.circuits))]
    cfgs = configs(g, bw, precs)
    cs = g.CandSet(3, bw.candidates)
    print(f"[gpu-case] batch of {len(bw.circuits)} circuits, lanes=3", flush=True)
    res, stats = g.batch_run(bw.circuits, cfgs, cs, lanes=3)
    assert stats["circuits"] == len(bw.circuits)
    assert stats["gates"] == bw.n_phase_gates
    assert stats["lanes"] == 3
    for i, (c, cfg, r) in enumerate(zip(bw.circuits, cfgs, res)):
        print(f"[gpu-case] circuit {i}: n={c.n} T={c.n_phase_gates} prec={cfg.score_prec}", flush=True)
        assert r["status"] == 0
        st, z = single_state(g, c, cfg, cs)
        assert r["fidelity"] == st.fidelity()
        assert r["bond_dims"] == st.bond_dims()
        assert np.array_equal(r["choices"], st.choice_log())
        assert np.array_equal(r["z_expect"], z)
        orc = run_circuit(c, bw.candidates, Config(chi_max=bw.chi_max, cutoff=bw.cutoff, max_sweeps=2))
        mine = [list(map(int, e)) for e in r["choices"]]
        theirs = [[e.gate, e.sweep, e.bond, e.choice] for e in orc.choice_log]
        assert mine == theirs, f"choices differ in circuit {i}"
        assert r["bond_dims"] == orc.mps.bond_dims()
        assert abs(r["fidelity"] - orc.f_est) <= F_TOL * orc.f_est
        zo = np.array([orc.expectation([0] * c.n, [int(k == j) for k in range(c.n)], 0) for j in range(c.n)])
        assert np.max(np.abs(r["z_expect"] - zo)) <= Z_TOL


def test_batch_results_do_not_depend_on_lane_count():
    from paper_2511_06672_amd import gcamps as g
    bw = small_batch(count=5, seed=3200)
    cfgs = configs(g, bw, [1] * 5)
    cs = g.CandSet(3, bw.candidates)
    print("[gpu-case] batch lanes 1 vs 5", flush=True)
    r1, s1 = g.batch_run(bw.circuits, cfgs, cs, lanes=1)
    r5, s5 = g.batch_run(bw.circuits, cfgs, cs, lanes=5)
    assert s1["lanes"] == 1 and s5["lanes"] == 5
    for a, b in zip(r1, r5):
        assert a["fidelity"] == b["fidelity"] and a["bond_dims"] == b["bond_dims"]
        assert np.array_equal(a["choices"], b["choices"])
        assert np.array_equal(a["z_expect"], b["z_expect"])


def test_batch_reports_the_failing_item_and_finishes_the_rest():
    from paper_2511_06672_amd import gcamps as g
    bw = small_batch(count=4, seed=3300)
    cfgs = configs(g, bw, [0] * 4)
    cfgs[2].max_candidates = 8          # smaller than the 48-word set: ECAPACITY for item 2 only
    cs = g.CandSet(3, bw.candidates)
    print("[gpu-case] batch with one failing item", flush=True)
    with pytest.raises(g.GcampsError) as e:
        g.batch_run(bw.circuits, cfgs, cs, lanes=2)
    assert e.value.code == -4
    assert "batch item 2" in str(e.value)


def test_batch_without_candidates_only_compresses():
    from paper_2511_06672_amd import gcamps as g
    bw = small_batch(count=3, seed=3400)
    cfgs = configs(g, bw, [0] * 3)
    print("[gpu-case] batch without candidate set", flush=True)
    res, stats = g.batch_run(bw.circuits, cfgs, None, lanes=2)
    assert stats["bonds"] == 0
    for r in res:
        assert r["status"] == 0 and r["choices_len"] == 0


def test_many_lanes_on_the_batch_workload():
    """32 circuits of the batch workload on 12 concurrent lanes: every circuit completes, and two
    of them equal their single-state runs bit for bit.  (Concurrent lanes slow some waves of a
    workgroup relative to others; the single-workgroup eigensolver once read its convergence
    flag after the next sweep had reset it, which only showed up under such load.)"""
    from paper_2511_06672_amd import gcamps as g
    from paper_2511_06672_amd.workload import batch_workload
    print("[gpu-case] batch workload, 32 circuits on 12 lanes", flush=True)
    bw = batch_workload(count=32)
    cfgs = [g.make_config(3, c.n, bw.chi_max, bw.cutoff, score_prec=g.SCORE_FP32, near_tie=1e-4,
                          max_sweeps=bw.max_sweeps, max_candidates=len(bw.candidates)) for c in bw.circuits]
    cs = g.CandSet(3, bw.candidates)
    res, stats = g.batch_run(bw.circuits, cfgs, cs, lanes=12)
    assert all(r["status"] == 0 for r in res) and stats["circuits"] == 32
    for i in (0, 19):
        st, _ = single_state(g, bw.circuits[i], cfgs[i], cs)
        assert res[i]["fidelity"] == st.fidelity()
        assert res[i]["bond_dims"] == st.bond_dims()


def test_batch_workload_sample_against_oracle_reference():
    """The first 32 circuits of the batch workload in one batch on 12 lanes (the benchmark's
    configuration: FP32 scoring with the FP64 near-tie window); eight of them, from product-like
    to one that reaches chi_max = 128 with truncation, against the oracle's references
    (tests/golden/batch_d3_sample_oracle.json, written by make_batch_reference.py from oracle/
    only): choices and bond dimensions exact, F_est within F_TOL, <Z_j> within Z_TOL."""
    import json
    import os
    from paper_2511_06672_amd import gcamps as g
    from paper_2511_06672_amd.workload import batch_workload
    ref = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "batch_d3_sample_oracle.json")))
    bw = batch_workload(count=32)
    assert ref["chi_max"] == bw.chi_max and ref["candidates"] == len(bw.candidates)
    print("[gpu-case] batch workload, 32 circuits on 12 lanes, oracle sample", flush=True)
    cfgs = [g.make_config(3, c.n, bw.chi_max, bw.cutoff, score_prec=g.SCORE_FP32, near_tie=1e-4,
                          max_sweeps=bw.max_sweeps, max_candidates=len(bw.candidates)) for c in bw.circuits]
    res, _ = g.batch_run(bw.circuits, cfgs, g.CandSet(3, bw.candidates), lanes=12)
    for r in ref["circuits"]:
        i = r["index"]
        mine = res[i]
        print(f"[gpu-case] circuit {i}: n={r['n']} T={r['t_gates']}", flush=True)
        assert mine["status"] == 0
        assert [list(map(int, e)) for e in mine["choices"]] == r["choices"], f"choices differ in circuit {i}"
        assert mine["bond_dims"] == r["bond_dims"]
        assert abs(mine["fidelity"] - r["f_est"]) <= F_TOL * r["f_est"]
        zo = np.array(r["z_re"]) + 1j * np.array(r["z_im"])
        assert np.max(np.abs(mine["z_expect"] - zo)) <= Z_TOL
