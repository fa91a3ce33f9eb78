"""Write the oracle's reference outputs for a prefix of the mixed-run workloads
(qubits: n = 64, 64 layers, one T per layer, chi_max = 1024, cutoff 1e-12, the 720 elements
of Sp(4, Z_2) as candidates; qutrits: n = 48, 60 layers, one T per layer, chi_max = 1024,
cutoff 1e-12, identity + 719 random candidates), FP64 scoring.

Calls only ``oracle/`` (and the seeded workload generator).  The JSON is rewritten after every
non-Clifford gate; ``gates_done`` says how many gates are covered.  The run stops after
``max_gates`` gates or once ``budget`` CPU seconds have passed.

    OPENBLAS_NUM_THREADS=4 python tests/golden/make_mixed_reference.py {2|3} [max_gates] [budget_s] [out_dir]
"""
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle.disentanglers import all_cliffords  # noqa: E402
from oracle.gcamps import Config, Gcamps  # noqa: E402
from oracle.mps import bond_renyi2  # noqa: E402
from paper_2511_06672_amd.workload import Word, workload  # noqa: E402


def tableau_digest(tab) -> str:
    """SHA-256 of the [2n][2n+1] tableau as little-endian int64 (first 16 hex digits)."""
    return hashlib.sha256(np.ascontiguousarray(tab, dtype="<i8").tobytes()).hexdigest()[:16]


def candidates(wl):
    if wl.candidate_set == "all_sp4":
        return [Word(w, (0, 0, 0, 0)) for w, _ in all_cliffords(wl.circuit.d)]
    return wl.candidates


def finish(rec, g, out_path):
    """Record the final state at the end of the covered prefix: <Z_j> for every site and the
    tableau.  Written once, after the last covered gate."""
    zs = []
    for j in range(g.n):
        z = np.zeros(g.n, np.int64)
        z[j] = 1
        v = g.expectation(np.zeros(g.n, np.int64), z, 0)
        zs.append([v.real, v.imag])
    rec["final_z_expectations"] = zs
    rec["final_tableau"] = g.tab.export().tolist()
    rec["final_bond_renyi2"] = bond_renyi2(g.mps.tensors)
    rec["final_after_gates"] = rec.get("gates_done", 0)
    with open(out_path + ".tmp", "w") as f:
        json.dump(rec, f)
    os.replace(out_path + ".tmp", out_path)
    print(f"final <Z_j> written after {rec['final_after_gates']} gates", flush=True)


def main():
    d = int(sys.argv[1])
    max_gates = int(sys.argv[2]) if len(sys.argv) > 2 else 10 ** 6
    budget = float(sys.argv[3]) if len(sys.argv) > 3 else 3600.0
    out_dir = sys.argv[4] if len(sys.argv) > 4 else HERE
    name = "mixed_d2_n64" if d == 2 else "mixed_d3_n48"
    wl = workload(name)
    c = wl.circuit
    cands = candidates(wl)
    out_path = os.path.join(out_dir, f"{name}_oracle.json")
    g = Gcamps(c.d, c.n, Config(chi_max=wl.chi_max, cutoff=wl.cutoff, max_sweeps=wl.max_sweeps), cands)
    rec = {"workload": wl.name, "d": c.d, "n": c.n, "layers": len(c.layers), "chi_max": wl.chi_max,
           "cutoff": wl.cutoff, "candidates": len(cands), "candidate_set": wl.candidate_set,
           "written_by": "oracle/ only", "gates": []}
    gi = 0
    t_start = time.time()
    for L, layer in enumerate(c.layers):
        # the covered prefix ends after a layer's non-Clifford gate, before the next layer's
        # bricks, which is where the GPU test stops too (one T gate per layer here)
        if gi >= max_gates or time.time() - t_start > budget:
            return finish(rec, g, out_path)
        for b in layer.bricks:
            g.apply_clifford(b.site, b.word.gens, b.word.weyl)
        for ph in layer.phases:
            t0 = time.time()
            g.apply_phase_rotation(ph.site, ph.phi)
            dt = time.time() - t0
            rec["gates"].append({
                "gate": gi, "layer": L, "site": ph.site, "support": list(g.last_support),
                "bond_dims": g.mps.bond_dims(), "f_est": g.f_est, "cpu_seconds": dt,
                "choices": [[e.sweep, e.bond, e.choice] for e in g.choice_log if e.gate == gi],
                "tableau_sha256": tableau_digest(g.tab.export()),
            })
            rec["gates_done"] = gi + 1
            rec["flags"] = g.flags
            rec["cpu_seconds_total"] = time.time() - t_start
            with open(out_path + ".tmp", "w") as f:
                json.dump(rec, f)
            os.replace(out_path + ".tmp", out_path)
            print(f"gate {gi} maxchi {max(g.mps.bond_dims())} f {g.f_est:.15f} {dt:.1f}s", flush=True)
            gi += 1
    finish(rec, g, out_path)


if __name__ == "__main__":
    main()
