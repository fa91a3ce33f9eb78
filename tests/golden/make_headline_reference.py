"""Write the oracle's reference outputs for the headline workload (qutrits, n = 32,
40 brickwork layers, one T gate per layer, chi_max = 256, cutoff 1e-10, 512
candidates, FP64 scoring).

Calls only ``oracle/`` (and the seeded workload generator).  The JSON is rewritten
after every non-Clifford gate, so an interrupted run still leaves a valid prefix:
``gates_done`` says how many gates are covered.

    OPENBLAS_NUM_THREADS=4 python tests/golden/make_headline_reference.py [n] [out_dir]
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

from oracle.gcamps import Config, Gcamps  # noqa: E402
from oracle.mps import bond_renyi2  # noqa: E402
from paper_2511_06672_amd.workload import workload  # noqa: E402


def tableau_digest(tab) -> str:
    """SHA-256 of the [2n][2n+1] tableau as little-endian int64 (first 16 hex digits)."""
    return hashlib.sha256(np.ascontiguousarray(tab, dtype="<i8").tobytes()).hexdigest()[:16]


def main():
    n = int(sys.argv[1]) if len(sys.argv) > 1 else 32
    wl = workload("headline_d3_n32", n=None if n == 32 else n)
    c = wl.circuit
    out_dir = sys.argv[2] if len(sys.argv) > 2 else HERE
    out_path = os.path.join(out_dir, f"headline_d3_n{n}_oracle.json")
    g = Gcamps(c.d, c.n, Config(chi_max=wl.chi_max, cutoff=wl.cutoff, max_sweeps=wl.max_sweeps),
               wl.candidates)
    rec = {"workload": wl.name, "d": c.d, "n": c.n, "layers": len(c.layers), "chi_max": wl.chi_max,
           "cutoff": wl.cutoff, "candidates": len(wl.candidates), "written_by": "oracle/ only",
           "gates": []}
    gi = 0
    t_start = time.time()
    for L, layer in enumerate(c.layers):
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
    zs = []
    for j in range(c.n):
        z = np.zeros(c.n, np.int64)
        z[j] = 1
        v = g.expectation(np.zeros(c.n, np.int64), z, 0)
        zs.append([v.real, v.imag])
    rec["final_z_expectations"] = zs
    rec["final_tableau"] = g.tab.export().tolist()
    rec["final_bond_renyi2"] = bond_renyi2(g.mps.tensors)
    rec["final_after_gates"] = rec["gates_done"]
    with open(out_path + ".tmp", "w") as f:
        json.dump(rec, f)
    os.replace(out_path + ".tmp", out_path)
    print("final <Z_j> written", flush=True)


if __name__ == "__main__":
    main()
