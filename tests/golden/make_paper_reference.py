"""Write the oracle's reference outputs for the paper's workload past the transition: qutrits,
N = 12, 18 layers (1.5 N) of a random Clifford followed by T on qudit 0 (§4, Fig. 3), no
truncation beyond the rank floor, the 90 unique disentanglers of §3 under the bond-dimension
criterion.

Calls only ``oracle/`` (and the seeded workload generator).  Per gate: choices, bond
dimensions, tableau digest, F_est; after the last gate <Z_j> on every site and the tableau.

    OPENBLAS_NUM_THREADS=4 python tests/golden/make_paper_reference.py [out_dir]
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

from oracle.disentanglers import exhaustive_disentanglers  # noqa: E402
from oracle.gcamps import Config, Gcamps  # noqa: E402
from paper_2511_06672_amd.workload import Word, workload  # noqa: E402

NAME, N, LAYERS = "paper_d3_n12", 12, 18


def tableau_digest(tab) -> str:
    """SHA-256 of the [2n][2n+1] tableau as little-endian int64 (first 16 hex digits)."""
    return hashlib.sha256(np.ascontiguousarray(tab, dtype="<i8").tobytes()).hexdigest()[:16]


def main():
    out_dir = sys.argv[1] if len(sys.argv) > 1 else HERE
    wl = workload(NAME, n=N, layers=LAYERS)
    c = wl.circuit
    words = [Word(tuple(w), (0, 0, 0, 0)) for w in exhaustive_disentanglers(c.d)]
    g = Gcamps(c.d, c.n, Config(chi_max=wl.chi_max, cutoff=wl.cutoff, criterion="bond_dim"), words)
    rec = {"workload": f"{NAME}, {LAYERS} layers", "d": c.d, "n": c.n, "layers": LAYERS, "chi_max": wl.chi_max,
           "cutoff": wl.cutoff, "candidates": len(words), "candidate_set": "exhaustive", "criterion": "bond_dim",
           "written_by": "oracle/ only", "gates": []}
    t_start = time.time()
    gi = 0
    for layer in c.layers:
        for b in layer.bricks:
            g.apply_clifford(b.site, b.word.gens, b.word.weyl)
        for ph in layer.phases:
            t0 = time.time()
            g.apply_phase_rotation(ph.site, ph.phi)
            rec["gates"].append({
                "gate": gi, "bond_dims": g.mps.bond_dims(), "f_est": g.f_est, "cpu_seconds": time.time() - t0,
                "choices": [[e.sweep, e.bond, e.choice] for e in g.choice_log if e.gate == gi],
                "tableau_sha256": tableau_digest(g.tab.export()),
            })
            print(f"gate {gi} maxchi {max(g.mps.bond_dims())} {time.time() - t0:.1f}s", flush=True)
            gi += 1
    zs = []
    for j in range(c.n):
        z = np.zeros(c.n, np.int64)
        z[j] = 1
        v = g.expectation(np.zeros(c.n, np.int64), z, 0)
        zs.append([v.real, v.imag])
    rec["gates_done"] = gi
    rec["cpu_seconds_total"] = time.time() - t_start
    rec["final_z_expectations"] = zs
    rec["final_tableau"] = g.tab.export().tolist()
    rec["final_after_gates"] = gi
    with open(os.path.join(out_dir, f"{NAME}_l{LAYERS}_oracle.json"), "w") as f:
        json.dump(rec, f)


if __name__ == "__main__":
    main()
