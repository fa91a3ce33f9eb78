"""Write the oracle's reference outputs for a sample of the batch workload's circuits (256
qutrit circuits, n ~ U{8..48}, T ~ U{4..60}, depth 2n, chi_max = 128, cutoff 1e-10, 512 shared
candidates, seed base 3000): the circuits given by index, each run whole.  Per circuit: the
choice log (gate, sweep, bond, choice), final bond dimensions, F_est and <Z_j> for every j.
FP64 scoring, two sweeps per gate.  Calls only ``oracle/`` (and the seeded workload generator).

    OPENBLAS_NUM_THREADS=4 python tests/golden/make_batch_reference.py [out_dir] [index ...]
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle.gcamps import Config, run_circuit  # noqa: E402
from paper_2511_06672_amd.workload import batch_workload  # noqa: E402

DEFAULT = [22, 1, 28, 8, 24, 27, 14, 12]   # small to mid circuits of the first 32; 27 reaches chi_max


def main():
    out_dir = sys.argv[1] if len(sys.argv) > 1 else HERE
    picks = [int(a) for a in sys.argv[2:]] or DEFAULT
    bw = batch_workload(count=256)
    rec = {"workload": "batch_d3 (256 circuits, seed base 3000)", "chi_max": bw.chi_max, "cutoff": bw.cutoff,
           "candidates": len(bw.candidates), "max_sweeps": bw.max_sweeps, "written_by": "oracle/ only",
           "circuits": []}
    for i in picks:
        c = bw.circuits[i]
        t0 = time.time()
        orc = run_circuit(c, bw.candidates, Config(chi_max=bw.chi_max, cutoff=bw.cutoff, max_sweeps=bw.max_sweeps))
        z = [orc.expectation([0] * c.n, [int(k == j) for k in range(c.n)], 0) for j in range(c.n)]
        rec["circuits"].append({
            "index": i, "n": c.n, "t_gates": c.n_phase_gates, "layers": len(c.layers),
            "choices": [[e.gate, e.sweep, e.bond, e.choice] for e in orc.choice_log],
            "bond_dims": orc.mps.bond_dims(), "f_est": orc.f_est,
            "z_re": [v.real for v in z], "z_im": [v.imag for v in z], "cpu_seconds": time.time() - t0,
        })
        print(f"circuit {i}: n={c.n} T={c.n_phase_gates} maxchi {max(orc.mps.bond_dims())} "
              f"f {orc.f_est:.15f} {time.time() - t0:.1f}s", flush=True)
    path = os.path.join(out_dir, "batch_d3_sample_oracle.json")
    with open(path + ".tmp", "w") as f:
        json.dump(rec, f)
    os.replace(path + ".tmp", path)


if __name__ == "__main__":
    main()
