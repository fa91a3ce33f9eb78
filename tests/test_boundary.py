"""CPU checks of the C-ABI library: it loads, exports every symbol declared in
include/gcamps.h, and rejects bad arguments before touching a device."""
import os
import re

import pytest

from paper_2511_06672_amd import gcamps as g
from paper_2511_06672_amd.workload import IDENTITY_WORD, Word, candidate_words

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    text = open(os.path.join(ROOT, "include", "gcamps.h")).read()
    return sorted(set(re.findall(r"\b(gcamps_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = g.lib()
    declared = header_symbols()
    assert declared == sorted(g.SYMBOLS)
    for name in declared:
        assert hasattr(lib, name), name


def test_workspace_sizing_and_validation():
    b1 = g.workspace_bytes(g.make_config(3, 8, 81, 0.0))
    b2 = g.workspace_bytes(g.make_config(3, 32, 256, 1e-10))
    assert 0 < b1 < b2 < 4 << 30
    with pytest.raises(g.GcampsError) as e:
        g.workspace_bytes(g.make_config(4, 8, 16, 0.0))          # non-prime d
    assert e.value.code == -2
    for bad in (g.make_config(3, 1, 16, 0.0), g.make_config(3, 8, 0, 0.0),
                g.make_config(3, 8, 16, -1.0), g.make_config(3, 8, 16, 0.0, score_prec=7),
                g.make_config(3, 8, 16, 0.0, score_prec=1, near_tie=1e-9),
                g.make_config(3, 8, 16, 0.0, max_candidates=0)):
        with pytest.raises(g.GcampsError) as e:
            g.workspace_bytes(bad)
        assert e.value.code == -1


def test_near_tie_floor_of_the_low_precision_modes():
    """FP32 and split-BF16 scoring need a re-score window of at least 1e-4 (twice their
    measured S2 error and more), so that the FP64 choice always lies inside it; replica
    scoring is FP64 arithmetic and keeps the 1e-6 floor; FP64 scoring ignores the field."""
    for prec in (g.SCORE_FP32, g.SCORE_BF16):
        assert g.workspace_bytes(g.make_config(3, 8, 16, 0.0, score_prec=prec, near_tie=1e-4)) > 0
        with pytest.raises(g.GcampsError) as e:
            g.workspace_bytes(g.make_config(3, 8, 16, 0.0, score_prec=prec, near_tie=9.9e-5))
        assert e.value.code == -1
    assert g.workspace_bytes(g.make_config(3, 8, 16, 0.0, score_prec=g.SCORE_REPLICA, near_tie=1e-6)) > 0
    assert g.workspace_bytes(g.make_config(3, 8, 16, 0.0, score_prec=g.SCORE_FP64, near_tie=0.0)) > 0


def test_dense_region_is_counted_only_for_small_states():
    """The amplitude call builds the dense state inside the ctx workspace (4 complex128 plus
    an 8 + n byte table per index) whenever d^n <= 2^16, so it needs no allocation."""
    def ws(d, n):
        return g.workspace_bytes(g.make_config(d, n, 4, 0.0))
    # qubits: 2^16 has the region, 2^17 does not; the difference dominates everything else
    assert ws(2, 16) - ws(2, 17) > (1 << 16) * (64 + 8 + 16) - (1 << 20)
    assert ws(2, 16) >= (1 << 16) * (64 + 8 + 16)


def test_replica_mode_sizing_and_validation():
    """Replica scoring: d = 2, 3 only; its workspace holds the candidate tables
    (2 * N_c * d^8 complex128) and scratch for the Gram of Theta over chi_max d^2 rows."""
    plain = g.workspace_bytes(g.make_config(3, 32, 256, 1e-10, score_prec=g.SCORE_FP32, max_candidates=512))
    rep = g.workspace_bytes(g.make_config(3, 32, 256, 1e-10, score_prec=g.SCORE_REPLICA, max_candidates=512))
    assert rep - plain >= 2 * 512 * 3 ** 8 * 16
    assert g.workspace_bytes(g.make_config(2, 16, 64, 1e-10, score_prec=g.SCORE_REPLICA)) > 0
    with pytest.raises(g.GcampsError) as e:
        g.workspace_bytes(g.make_config(5, 8, 16, 0.0, score_prec=g.SCORE_REPLICA))
    assert e.value.code == -2


def test_criterion_validation():
    assert g.workspace_bytes(g.make_config(3, 8, 27, 0.0, criterion=g.CRITERION_BOND_DIM)) > 0
    for bad in (g.make_config(3, 8, 27, 0.0, criterion=2),
                g.make_config(3, 8, 27, 0.0, score_prec=g.SCORE_REPLICA, criterion=g.CRITERION_BOND_DIM)):
        with pytest.raises(g.GcampsError) as e:
            g.workspace_bytes(bad)
        assert e.value.code == -1


def test_candset_validation():
    cs = g.CandSet(3, candidate_words(3, 8, 3))
    assert cs.count == 8
    with pytest.raises(g.GcampsError):                              # first word not identity
        g.CandSet(3, [Word((0,), (0, 0, 0, 0))])
    with pytest.raises(g.GcampsError):                              # bad generator code
        g.CandSet(3, [IDENTITY_WORD, Word((9,), (0, 0, 0, 0))])
    with pytest.raises(g.GcampsError):                              # Weyl exponent >= d
        g.CandSet(3, [IDENTITY_WORD, Word((1,), (0, 3, 0, 0))])
    with pytest.raises(g.GcampsError):                              # non-prime d
        g.CandSet(4, [IDENTITY_WORD])


def test_init_rejects_small_workspace_without_device_work():
    import ctypes as C
    cfg = g.make_config(3, 8, 16, 0.0)
    h = C.c_void_p()
    code = g.lib().gcamps_init(C.byref(cfg), C.c_void_p(256), 16, None, C.byref(h))
    assert code == -3                                               # EWORKSPACE
    code = g.lib().gcamps_init(C.byref(cfg), C.c_void_p(257), 1 << 40, None, C.byref(h))
    assert code == -1                                               # misaligned workspace


def test_struct_layouts_match_the_header(tmp_path):
    """The ctypes mirrors of the header's structs have the C compiler's sizes and offsets."""
    import ctypes as C
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    fields = {
        "gcamps_config": (g.Config, ["d", "n", "chi_max", "cutoff", "score_prec", "near_tie", "tie_tol",
                                     "max_sweeps", "auto_disentangle", "max_candidates", "max_gate_terms",
                                     "criterion"]),
        "gcamps_word": (g.CWord, ["len", "gens", "weyl"]),
        "gcamps_op": (g.COp, ["kind", "count", "sites", "words", "phi"]),
        "gcamps_batch_item": (g.CBatchItem, ["cfg", "ops", "n_ops", "status", "fidelity", "bond_dims",
                                             "z_expect", "choices", "choices_cap", "choices_len"]),
    }
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "gcamps.h"', "int main(void) {"]
    for cname, (_, names) in fields.items():
        lines.append(f'printf("%zu\\n", sizeof({cname}));')
        for f in names:
            lines.append(f'printf("%zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    vals = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    expect = []
    for cname, (cls, names) in fields.items():
        expect.append(C.sizeof(cls))
        expect.extend(getattr(cls, f).offset for f in names)
    assert vals == expect


def test_batch_validation_without_device_work():
    import ctypes as C
    from paper_2511_06672_amd.workload import brickwork_circuit
    c = brickwork_circuit(3, 5, 4, 2, 11, one_per_layer=False)
    keep = []
    ops, nops = g._circuit_ops(c, keep)
    items = (g.CBatchItem * 2)()
    for it in items:
        it.cfg = g.make_config(3, 5, 9, 0.0)
        it.ops = ops
        it.n_ops = nops
    b1, b2 = C.c_size_t(0), C.c_size_t(0)
    assert g.lib().gcamps_batch_workspace_bytes(items, 2, 1, C.byref(b1)) == 0
    assert g.lib().gcamps_batch_workspace_bytes(items, 2, 4, C.byref(b2)) == 0
    assert b2.value == 2 * b1.value                                  # min(lanes, count) slices
    assert b1.value >= g.workspace_bytes(items[0].cfg)
    assert g.lib().gcamps_batch_workspace_bytes(items, 2, 0, C.byref(b1)) == -1     # lanes < 1
    assert g.lib().gcamps_batch_workspace_bytes(items, 0, 1, C.byref(b1)) == -1     # empty batch
    items[1].cfg = g.make_config(4, 5, 9, 0.0)
    assert g.lib().gcamps_batch_workspace_bytes(items, 2, 1, C.byref(b1)) == -2     # non-prime d
    items[1].cfg = g.make_config(3, 5, 9, 0.0)
    ops[0].kind = 7
    assert g.lib().gcamps_batch_workspace_bytes(items, 2, 1, C.byref(b1)) == -1     # unknown op
    assert "unknown kind" in g.lib().gcamps_last_error().decode()
    ops[0].kind = g.OP_CLIFFORD_LAYER
    assert g.lib().gcamps_batch_run(items, 2, None, 1, C.c_void_p(256), 16, None) == -3  # EWORKSPACE
    assert g.lib().gcamps_batch_run(items, 2, None, 1, C.c_void_p(257), 1 << 40, None) == -1
