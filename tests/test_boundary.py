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
