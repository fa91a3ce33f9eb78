"""ctypes binding of libgcamps (include/gcamps.h), same names as the C ABI.

This module only marshals arguments: every step of the simulation runs in the
library's HIP kernels.  PyTorch supplies the device workspace (one uint8 tensor)
and the HIP stream.  Importing it without a built library raises: there is no
fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Iterable, List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgcamps.so")

GCAMPS_OK = 0
STATUS_NAMES = {0: "OK", -1: "EINVAL", -2: "EUNSUPPORTED", -3: "EWORKSPACE", -4: "ECAPACITY",
                -5: "EDEVICE", -6: "ENUMERIC"}
SCORE_FP64, SCORE_FP32, SCORE_BF16, SCORE_REPLICA = 0, 1, 2, 3
FACTORIZE_REDUCE = 1
WORDS_DISENTANGLERS, WORDS_ALL = 0, 1
CRITERION_RENYI2, CRITERION_BOND_DIM = 0, 1

SYMBOLS = [
    "gcamps_workspace_bytes", "gcamps_init", "gcamps_destroy", "gcamps_apply_clifford",
    "gcamps_apply_clifford_layer", "gcamps_apply_phase_rotation", "gcamps_apply_gate", "gcamps_candset_create",
    "gcamps_candset_destroy", "gcamps_clifford_words", "gcamps_set_candset", "gcamps_score_bond",
    "gcamps_factorize", "gcamps_disentangle", "gcamps_expectation",
    "gcamps_statevector", "gcamps_statevector_static", "gcamps_amplitude", "gcamps_get_tableau", "gcamps_get_bond_dims",
    "gcamps_get_fidelity", "gcamps_get_choice_log", "gcamps_get_site", "gcamps_get_stats",
    "gcamps_get_kernel_stats",
    "gcamps_batch_workspace_bytes", "gcamps_batch_run", "gcamps_grad_record", "gcamps_grad_loss",
    "gcamps_grad_gradient", "gcamps_grad_stats", "gcamps_grad_destroy", "gcamps_last_error",
]


class GcampsError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class Config(C.Structure):
    _fields_ = [("d", C.c_int32), ("n", C.c_int32), ("chi_max", C.c_int32), ("cutoff", C.c_double),
                ("score_prec", C.c_int32), ("near_tie", C.c_double), ("tie_tol", C.c_double),
                ("max_sweeps", C.c_int32), ("auto_disentangle", C.c_int32),
                ("max_candidates", C.c_int32), ("max_gate_terms", C.c_int32), ("criterion", C.c_int32)]


class CWord(C.Structure):
    _fields_ = [("len", C.c_int32), ("gens", C.POINTER(C.c_uint8)), ("weyl", C.c_int32 * 4)]


OP_CLIFFORD_LAYER, OP_PHASE = 0, 1


class COp(C.Structure):
    _fields_ = [("kind", C.c_int32), ("count", C.c_int32), ("sites", C.POINTER(C.c_int32)),
                ("words", C.POINTER(CWord)), ("phi", C.POINTER(C.c_double))]


class CBatchItem(C.Structure):
    _fields_ = [("cfg", Config), ("ops", C.POINTER(COp)), ("n_ops", C.c_int64),
                ("status", C.POINTER(C.c_int32)), ("fidelity", C.POINTER(C.c_double)),
                ("bond_dims", C.POINTER(C.c_int32)), ("z_expect", C.POINTER(C.c_double)),
                ("choices", C.POINTER(C.c_int32)), ("choices_cap", C.c_int64),
                ("choices_len", C.POINTER(C.c_int64))]


def load_library(path: str = LIB_PATH) -> C.CDLL:
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with __graft_entry__.build() "
                          "(python -m paper_2511_06672_amd.build)")
    # The library links the system HIP runtime while PyTorch carries its own; the GPU is
    # found by both only when PyTorch's runtime is initialised first.
    try:
        import torch
        if torch.cuda.is_available():
            torch.cuda.init()
    except ImportError:
        pass
    lib = C.CDLL(path)
    P, I32, I64, D, SZ = C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_size_t
    sig = {
        "gcamps_workspace_bytes": [C.POINTER(Config), C.POINTER(SZ)],
        "gcamps_init": [C.POINTER(Config), P, SZ, P, C.POINTER(P)],
        "gcamps_destroy": [P],
        "gcamps_apply_clifford": [P, I32, C.POINTER(CWord)],
        "gcamps_apply_clifford_layer": [P, C.POINTER(I32), C.POINTER(CWord), I32],
        "gcamps_apply_phase_rotation": [P, I32, C.POINTER(D)],
        "gcamps_apply_gate": [P, I32, I32, C.POINTER(D)],
        "gcamps_candset_create": [I32, C.POINTER(CWord), I32, C.POINTER(P)],
        "gcamps_candset_destroy": [P],
        "gcamps_set_candset": [P, P],
        "gcamps_score_bond": [P, I32, C.POINTER(D), I64],
        "gcamps_factorize": [P, C.POINTER(D), I32, I32, I32, C.POINTER(D), C.POINTER(I32), C.POINTER(D),
                             C.POINTER(D), C.POINTER(D)],
        "gcamps_clifford_words": [I32, I32, C.POINTER(I32), I32, C.POINTER(C.c_uint8), I64, C.POINTER(I32),
                                  C.POINTER(I64)],
        "gcamps_disentangle": [P, P, C.POINTER(I32), C.POINTER(I32)],
        "gcamps_expectation": [P, C.POINTER(C.c_int8), C.POINTER(C.c_int8), I32, C.POINTER(D)],
        "gcamps_statevector": [P, P, P, SZ],
        "gcamps_statevector_static": [P, P],
        "gcamps_amplitude": [P, C.POINTER(C.c_int8), C.POINTER(D)],
        "gcamps_get_tableau": [P, C.POINTER(I32)],
        "gcamps_get_bond_dims": [P, C.POINTER(I32)],
        "gcamps_get_fidelity": [P, C.POINTER(D)],
        "gcamps_get_choice_log": [P, C.POINTER(I32), I64, C.POINTER(I64)],
        "gcamps_get_site": [P, I32, C.POINTER(D), I64, C.POINTER(I32)],
        "gcamps_get_stats": [P, C.POINTER(D)],
        "gcamps_get_kernel_stats": [P, C.POINTER(D)],
        "gcamps_batch_workspace_bytes": [C.POINTER(CBatchItem), I32, I32, C.POINTER(SZ)],
        "gcamps_batch_run": [C.POINTER(CBatchItem), I32, P, I32, P, SZ, C.POINTER(D)],
        "gcamps_grad_record": [C.POINTER(Config), C.POINTER(COp), I64, C.POINTER(I32), C.POINTER(D), I32, P, P,
                               SZ, P, C.POINTER(P), C.POINTER(D)],
        "gcamps_grad_loss": [P, C.POINTER(D), C.POINTER(D)],
        "gcamps_grad_gradient": [P, C.POINTER(D), C.POINTER(D), C.POINTER(D)],
        "gcamps_grad_stats": [P, C.POINTER(D)],
        "gcamps_grad_destroy": [P],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = I32
    lib.gcamps_last_error.argtypes = []
    lib.gcamps_last_error.restype = C.c_char_p
    return lib


_LIB: Optional[C.CDLL] = None


def lib() -> C.CDLL:
    global _LIB
    if _LIB is None:
        _LIB = load_library()
    return _LIB


def _check(code: int):
    if code != GCAMPS_OK:
        raise GcampsError(code, lib().gcamps_last_error().decode())


def _words(words) -> tuple:
    """Marshal workload Word objects (gens, weyl) into a CWord array (keeps buffers alive)."""
    arr = (CWord * len(words))()
    keep = []
    for i, w in enumerate(words):
        g = (C.c_uint8 * max(1, len(w.gens)))(*w.gens)
        keep.append(g)
        arr[i].len = len(w.gens)
        arr[i].gens = C.cast(g, C.POINTER(C.c_uint8))
        for j in range(4):
            arr[i].weyl[j] = int(w.weyl[j])
    return arr, keep


def make_config(d, n, chi_max, cutoff, score_prec=SCORE_FP64, near_tie=1e-4, tie_tol=1e-10,
                max_sweeps=2, auto_disentangle=True, max_candidates=512, max_gate_terms=0,
                criterion=0) -> Config:
    return Config(d, n, chi_max, cutoff, score_prec, near_tie, tie_tol, max_sweeps,
                  1 if auto_disentangle else 0, max_candidates, max_gate_terms, criterion)


def workspace_bytes(cfg: Config) -> int:
    b = C.c_size_t(0)
    _check(lib().gcamps_workspace_bytes(C.byref(cfg), C.byref(b)))
    return b.value


def clifford_words(d: int, kind: int = WORDS_DISENTANGLERS):
    """Exhaustive two-qudit Clifford set as Word objects (gcamps_clifford_words): the unique
    disentanglers (kind WORDS_DISENTANGLERS) or all of Sp(4, Z_d) (WORDS_ALL), identity first."""
    from .workload import Word
    cnt, tot = C.c_int32(0), C.c_int64(0)
    _check(lib().gcamps_clifford_words(d, kind, None, 0, None, 0, C.byref(cnt), C.byref(tot)))
    lens = (C.c_int32 * max(1, cnt.value))()
    gens = (C.c_uint8 * max(1, tot.value))()
    _check(lib().gcamps_clifford_words(d, kind, lens, cnt.value, gens, tot.value, C.byref(cnt), C.byref(tot)))
    out, o = [], 0
    for i in range(cnt.value):
        out.append(Word(tuple(int(g) for g in gens[o:o + lens[i]]), (0, 0, 0, 0)))
        o += lens[i]
    return out


class CandSet:
    def __init__(self, d: int, words):
        arr, keep = _words(words)
        h = C.c_void_p()
        _check(lib().gcamps_candset_create(d, arr, len(words), C.byref(h)))
        self.handle = h
        self.d = d
        self.count = len(words)

    def __del__(self):
        if getattr(self, "handle", None) and _LIB is not None:
            _LIB.gcamps_candset_destroy(self.handle)
            self.handle = None


class State:
    """One GCAMPS state psi = C|MPS> on a GPU (gcamps_ctx)."""

    def __init__(self, cfg: Config, device: str = "cuda:0", stream=None):
        import torch
        self.cfg = cfg
        self.d, self.n = cfg.d, cfg.n
        self.device = torch.device(device)
        nbytes = workspace_bytes(cfg)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        aligned = (base + 255) & ~255
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        _check(lib().gcamps_init(C.byref(cfg), C.c_void_p(aligned), nbytes,
                                 C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self.handle = h
        self._candset = None

    def close(self):
        if getattr(self, "handle", None):
            lib().gcamps_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- operations
    def apply_clifford(self, site: int, word):
        arr, keep = _words([word])
        _check(lib().gcamps_apply_clifford(self.handle, site, arr))

    def apply_clifford_layer(self, sites: Sequence[int], words):
        if not sites:
            return
        arr, keep = _words(words)
        s = (C.c_int32 * len(sites))(*sites)
        _check(lib().gcamps_apply_clifford_layer(self.handle, s, arr, len(sites)))

    def apply_phase_rotation(self, site: int, phi: Sequence[float]):
        a = (C.c_double * self.d)(*phi)
        _check(lib().gcamps_apply_phase_rotation(self.handle, site, a))

    def apply_gate(self, site: int, u):
        """General non-Clifford gate (gcamps_apply_gate): u is d^k x d^k (k = 1, 2) acting on
        sites site..site+k-1, site `site` the most significant digit."""
        u = np.ascontiguousarray(np.asarray(u, dtype=np.complex128))
        k = 1 if u.shape[0] == self.d else 2
        buf = (C.c_double * (2 * u.size))(*u.view(np.float64).reshape(-1))
        _check(lib().gcamps_apply_gate(self.handle, site, k, buf))

    def set_candset(self, cs: CandSet):
        self._candset = cs
        _check(lib().gcamps_set_candset(self.handle, cs.handle))

    def score_bond(self, bond: int) -> np.ndarray:
        """S2 of every candidate of the attached set at bond (bond, bond + 1), in the
        configured scoring mode (gcamps_score_bond); moves the orthogonality centre there."""
        cs = getattr(self, "_candset", None)
        if cs is None:
            raise GcampsError("score_bond needs a candidate set attached with set_candset")
        cnt = cs.count
        buf = (C.c_double * cnt)()
        _check(lib().gcamps_score_bond(self.handle, bond, buf, cnt))
        return np.frombuffer(buf, dtype=np.float64).copy()

    def factorize(self, m, factors: bool = False, reduce: bool = False):
        """The split's factorisation of a host matrix m (p x q complex) under this ctx's
        truncation rule (gcamps_factorize; ``reduce`` selects the rank-reduced path of the
        splits after a disentangler).  Returns (singular values in descending order, kept
        rank, discarded weight, L, R); L (p x kept) and R (kept x q) only with factors,
        else None."""
        m = np.ascontiguousarray(np.asarray(m, dtype=np.complex128))
        p, q = m.shape
        mn = min(p, q)
        sig = np.zeros(mn)
        kept, eps = C.c_int32(0), C.c_double(0.0)
        lbuf = np.zeros(p * mn, dtype=np.complex128) if factors else None
        rbuf = np.zeros(mn * q, dtype=np.complex128) if factors else None
        dp = lambda a: a.ctypes.data_as(C.POINTER(C.c_double)) if a is not None else None  # noqa: E731
        _check(lib().gcamps_factorize(self.handle, dp(m), p, q, FACTORIZE_REDUCE if reduce else 0, dp(sig),
                                      C.byref(kept), C.byref(eps), dp(lbuf), dp(rbuf)))
        k = kept.value
        L = lbuf[:p * k].reshape(p, k) if factors else None
        R = rbuf[:k * q].reshape(k, q) if factors else None
        return sig, k, eps.value, L, R

    def disentangle(self, cs: Optional[CandSet] = None):
        sw, ch = C.c_int32(0), C.c_int32(0)
        _check(lib().gcamps_disentangle(self.handle, cs.handle if cs else None, C.byref(sw),
                                        C.byref(ch)))
        return sw.value, ch.value

    def expectation(self, x, z, p: int = 0) -> complex:
        xa = (C.c_int8 * self.n)(*[int(v) for v in x])
        za = (C.c_int8 * self.n)(*[int(v) for v in z])
        out = (C.c_double * 2)()
        _check(lib().gcamps_expectation(self.handle, xa, za, p, out))
        return complex(out[0], out[1])

    def statevector(self) -> np.ndarray:
        import torch
        D = self.d ** self.n
        out = torch.empty(2 * D, dtype=torch.float64, device=self.device)
        scratch = torch.empty(6 * D, dtype=torch.float64, device=self.device)
        _check(lib().gcamps_statevector(self.handle, C.c_void_p(out.data_ptr()),
                                        C.c_void_p(scratch.data_ptr()), scratch.numel() * 8))
        v = out.cpu().numpy()
        return v[0::2] + 1j * v[1::2]

    def statevector_static(self) -> np.ndarray:
        """gcamps_statevector_static: the dense state with the library's static scratch."""
        import torch
        D = self.d ** self.n
        out = torch.empty(2 * D, dtype=torch.float64, device=self.device)
        _check(lib().gcamps_statevector_static(self.handle, C.c_void_p(out.data_ptr())))
        v = out.cpu().numpy()
        return v[0::2] + 1j * v[1::2]

    def amplitude(self, digits) -> complex:
        a = (C.c_int8 * self.n)(*[int(v) for v in digits])
        out = (C.c_double * 2)()
        _check(lib().gcamps_amplitude(self.handle, a, out))
        return complex(out[0], out[1])

    # ---------------------------------------------------------------- getters
    def tableau(self) -> np.ndarray:
        n = self.n
        buf = (C.c_int32 * (2 * n * (2 * n + 1)))()
        _check(lib().gcamps_get_tableau(self.handle, buf))
        return np.frombuffer(buf, dtype=np.int32).reshape(2 * n, 2 * n + 1).astype(np.int64)

    def bond_dims(self) -> List[int]:
        buf = (C.c_int32 * (self.n - 1))()
        _check(lib().gcamps_get_bond_dims(self.handle, buf))
        return list(buf)

    def fidelity(self) -> float:
        f = C.c_double(0)
        _check(lib().gcamps_get_fidelity(self.handle, C.byref(f)))
        return f.value

    def choice_log(self) -> np.ndarray:
        ln = C.c_int64(0)
        _check(lib().gcamps_get_choice_log(self.handle, None, 0, C.byref(ln)))
        buf = (C.c_int32 * (4 * max(1, ln.value)))()
        _check(lib().gcamps_get_choice_log(self.handle, buf, ln.value, C.byref(ln)))
        return np.frombuffer(buf, dtype=np.int32)[:4 * ln.value].reshape(-1, 4).copy()

    def site(self, i: int) -> np.ndarray:
        dims = (C.c_int32 * 3)()
        _check(lib().gcamps_get_site(self.handle, i, None, 0, dims))
        cnt = dims[0] * dims[1] * dims[2]
        buf = (C.c_double * (2 * cnt))()
        _check(lib().gcamps_get_site(self.handle, i, buf, cnt, dims))
        v = np.frombuffer(buf, dtype=np.float64)
        return (v[0::2] + 1j * v[1::2]).reshape(dims[0], dims[1], dims[2])

    def kernel_stats(self) -> dict:
        """Compression and MPO counters (gcamps_get_kernel_stats)."""
        out = (C.c_double * 8)()
        _check(lib().gcamps_get_kernel_stats(self.handle, out))
        keys = ["factorisations", "factor_svd_flops", "factor_ms", "mpo_launches", "mpo_bytes", "mpo_ms",
                "reduced", "reduced_basis_frac"]
        return dict(zip(keys, list(out)))

    def stats(self) -> dict:
        out = (C.c_double * 16)()
        _check(lib().gcamps_get_stats(self.handle, out))
        keys = ["gates", "bonds_scored", "rescored", "degenerate_cuts", "score_flops",
                "factor_flops", "score_ms", "host_ms", "rescore_flops", "rescore_ms",
                "score_launches", "tiled_launches", "tiled_ms", "tiled_flops", "centre_splits", "tiled_bytes"]
        return dict(zip(keys, list(out)))


def run_circuit(state: State, circuit, phases_override=None):
    """Apply a workload circuit layer by layer (bricks as one layer launch, then phases, then
    general gates)."""
    for layer in circuit.layers:
        if layer.bricks:
            state.apply_clifford_layer([b.site for b in layer.bricks], [b.word for b in layer.bricks])
        for ph in layer.phases:
            phi = ph.phi
            if phases_override is not None and ph.param >= 0:
                phi = phases_override[ph.param]
            state.apply_phase_rotation(ph.site, phi)
        for gg in layer.gates:
            D = state.d ** gg.k
            state.apply_gate(gg.site, np.array(gg.u, dtype=np.complex128).reshape(D, D))
    return state


def _circuit_ops(circuit, keep: list, phases_override=None):
    """Marshal a workload Circuit into a gcamps_op array (buffers kept alive in `keep`)."""
    ops = []
    params = []
    for layer in circuit.layers:
        if layer.gates:
            raise GcampsError(-2, "batched circuits carry Clifford layers and phase gates only; "
                                  "apply general gates through State.apply_gate")
        if layer.bricks:
            arr, kw = _words([b.word for b in layer.bricks])
            sites = (C.c_int32 * len(layer.bricks))(*[b.site for b in layer.bricks])
            keep.extend([arr, kw, sites])
            ops.append((OP_CLIFFORD_LAYER, len(layer.bricks), sites, arr, None))
            params.append(-1)
        for ph in layer.phases:
            phi = ph.phi
            if phases_override is not None and ph.param >= 0:
                phi = phases_override[ph.param]
            site = (C.c_int32 * 1)(ph.site)
            a = (C.c_double * circuit.d)(*phi)
            keep.extend([site, a])
            ops.append((OP_PHASE, 1, site, None, a))
            params.append(ph.param)
    keep.append(params)
    out = (COp * max(1, len(ops)))()
    for i, (kind, cnt, sites, words, phi) in enumerate(ops):
        out[i].kind = kind
        out[i].count = cnt
        out[i].sites = C.cast(sites, C.POINTER(C.c_int32))
        out[i].words = C.cast(words, C.POINTER(CWord)) if words is not None else None
        out[i].phi = C.cast(phi, C.POINTER(C.c_double)) if phi is not None else None
    keep.append(out)
    return out, len(ops)


def batch_run(circuits, cfgs, candset: Optional[CandSet] = None, lanes: int = 4,
              device: str = "cuda:0"):
    """gcamps_batch_run over workload Circuits with per-circuit Configs.

    Returns (results, stats): one dict per circuit (status, fidelity, bond_dims,
    z_expect, choices) and the batch statistics.
    """
    import torch
    assert len(circuits) == len(cfgs) and circuits
    keep: list = []
    count = len(circuits)
    items = (CBatchItem * count)()
    outs = []
    for i, (c, cfg) in enumerate(zip(circuits, cfgs)):
        ops, nops = _circuit_ops(c, keep)
        status = (C.c_int32 * 1)(-99)
        fid = (C.c_double * 1)()
        bonds = (C.c_int32 * (c.n - 1))()
        zexp = (C.c_double * (2 * c.n))()
        cap = max(1, c.n_phase_gates * max(1, cfg.max_sweeps) * (c.n - 1))
        ch = (C.c_int32 * (4 * cap))()
        chlen = (C.c_int64 * 1)()
        keep.extend([status, fid, bonds, zexp, ch, chlen])
        it = items[i]
        it.cfg = cfg
        it.ops = ops
        it.n_ops = nops
        it.status = C.cast(status, C.POINTER(C.c_int32))
        it.fidelity = C.cast(fid, C.POINTER(C.c_double))
        it.bond_dims = C.cast(bonds, C.POINTER(C.c_int32))
        it.z_expect = C.cast(zexp, C.POINTER(C.c_double))
        it.choices = C.cast(ch, C.POINTER(C.c_int32))
        it.choices_cap = cap
        it.choices_len = C.cast(chlen, C.POINTER(C.c_int64))
        outs.append((status, fid, bonds, zexp, ch, chlen, c.n))
    nbytes = C.c_size_t(0)
    _check(lib().gcamps_batch_workspace_bytes(items, count, lanes, C.byref(nbytes)))
    dev = torch.device(device)
    with torch.cuda.device(dev):
        ws = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=dev)
        aligned = (ws.data_ptr() + 255) & ~255
        torch.cuda.synchronize(dev)
        st = (C.c_double * 16)()
        rc = lib().gcamps_batch_run(items, count, candset.handle if candset else None, lanes,
                                    C.c_void_p(aligned), nbytes.value, st)
    results = []
    for status, fid, bonds, zexp, ch, chlen, n in outs:
        z = np.frombuffer(zexp, dtype=np.float64)
        ln = min(chlen[0], len(ch) // 4)
        results.append({"status": status[0], "fidelity": fid[0], "bond_dims": list(bonds),
                        "z_expect": z[0::2] + 1j * z[1::2],
                        "choices": np.frombuffer(ch, dtype=np.int32)[:4 * ln].reshape(-1, 4).copy(),
                        "choices_len": chlen[0]})
    del ws
    _check(rc)
    keys = ["circuits", "gates", "wall_ms", "busy_ms", "lanes", "score_ms", "bonds", "tiled_launches",
            "tiled_ms", "tiled_flops"]
    return results, dict(zip(keys, list(st)))


class Gradient:
    """Loss Re sum_j <Z_j> of a parametrised circuit and its gradient (gcamps_grad_*).

    Parameter block b of the circuit (PhaseGate.param == b) uses theta[(d-1)b : (d-1)(b+1)]
    as (phi_1, ..., phi_{d-1}); decisions are recorded at theta0 and frozen afterwards.
    """

    def __init__(self, cfg: Config, circuit, candset: Optional[CandSet], theta0, arena_bytes: Optional[int] = None,
                 device: str = "cuda:0", stream=None):
        import torch
        self.cfg = cfg
        self.d = cfg.d
        self._keep: list = []
        self.ops, self.n_ops = _circuit_ops(circuit, self._keep)
        params = self._keep[-2]
        self.op_param = (C.c_int32 * max(1, len(params)))(*params)
        self.n_theta = len(theta0)
        ctx_bytes = (workspace_bytes(cfg) + 255) & ~255
        if arena_bytes is None:
            slot = (cfg.chi_max * cfg.d) ** 2 * cfg.d * 16
            arena_bytes = min(24 << 30, 96 * (cfg.n + 16) * slot)
        self.device = torch.device(device)
        self.workspace = torch.empty(ctx_bytes + arena_bytes + 256, dtype=torch.uint8, device=self.device)
        aligned = (self.workspace.data_ptr() + 255) & ~255
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        th = (C.c_double * max(1, self.n_theta))(*[float(x) for x in theta0])
        h = C.c_void_p()
        loss = C.c_double(0)
        self._candset = candset
        _check(lib().gcamps_grad_record(C.byref(cfg), self.ops, self.n_ops, self.op_param, th, self.n_theta,
                                        candset.handle if candset else None, C.c_void_p(aligned),
                                        ctx_bytes + arena_bytes, C.c_void_p(self.stream.cuda_stream),
                                        C.byref(h), C.byref(loss)))
        self.handle = h
        self.loss0 = loss.value

    def _theta(self, theta):
        assert len(theta) == self.n_theta
        return (C.c_double * max(1, self.n_theta))(*[float(x) for x in theta])

    def loss(self, theta) -> float:
        out = C.c_double(0)
        _check(lib().gcamps_grad_loss(self.handle, self._theta(theta), C.byref(out)))
        return out.value

    def gradient(self, theta):
        out = C.c_double(0)
        g = (C.c_double * max(1, self.n_theta))()
        _check(lib().gcamps_grad_gradient(self.handle, self._theta(theta), C.byref(out), g))
        return out.value, np.frombuffer(g, dtype=np.float64)[:self.n_theta].copy()

    def stats(self) -> dict:
        out = (C.c_double * 8)()
        _check(lib().gcamps_grad_stats(self.handle, out))
        keys = ["replay_ms", "reverse_ms", "arena_peak_bytes", "tape_steps", "gates", "record_ms",
                "factorisations", "choices"]
        return dict(zip(keys, list(out)))

    def close(self):
        if getattr(self, "handle", None):
            lib().gcamps_grad_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
