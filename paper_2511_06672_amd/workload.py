"""Seeded synthetic workloads: T-doped brickwork Clifford circuits and candidate sets.

This module produces *data only* (gate lists, angles, candidate words).  It holds
none of the simulation method's arithmetic and is the one module shared by the
GPU path, the tests and the benchmark harness.

Random numbers come from SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014):

    state += 0x9E3779B97F4A7C15
    z = state
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9
    z = (z ^ (z >> 27)) * 0x94D049BB133111EB
    out = z ^ (z >> 31)                        (all mod 2**64)

Integers below k are drawn as ``out % k`` (the bias is below 2**-58 for the
k <= 64 used here); reals in [0, 1) as ``(out >> 11) * 2**-53``.  Independent
streams for one workload are seeded with ``seed ^ (stream_id << 32)``.

Workload shape (the benchmark circuits of the paper's results section, a random
Clifford layer followed by non-Clifford phase gates, in brickwork form):

* layer ``L`` holds two-qudit Clifford bricks on pairs (0,1),(2,3),... when L is
  even and (1,2),(3,4),... when L is odd (open chain);
* every brick is a word of ``ngens`` generators drawn uniformly from
  ``{F_a, F_b, P_a, P_b, SUM_a->b, SUM^-1_a->b}`` (codes 0..5, ``gens[0]``
  applied first) followed by a Weyl shift ``X^w0 Z^w1`` on the first qudit and
  ``X^w2 Z^w3`` on the second, each exponent uniform in Z_d;
* the layer's diagonal phase gates act after its bricks, in draw order.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Sequence, Tuple

MASK64 = (1 << 64) - 1

# generator codes of a two-qudit Clifford word
GEN_F_A, GEN_F_B, GEN_P_A, GEN_P_B, GEN_SUM, GEN_SUM_INV = range(6)

# stream ids
STREAM_CIRCUIT = 1
STREAM_PHASE_POS = 2
STREAM_CANDIDATES = 3
STREAM_THETA = 4
STREAM_BATCH = 5
STREAM_GATES = 6


class SplitMix64:
    """SplitMix64 generator (see the module docstring for the definition)."""

    def __init__(self, seed: int):
        self.state = seed & MASK64

    def next_u64(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        return z ^ (z >> 31)

    def below(self, k: int) -> int:
        return self.next_u64() % k

    def uniform(self) -> float:
        return (self.next_u64() >> 11) * (1.0 / (1 << 53))


def substream(seed: int, stream_id: int) -> SplitMix64:
    return SplitMix64(seed ^ (stream_id << 32))


@dataclass
class Word:
    """A two-qudit Clifford word: generator codes then a Weyl shift."""
    gens: Tuple[int, ...]
    weyl: Tuple[int, int, int, int]

    def is_identity(self) -> bool:
        return len(self.gens) == 0 and not any(self.weyl)


IDENTITY_WORD = Word((), (0, 0, 0, 0))


@dataclass
class Brick:
    site: int          # acts on (site, site + 1)
    word: Word


@dataclass
class PhaseGate:
    site: int
    phi: Tuple[float, ...]   # diag(exp(i phi_0), ..., exp(i phi_{d-1}))
    param: int = -1          # index of the parameter pair for trainable gates, else -1


@dataclass
class GeneralGate:
    site: int                  # acts on sites site .. site + k - 1 (site the most significant digit)
    k: int
    u: Tuple[complex, ...]     # the d^k x d^k unitary, row-major


@dataclass
class Layer:
    bricks: List[Brick] = field(default_factory=list)
    phases: List[PhaseGate] = field(default_factory=list)
    gates: List[GeneralGate] = field(default_factory=list)   # applied after the phases


@dataclass
class Circuit:
    d: int
    n: int
    layers: List[Layer]

    @property
    def n_phase_gates(self) -> int:
        return sum(len(L.phases) for L in self.layers)

    @property
    def n_general_gates(self) -> int:
        return sum(len(L.gates) for L in self.layers)


def t_gate_phases(d: int) -> Tuple[float, ...]:
    """Angles of the non-Clifford T gate used by the workloads.

    d = 2: diag(1, e^{i pi/4}).  d = 3: diag(1, e^{2 pi i/9}, e^{-2 pi i/9}), the
    qutrit T gate whose cube is Z (the qutrit matrix printed in §2.3.2 does not have
    that property and is taken to be garbled).
    """
    if d == 2:
        return (0.0, math.pi / 4)
    if d == 3:
        return (0.0, 2 * math.pi / 9, -2 * math.pi / 9)
    raise ValueError("T gate defined for d in {2, 3}")


def random_word(rng: SplitMix64, d: int, ngens: int = 30) -> Word:
    gens = tuple(rng.below(6) for _ in range(ngens))
    weyl = tuple(rng.below(d) for _ in range(4))
    return Word(gens, weyl)  # type: ignore[arg-type]


def brick_sites(n: int, layer: int) -> List[int]:
    start = layer % 2
    return list(range(start, n - 1, 2))


def brickwork_circuit(d: int, n: int, layers: int, n_phase: int, seed: int,
                      phases: Sequence[float] | None = None,
                      one_per_layer: bool | None = None,
                      parametrised: bool = False,
                      ngens: int = 30) -> Circuit:
    """Seeded T-doped brickwork circuit.

    Phase-gate positions: when ``one_per_layer`` (default: n_phase == layers) each
    layer gets one gate at a uniform site; otherwise every gate draws (layer, site)
    uniformly and several may share a layer.  With ``parametrised`` the gates are
    diag(1, e^{i t1}, ..., e^{i t_{d-1}}) with t ~ U[0, 2 pi) from the theta stream
    and carry their parameter index.
    """
    if one_per_layer is None:
        one_per_layer = (n_phase == layers)
    rc = substream(seed, STREAM_CIRCUIT)
    rp = substream(seed, STREAM_PHASE_POS)
    rt = substream(seed, STREAM_THETA)
    if phases is None and not parametrised:
        phases = t_gate_phases(d)
    out = [Layer() for _ in range(layers)]
    for L in range(layers):
        for s in brick_sites(n, L):
            out[L].bricks.append(Brick(s, random_word(rc, d, ngens)))
    for g in range(n_phase):
        if one_per_layer:
            L = g % layers
        else:
            L = rp.below(layers)
        site = rp.below(n)
        if parametrised:
            phi = (0.0,) + tuple(2 * math.pi * rt.uniform() for _ in range(d - 1))
            out[L].phases.append(PhaseGate(site, phi, g))
        else:
            out[L].phases.append(PhaseGate(site, tuple(phases)))
    return Circuit(d, n, out)


def paper_circuit(d: int, n: int, layers: int, seed: int, depth: int | None = None) -> Circuit:
    """The paper's benchmark circuit (Fig. 3 of §4): each layer is a random Clifford followed by
    one T gate on the first qudit.  The random Clifford is `depth` (default n) brickwork
    sublayers of random two-qudit words, a deep random Clifford circuit standing in for a draw
    from the whole n-qudit Clifford group; the T gate follows the layer's last sublayer."""
    depth = n if depth is None else depth
    rc = substream(seed, STREAM_CIRCUIT)
    out: List[Layer] = []
    for _ in range(layers):
        for s in range(depth):
            out.append(Layer([Brick(site, random_word(rc, d)) for site in brick_sites(n, s)]))
        out[-1].phases.append(PhaseGate(0, t_gate_phases(d)))
    return Circuit(d, n, out)


def haar_unitary(rng: SplitMix64, D: int) -> Tuple[complex, ...]:
    """Haar-random D x D unitary, row-major: the columns of a matrix of standard complex
    Gaussians (Box-Muller on the stream's uniforms, drawn row by row) orthonormalised by
    modified Gram-Schmidt, which is QR with a positive diagonal in R, so the result is Haar
    distributed (Mezzadri, "How to generate random matrices from the classical compact groups",
    2007).  Plain Python arithmetic, so every machine draws the same matrix."""
    z = [[0j] * D for _ in range(D)]
    for i in range(D):
        for j in range(D):
            u1 = 1.0 - rng.uniform()          # (0, 1]
            u2 = rng.uniform()
            rad = math.sqrt(-math.log(u1))    # |z|^2 ~ Exp(1): unit variance complex
            z[i][j] = complex(rad * math.cos(2 * math.pi * u2), rad * math.sin(2 * math.pi * u2))
    cols = [[z[i][j] for i in range(D)] for j in range(D)]
    for j in range(D):
        v = cols[j]
        for q in cols[:j]:
            ov = sum(a.conjugate() * b for a, b in zip(q, v))
            v = [b - ov * a for a, b in zip(q, v)]
        nrm = math.sqrt(sum(abs(b) ** 2 for b in v))
        cols[j] = [b / nrm for b in v]
    return tuple(cols[j][i] for i in range(D) for j in range(D))


def general_circuit(d: int, n: int, layers: int, k: int, seed: int, ngens: int = 30) -> Circuit:
    """Brickwork Clifford layers (the word stream of ``brickwork_circuit``), each followed by one
    Haar-random k-qudit unitary (k = 1, 2) on sites (s, .., s + k - 1), s uniform in
    0 .. n - k: general non-diagonal non-Clifford gates, expanded on the d^(2k) Weyl operators."""
    rc = substream(seed, STREAM_CIRCUIT)
    rp = substream(seed, STREAM_PHASE_POS)
    ru = substream(seed, STREAM_GATES)
    out = [Layer() for _ in range(layers)]
    for L in range(layers):
        for s in brick_sites(n, L):
            out[L].bricks.append(Brick(s, random_word(rc, d, ngens)))
        site = rp.below(n - k + 1)
        out[L].gates.append(GeneralGate(site, k, haar_unitary(ru, d ** k)))
    return Circuit(d, n, out)


def candidate_words(d: int, count: int, seed: int, ngens: int = 30) -> List[Word]:
    """Candidate disentanglers: index 0 is the identity, the rest seeded random words."""
    rng = substream(seed, STREAM_CANDIDATES)
    words = [IDENTITY_WORD]
    for _ in range(count - 1):
        words.append(random_word(rng, d, ngens))
    return words


# ----------------------------------------------------------------------------------
# Named workloads.  Sizes follow the benchmark table; seeds are fixed here.
# ----------------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    circuit: Circuit
    candidates: List[Word]
    chi_max: int
    cutoff: float
    max_sweeps: int = 2
    # "listed": `candidates` is the set; "all_sp4": every two-qudit Clifford up to Weyl shifts
    # (720 for qubits); "exhaustive": the unique disentanglers (20 / 90); the last two are
    # enumerated by the caller (this module holds no Clifford arithmetic)
    candidate_set: str = "listed"


def workload(name: str, n: int | None = None, layers: int | None = None) -> Workload:
    """Named workloads.  ``n`` overrides the chain length (keeping the recipe); ``layers``
    overrides the layer count of the paper workloads (default N, the onset of the transition;
    the runs past it use up to 2N)."""
    if name == "exact_d3_n8":
        nn = 8 if n is None else n
        seed = 1000
        c = brickwork_circuit(3, nn, 20, 8, seed, one_per_layer=False)
        return Workload(name, c, candidate_words(3, 512, seed), chi_max=3 ** (nn // 2),
                        cutoff=0.0)
    if name == "headline_d3_n32":
        nn = 32 if n is None else n
        seed = 2000
        layers = 40 if n is None else max(8, (40 * nn) // 32)
        c = brickwork_circuit(3, nn, layers, layers, seed)
        return Workload(name, c, candidate_words(3, 512, seed), chi_max=256, cutoff=1e-10)
    if name == "grad_d3_n24":
        nn = 24 if n is None else n
        seed = 5000
        c = brickwork_circuit(3, nn, 2 * nn, 32, seed, one_per_layer=False,
                              parametrised=True)
        return Workload(name, c, candidate_words(3, 512, seed), chi_max=256, cutoff=1e-10)
    if name in ("paper_d3_n12", "paper_d2_n12"):
        # the paper's own workload: N = 12 qudits, N layers of (random Clifford, T on qudit 0),
        # no truncation beyond the rank floor; disentangled with the exhaustive set under the
        # bond-dimension criterion (the caller supplies the set: gcamps_clifford_words)
        dd = 3 if name == "paper_d3_n12" else 2
        nn = 12 if n is None else n
        seed = 6000 + dd
        c = paper_circuit(dd, nn, nn if layers is None else layers, seed)
        return Workload(name, c, [], chi_max=min(dd ** (nn // 2), 1024), cutoff=0.0, candidate_set="exhaustive")
    if name == "mixed_d2_n64":
        # mixed run, qubit part: one T = diag(1, e^{i pi/4}) per layer, chi_max 1024, cutoff
        # 1e-12, the 720 elements of Sp(4, Z_2) as candidates
        nn = 64 if n is None else n
        seed = 3001
        layers = 64 if n is None else nn
        c = brickwork_circuit(2, nn, layers, layers, seed)
        return Workload(name, c, [], chi_max=1024, cutoff=1e-12, candidate_set="all_sp4")
    if name == "mixed_d3_n48":
        # mixed run, qutrit part: 60 layers with one T each, chi_max 1024, cutoff 1e-12,
        # identity + 719 seeded random candidates
        nn = 48 if n is None else n
        seed = 3002
        layers = 60 if n is None else max(8, (60 * nn) // 48)
        c = brickwork_circuit(3, nn, layers, layers, seed)
        return Workload(name, c, candidate_words(3, 720, seed), chi_max=1024, cutoff=1e-12)
    if name == "general_d3_n24":
        # general gates, single-qutrit: 24 layers, a Haar-random 3x3 unitary after each (up to
        # 9 Weyl terms, MPO bond <= 9), chi_max 64, cutoff 1e-10, identity + 511 random candidates
        nn = 24 if n is None else n
        seed = 7003
        c = general_circuit(3, nn, nn, 1, seed)
        return Workload(name, c, candidate_words(3, 512, seed), chi_max=64, cutoff=1e-10)
    if name == "general_d2_n24":
        # general gates, two-qubit: 24 layers, a Haar-random 4x4 unitary on two neighbouring
        # qubits after each (up to 16 Weyl terms), chi_max 64, cutoff 1e-10, the 720 elements of
        # Sp(4, Z_2) as candidates
        nn = 24 if n is None else n
        seed = 7002
        c = general_circuit(2, nn, nn, 2, seed)
        return Workload(name, c, [], chi_max=64, cutoff=1e-10, candidate_set="all_sp4")
    raise KeyError(name)


@dataclass
class BatchWorkload:
    name: str
    circuits: List[Circuit]
    candidates: List[Word]
    chi_max: int
    cutoff: float
    max_sweeps: int = 2

    @property
    def n_phase_gates(self) -> int:
        return sum(c.n_phase_gates for c in self.circuits)


def batch_workload(count: int = 256, seed: int = 3000, n_range: Tuple[int, int] = (8, 48),
                   t_range: Tuple[int, int] = (4, 60), chi_max: int = 128, cutoff: float = 1e-10,
                   n_candidates: int = 512, name: str = "batch_d3") -> BatchWorkload:
    """Independent qutrit circuits of uneven size.

    Circuit i draws n_i ~ U{n_lo..n_hi} and T_i ~ U{t_lo..t_hi} from the batch stream
    of ``seed``, has 2 n_i brickwork layers and T_i T gates at uniform (layer, site),
    and is generated with seed ``seed + 1 + i``.  One candidate set (seed ``seed``) is
    shared by every circuit.
    """
    rng = substream(seed, STREAM_BATCH)
    circuits = []
    for i in range(count):
        n = n_range[0] + rng.below(n_range[1] - n_range[0] + 1)
        t = t_range[0] + rng.below(t_range[1] - t_range[0] + 1)
        circuits.append(brickwork_circuit(3, n, 2 * n, t, seed + 1 + i, one_per_layer=False))
    return BatchWorkload(name, circuits, candidate_words(3, n_candidates, seed), chi_max, cutoff)


def circuit_to_json(c: Circuit) -> dict:
    return {
        "d": c.d, "n": c.n,
        "layers": [
            {"bricks": [[b.site, list(b.word.gens), list(b.word.weyl)] for b in L.bricks],
             "phases": [[p.site, list(p.phi), p.param] for p in L.phases]}
            for L in c.layers
        ],
    }
