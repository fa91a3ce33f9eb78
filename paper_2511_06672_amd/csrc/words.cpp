// Compilation of two-qudit Clifford words (host side).
//
// A word acts on the ordered pair (a, b).  Its action on two-qudit Weyl operators
// tau^p X_a^{xa} Z_a^{za} X_b^{xb} Z_b^{zb} is tabulated once per word over all
// d^4 exponent vectors: conjugation maps (v, p) to (f(v), p + g(v)), so one
// table entry per v holds f(v) and g(v).  The per-generator rules are those of
// Table 1 extended to powers with exact tau-phases (§2.3):
//   F (= H_d):   (x, z, p) -> (-z, x, p - 2xz)
//   P (= S_d):   (x, z, p) -> (x, z + x, p + x(x-1))  (odd d),  p + x^2 (even d)
//   X^s Z^t:     (x, z, p) -> (x, z, p + 2(t x - s z))
//   SUM a->b:    x_b += x_a, z_a -= z_b
// The inverse table (U^dagger W U) is the inverse permutation with negated
// phase increments.  The dense d^2 x d^2 unitary is the ordered product of the
// §2.3 gate matrices.
#include <array>
#include <cmath>
#include <complex>
#include <unordered_set>

#include "internal.h"

namespace gc {

namespace {

struct W2 {
  int xa, za, xb, zb, p;
};

inline int md(int v, int m) {
  v %= m;
  return v < 0 ? v + m : v;
}

void apply_gen(int d, W2& w, int g) {
  auto F = [&](int& x, int& z) {
    int x0 = x, z0 = z;
    x = md(-z0, d);
    z = x0;
    w.p = md(w.p - 2 * x0 * z0, 2 * d);
  };
  auto P = [&](int& x, int& z) {
    z = md(z + x, d);
    w.p = md(w.p + ((d % 2) ? x * (x - 1) : x * x), 2 * d);
  };
  switch (g) {
    case 0: F(w.xa, w.za); break;
    case 1: F(w.xb, w.zb); break;
    case 2: P(w.xa, w.za); break;
    case 3: P(w.xb, w.zb); break;
    case 4:
      w.xb = md(w.xb + w.xa, d);
      w.za = md(w.za - w.zb, d);
      break;
    case 5:
      w.xb = md(w.xb - w.xa, d);
      w.za = md(w.za + w.zb, d);
      break;
    default: throw Error{GCAMPS_EINVAL, "generator code out of range"};
  }
}

using C = std::complex<double>;

std::vector<C> matmul(const std::vector<C>& a, const std::vector<C>& b, int D) {
  std::vector<C> c(D * D, 0.0);
  for (int i = 0; i < D; ++i)
    for (int k = 0; k < D; ++k)
      for (int j = 0; j < D; ++j) c[i * D + j] += a[i * D + k] * b[k * D + j];
  return c;
}

// single-qudit matrices
std::vector<C> mat_F(int d) {
  std::vector<C> m(d * d);
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j) m[j * d + i] = std::polar(1.0 / std::sqrt((double)d), 2 * M_PI * i * j / d);
  return m;
}
std::vector<C> mat_P(int d) {
  std::vector<C> m(d * d, 0.0);
  for (int j = 0; j < d; ++j) {
    double ang = (d % 2) ? 2 * M_PI * (j * (j - 1) / 2) / d : M_PI * j * j / d;
    m[j * d + j] = std::polar(1.0, ang);
  }
  return m;
}
std::vector<C> mat_XZ(int d, int x, int z) {  // X^x Z^z: |j> -> omega^{zj} |j + x>
  std::vector<C> m(d * d, 0.0);
  for (int j = 0; j < d; ++j) m[md(j + x, d) * d + j] = std::polar(1.0, 2 * M_PI * z * j / d);
  return m;
}
std::vector<C> kron(const std::vector<C>& a, const std::vector<C>& b, int d) {
  std::vector<C> m(d * d * d * d);
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j)
      for (int k = 0; k < d; ++k)
        for (int l = 0; l < d; ++l) m[(i * d + k) * d * d + (j * d + l)] = a[i * d + j] * b[k * d + l];
  return m;
}
std::vector<C> eye(int D) {
  std::vector<C> m(D * D, 0.0);
  for (int i = 0; i < D; ++i) m[i * D + i] = 1.0;
  return m;
}
std::vector<C> gen_matrix(int d, int g) {
  int D = d * d;
  auto I = eye(d);
  switch (g) {
    case 0: return kron(mat_F(d), I, d);
    case 1: return kron(I, mat_F(d), d);
    case 2: return kron(mat_P(d), I, d);
    case 3: return kron(I, mat_P(d), d);
    case 4:
    case 5: {
      std::vector<C> m(D * D, 0.0);
      for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) {
          int out = (g == 4) ? md(i + j, d) : md(j - i, d);
          m[(i * d + out) * D + (i * d + j)] = 1.0;
        }
      return m;
    }
  }
  throw Error{GCAMPS_EINVAL, "generator code out of range"};
}

}  // namespace

CompiledWord compile_word(int d, const gcamps_word& w) {
  GC_CHECK(w.len >= 0 && (w.len == 0 || w.gens != nullptr), GCAMPS_EINVAL, "word: bad generator list");
  for (int i = 0; i < w.len; ++i) GC_CHECK(w.gens[i] < 6, GCAMPS_EINVAL, "word: generator code out of range");
  for (int i = 0; i < 4; ++i)
    GC_CHECK(w.weyl[i] >= 0 && w.weyl[i] < d, GCAMPS_EINVAL, "word: Weyl exponent out of range");
  const int D4 = d * d * d * d;
  CompiledWord cw;
  cw.fwd.assign(D4, 0);
  cw.inv.assign(D4, 0);
  for (int v = 0; v < D4; ++v) {
    W2 s{v / (d * d * d), (v / (d * d)) % d, (v / d) % d, v % d, 0};
    for (int i = 0; i < w.len; ++i) apply_gen(d, s, w.gens[i]);
    // Weyl shift X^w0 Z^w1 on a, X^w2 Z^w3 on b, applied last
    s.p = md(s.p + 2 * (w.weyl[1] * s.xa - w.weyl[0] * s.za), 2 * d);
    s.p = md(s.p + 2 * (w.weyl[3] * s.xb - w.weyl[2] * s.zb), 2 * d);
    uint32_t img = ((s.xa * d + s.za) * d + s.xb) * d + s.zb;
    cw.fwd[v] = img | ((uint32_t)s.p << 16);
    cw.inv[img] = (uint32_t)v | ((uint32_t)md(-s.p, 2 * d) << 16);
  }
  const int D = d * d;
  std::vector<C> u = eye(D);
  for (int i = 0; i < w.len; ++i) u = matmul(gen_matrix(d, w.gens[i]), u, D);
  u = matmul(kron(mat_XZ(d, w.weyl[0], w.weyl[1]), mat_XZ(d, w.weyl[2], w.weyl[3]), d), u, D);
  cw.mat.resize(D * D);
  for (int i = 0; i < D * D; ++i) cw.mat[i] = z64{u[i].real(), u[i].imag()};
  return cw;
}

// ----------------------------------------------------------------- exhaustive word sets
// Up to Weyl shifts and phases a two-qudit Clifford is the 4x4 matrix over Z_d of its
// conjugation action on the exponents (x_a, z_a, x_b, z_b) (the phase-free part of the rules
// above); S_{Q2 Q1} = S_{Q2} S_{Q1}.  Single-qudit Cliffords L applied after Q leave the
// entanglement of Q|psi> unchanged (§3.1), so the disentanglers are the classes {L Q}.  These
// classes are permuted by right multiplication with the generators (S -> S S_g: g applied
// before Q), so a breadth-first search over classes from the identity, each class keyed by
// its smallest member L S (base-d number of the entries, row by row), visits every class once
// and labels it with a shortest word.  The whole group is enumerated the same way with the
// matrix itself as the key.
namespace {

using Sym = std::array<uint8_t, 16>;  // row-major 4 x 4 over Z_d

Sym sym_identity() {
  Sym s{};
  for (int i = 0; i < 4; ++i) s[i * 5] = 1;
  return s;
}

Sym sym_of_generator(int d, int g) {
  Sym s{};
  for (int c = 0; c < 4; ++c) {
    W2 w{c == 0, c == 1, c == 2, c == 3, 0};
    apply_gen(d, w, g);
    s[0 * 4 + c] = (uint8_t)w.xa;
    s[1 * 4 + c] = (uint8_t)w.za;
    s[2 * 4 + c] = (uint8_t)w.xb;
    s[3 * 4 + c] = (uint8_t)w.zb;
  }
  return s;
}

Sym sym_mul(int d, const Sym& a, const Sym& b) {
  Sym c{};
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      int acc = 0;
      for (int k = 0; k < 4; ++k) acc += a[i * 4 + k] * b[k * 4 + j];
      c[i * 4 + j] = (uint8_t)(acc % d);
    }
  return c;
}

uint64_t sym_code(int d, const Sym& s) {
  uint64_t v = 0;
  for (int i = 0; i < 16; ++i) v = v * (uint64_t)d + s[i];
  return v;
}

}  // namespace

std::vector<std::vector<uint8_t>> clifford_word_set(int d, int kind) {
  GC_CHECK(d == 2 || d == 3, GCAMPS_EUNSUPPORTED, "exhaustive Clifford sets are built for d = 2 and 3");
  GC_CHECK(kind == GCAMPS_WORDS_DISENTANGLERS || kind == GCAMPS_WORDS_ALL, GCAMPS_EINVAL, "unknown word-set kind");
  Sym gen[6];
  for (int g = 0; g < 6; ++g) gen[g] = sym_of_generator(d, g);
  // single-qudit Cliffords: the group generated by F and P on either site
  std::vector<Sym> local{sym_identity()};
  {
    std::unordered_set<uint64_t> seen{sym_code(d, local[0])};
    for (size_t i = 0; i < local.size(); ++i)
      for (int g = 0; g < 4; ++g) {
        const Sym t = sym_mul(d, gen[g], local[i]);
        if (seen.insert(sym_code(d, t)).second) local.push_back(t);
      }
  }
  auto key = [&](const Sym& s) {
    if (kind == GCAMPS_WORDS_ALL) return sym_code(d, s);
    uint64_t best = UINT64_MAX;
    for (const Sym& l : local) best = std::min(best, sym_code(d, sym_mul(d, l, s)));
    return best;
  };
  std::vector<std::vector<uint8_t>> words{{}};
  std::vector<Sym> reps{sym_identity()};
  std::unordered_set<uint64_t> seen{key(reps[0])};
  for (size_t i = 0; i < reps.size(); ++i)
    for (int g = 0; g < 6; ++g) {
      const Sym t = sym_mul(d, reps[i], gen[g]);
      if (seen.insert(key(t)).second) {
        std::vector<uint8_t> w;
        w.reserve(words[i].size() + 1);
        w.push_back((uint8_t)g);
        w.insert(w.end(), words[i].begin(), words[i].end());
        words.push_back(std::move(w));
        reps.push_back(t);
      }
    }
  return words;
}

}  // namespace gc
