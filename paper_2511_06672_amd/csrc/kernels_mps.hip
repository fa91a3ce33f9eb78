// MPS-side kernels of the GCAMPS bottom loop (§2.4, §3):
//  * block-MPO application of sum_b c_b P^b on the support of the commuted Weyl operator,
//  * Theta <- Q Theta for the selected disentangler,
//  * candidate scoring by the Renyi-2 purity of the two-site cut (FP64, FP32 or split BF16), as a
//    fused one-workgroup-per-candidate kernel for small cuts; for large cuts the rotated
//    matrices of a chunk of candidates are written to HBM and Hermitian Gram tiles on MFMA
//    (128 x 128 FP32 and BF16 with direct-to-LDS loads, 64 x 64 FP64 for the re-score window)
//    give sum |rho|^2,
//  * FP64 selection (lowest index within tie_tol of the minimum) and the low-precision window,
//  * dense helpers for the validation state vector.
#include <algorithm>
#include <type_traits>
#include <cfloat>

#include "kernels.h"
#include "tune.h"

namespace gc {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

namespace {

inline unsigned blocks_for(size_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

// ===================================================================================== MPO
// (X^a Z^c A)[al, s, be] = omega^{c (s - a)} A[al, s - a, be]   (indices mod d)
__global__ void k_mpo_site(int kind, int d, int chil, int chir, int dx, int dz, MpoCoeff co,
                           const z64* __restrict__ in, z64* __restrict__ out) {
  size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  int ol = (kind == 1 || kind == 2) ? d * chil : chil;
  int orr = (kind == 0 || kind == 1) ? d * chir : chir;
  size_t total = (size_t)ol * d * orr;
  if (idx >= total) return;
  int col = (int)(idx % orr);
  int s = (int)((idx / orr) % d);
  int row = (int)(idx / ((size_t)orr * d));
  auto term = [&](int b, int al, int be) -> z64 {
    int a = (b * dx) % d, c = (b * dz) % d;
    int src = (s - a + d) % d;
    z64 v = in[((size_t)al * d + src) * chir + be];
    return cmul(co.w[(c * src) % d], v);
  };
  z64 v = {0.0, 0.0};
  if (kind == 3) {
    for (int b = 0; b < d; ++b) v = cadd(v, cmul(co.k[b], term(b, row, col)));
  } else if (kind == 0) {
    int b = col / chir, be = col % chir;
    v = cmul(co.k[b], term(b, row, be));
  } else if (kind == 2) {
    int b = row / chil, al = row % chil;
    v = term(b, al, col);
  } else {
    int bl = row / chil, al = row % chil, br = col / chir, be = col % chir;
    if (bl == br) v = term(bl, al, be);
  }
  out[idx] = v;
}

// Site tensor of the MPO sum_j c_j (x)_i X^{x_ji} Z^{z_ji} (bond J, block-diagonal in j):
//   kind 0 (left end):  out[al, s, (j, be)] = c_j (X^x_j Z^z_j A)[al, s, be]
//   kind 1 (interior):  out[(j, al), s, (j', be)] = delta_jj' (X^x_j Z^z_j A)[al, s, be]
//   kind 2 (right end): out[(j, al), s, be] = (X^x_j Z^z_j A)[al, s, be]
//   kind 3 (one site):  out[al, s, be] = sum_j c_j (X^x_j Z^z_j A)[al, s, be]
__global__ void k_mpo_sum_site(int kind, int d, int J, int chil, int chir, MpoTerms tm, const z64* __restrict__ in,
                               z64* __restrict__ out) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int ol = (kind == 1 || kind == 2) ? J * chil : chil;
  const int orr = (kind == 0 || kind == 1) ? J * chir : chir;
  const size_t total = (size_t)ol * d * orr;
  if (idx >= total) return;
  const int col = (int)(idx % orr);
  const int s = (int)((idx / orr) % d);
  const int row = (int)(idx / ((size_t)orr * d));
  auto term = [&](int j, int al, int be) -> z64 {
    const int a = tm.x[j], c = tm.z[j];
    const int src = (s - a + d) % d;
    const double ang = 2.0 * M_PI * (double)((c * src) % d) / (double)d;
    const z64 v = in[((size_t)al * d + src) * chir + be];
    return cmul(z64{cos(ang), sin(ang)}, v);
  };
  z64 v = {0.0, 0.0};
  if (kind == 3) {
    for (int j = 0; j < J; ++j) v = cadd(v, cmul(tm.coef[j], term(j, row, col)));
  } else if (kind == 0) {
    const int j = col / chir, be = col % chir;
    v = cmul(tm.coef[j], term(j, row, be));
  } else if (kind == 2) {
    const int j = row / chil, al = row % chil;
    v = term(j, al, col);
  } else {
    const int jl = row / chil, al = row % chil, jr = col / chir, be = col % chir;
    if (jl == jr) v = term(jl, al, be);
  }
  out[idx] = v;
}

// ===================================================================================== apply Q
__global__ void k_apply_q(int d, int chil, int chir, const DevStatus* __restrict__ st, const z64* __restrict__ qm,
                          z64* __restrict__ theta) {
  const int c = st->cstar;
  if (c == 0) return;
  size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)chil * chir) return;
  const int a = (int)(idx / chir), b = (int)(idx % chir);
  const int D2 = d * d;
  const z64* q = qm + (size_t)c * D2 * D2;
  z64 v[kMaxD * kMaxD];
  for (int x = 0; x < D2; ++x) v[x] = theta[((size_t)a * D2 + x) * chir + b];
  for (int y = 0; y < D2; ++y) {
    z64 acc = {0.0, 0.0};
    for (int x = 0; x < D2; ++x) acc = cadd(acc, cmul(q[y * D2 + x], v[x]));
    theta[((size_t)a * D2 + y) * chir + b] = acc;
  }
}

// out = Q_c Theta for an explicit candidate c (a copy when c == 0); Theta (chil, d, d, chir).
__global__ void k_rotate_copy(int d, int chil, int chir, int c, const z64* __restrict__ qm,
                              const z64* __restrict__ theta, z64* __restrict__ out) {
  size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)chil * chir) return;
  const int a = (int)(idx / chir), b = (int)(idx % chir);
  const int D2 = d * d;
  const z64* q = qm + (size_t)c * D2 * D2;
  z64 v[kMaxD * kMaxD];
  for (int x = 0; x < D2; ++x) v[x] = theta[((size_t)a * D2 + x) * chir + b];
  for (int y = 0; y < D2; ++y) {
    z64 acc = {0.0, 0.0};
    if (c == 0)
      acc = v[y];
    else
      for (int x = 0; x < D2; ++x) acc = cadd(acc, cmul(q[y * D2 + x], v[x]));
    out[((size_t)a * D2 + y) * chir + b] = acc;
  }
}

// ===================================================================================== scoring
// Element of M_c = reshape(Q_c Theta) at row (a, s1') and column (s2', b):
//   M[(a s1'), (s2' b)] = sum_{s1 s2} Q[(s1' s2'), (s1 s2)] Theta[a, s1, s2, b]
template <typename T>
__device__ __forceinline__ cx<T> melem(int d, int chir, const z64* __restrict__ theta, const cx<T>* q, int a,
                                       int s1p, int s2p, int b) {
  const int D2 = d * d;
  const cx<T>* qrow = q + (s1p * d + s2p) * D2;
  const z64* th = theta + (size_t)a * D2 * chir + b;
  cx<T> acc = {T(0), T(0)};
  for (int x = 0; x < D2; ++x) {
    z64 tv = th[(size_t)x * chir];
    cx<T> t = {T(tv.re), T(tv.im)};
    acc = cadd(acc, cmul(qrow[x], t));
  }
  return acc;
}

// Element (i, col) of the scored matrix N: N = M when chil*d <= d*chir (rows (a s1'), cols
// (s2' b)), else N = M^T (rows (s2' b), cols (a s1')).  ||N N^H||_F = ||M M^H||_F.
template <typename T>
__device__ __forceinline__ cx<T> nelem(int d, int chil, int chir, bool rows_first, const z64* __restrict__ theta,
                                       const cx<T>* q, int i, int col) {
  int a, s1p, s2p, b;
  if (rows_first) {
    a = i / d;
    s1p = i % d;
    s2p = col / chir;
    b = col % chir;
  } else {
    s2p = i / chir;
    b = i % chir;
    a = col / d;
    s1p = col % d;
  }
  return melem<T>(d, chir, theta, q, a, s1p, s2p, b);
}

constexpr int SMALL_M = kScoreSmallM;
constexpr int SMALL_KC = 32;
constexpr int SMALL_THREADS = 512;
constexpr int SMALL_PPT = (SMALL_M * (SMALL_M + 1) / 2 + SMALL_THREADS - 1) / SMALL_THREADS;

template <typename T>
__device__ __forceinline__ const cx<T>* qsel(const z64* q64, const c32* q32);
template <>
__device__ __forceinline__ const cx<double>* qsel<double>(const z64* q64, const c32*) {
  return q64;
}
template <>
__device__ __forceinline__ const cx<float>* qsel<float>(const z64*, const c32* q32) {
  return q32;
}

// Deterministic block sum of one double per thread (blockDim.x a power of two <= 1024).
__device__ double block_sum(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  double r = red[0];
  __syncthreads();
  return r;
}

template <typename T>
__global__ __launch_bounds__(SMALL_THREADS) void k_score_small(int d, int chil, int chir,
                                                               const z64* __restrict__ theta,
                                                               const z64* __restrict__ q64,
                                                               const c32* __restrict__ q32,
                                                               const int* __restrict__ list,
                                                               const int* __restrict__ nlimit,
                                                               double* __restrict__ s2) {
  const int slot = blockIdx.x;
  if (nlimit && slot >= *nlimit) return;
  const int c = list ? list[slot] : slot;
  const bool rows_first = chil * d <= d * chir;
  const int m = rows_first ? chil * d : d * chir;
  const int k = rows_first ? d * chir : chil * d;
  const int D4 = d * d * d * d;
  __shared__ cx<T> qs[kMaxD * kMaxD * kMaxD * kMaxD];
  __shared__ cx<T> chunk[SMALL_M * SMALL_KC];
  __shared__ double red[SMALL_THREADS];
  const int t = threadIdx.x;
  const cx<T>* qall = qsel<T>(q64, q32);
  for (int i = t; i < D4; i += SMALL_THREADS) qs[i] = qall[(size_t)c * D4 + i];
  const int npairs = m * (m + 1) / 2;
  int pi[SMALL_PPT], pj[SMALL_PPT];
  cx<T> acc[SMALL_PPT];
  for (int u = 0; u < SMALL_PPT; ++u) {
    int e = t + u * SMALL_THREADS;
    pi[u] = pj[u] = -1;
    acc[u] = {T(0), T(0)};
    if (e < npairs) {
      // e -> (i, j), i <= j, row-major over the upper triangle
      int i = 0, rem = e;
      while (rem >= m - i) {
        rem -= m - i;
        ++i;
      }
      pi[u] = i;
      pj[u] = i + rem;
    }
  }
  __syncthreads();
  for (int k0 = 0; k0 < k; k0 += SMALL_KC) {
    const int kc = (k - k0 < SMALL_KC) ? k - k0 : SMALL_KC;
    for (int e = t; e < m * SMALL_KC; e += SMALL_THREADS) {
      int i = e / SMALL_KC, kk = e % SMALL_KC;
      chunk[e] = (kk < kc) ? nelem<T>(d, chil, chir, rows_first, theta, qs, i, k0 + kk) : cx<T>{T(0), T(0)};
    }
    __syncthreads();
    for (int u = 0; u < SMALL_PPT; ++u) {
      if (pi[u] < 0) continue;
      const cx<T>* ri = chunk + pi[u] * SMALL_KC;
      const cx<T>* rj = chunk + pj[u] * SMALL_KC;
      cx<T> a = acc[u];
      for (int kk = 0; kk < kc; ++kk) {
        cx<T> x = ri[kk], y = rj[kk];
        a.re += x.re * y.re + x.im * y.im;
        a.im += x.im * y.re - x.re * y.im;
      }
      acc[u] = a;
    }
    __syncthreads();
  }
  double pur = 0.0, tr = 0.0;
  for (int u = 0; u < SMALL_PPT; ++u) {
    if (pi[u] < 0) continue;
    double a2 = (double)acc[u].re * acc[u].re + (double)acc[u].im * acc[u].im;
    pur += (pi[u] == pj[u]) ? a2 : 2.0 * a2;
    if (pi[u] == pj[u]) tr += (double)acc[u].re;
  }
  pur = block_sum(pur, red);
  tr = block_sum(tr, red);
  if (t == 0) s2[slot] = -log(pur / (tr * tr));
}

// ----------------------------------------------------------------------- tiled MFMA scoring
__device__ __forceinline__ d4 mfma_t(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mfma_t(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
template <typename T>
struct AccT;
template <>
struct AccT<double> {
  typedef d4 type;
};
template <>
struct AccT<float> {
  typedef f4 type;
};

__device__ __forceinline__ void tile_pair(int idx, int nt, int& I, int& J) {
  int i = 0, rem = idx;
  while (rem >= nt - i) {
    rem -= nt - i;
    ++i;
  }
  I = i;
  J = i + rem;
}

// Candidates per generator thread: for chunks of at least kGenMinChunk candidates the tuner's
// pick among kGenCpt per (precision, d, chi_l, chi_r) (kGenCands without tuning), else one.
// Lists whose length is only known on the device (the window re-score) take one too: they are
// usually short, and a few candidates need every block they can get.  The generated matrices
// are the same for every choice.
constexpr int kGenCands = 8, kGenMinChunk = 64;
constexpr int kGenCpt[] = {1, 2, 4, 8};

// Rotated two-site matrices N_c (m x k, row-major, leading dimension ldk >= k) for a chunk of
// candidates.  One thread per (a, b) loads Theta(a, :, :, b) once and writes the d^2 entries
// (Q_c Theta)(a, s1', s2', b) to their (row, col) positions: rows (a s1'), cols (s2' b) when
// chil*d <= d*chir, else transposed.  Columns k..ldk-1 of every row are written as zeros.  A
// thread serves cpt consecutive candidates of the chunk (blockIdx.y picks the group), so Theta
// is read once per group rather than once per candidate.
template <typename T, int DD>
__global__ __launch_bounds__(256) void k_gen_rotated(int d_rt, int chil, int chir, const z64* __restrict__ theta,
                                                     const cx<T>* __restrict__ qall, const int* __restrict__ list,
                                                     int c0, int cnt, const int* __restrict__ nlimit,
                                                     cx<T>* __restrict__ out, size_t stride, int ldk, int cpt) {
  // DD > 0: qudit dimension fixed at compile time (the d^2-vector stays in registers)
  const int d = DD > 0 ? DD : d_rt;
  constexpr int VMAX = DD > 0 ? DD * DD : kMaxD * kMaxD;
  const bool rows_first = chil * d <= d * chir;
  const int k = rows_first ? d * chir : chil * d;
  const int m = rows_first ? chil * d : d * chir;
  const int g0 = blockIdx.y * cpt;  // first candidate of this block's group
  if (g0 >= cnt || (nlimit && c0 + g0 >= *nlimit)) return;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool active = idx < (size_t)chil * chir;
  // rows_first: b fastest (contiguous columns s2'*chir + b); otherwise a fastest
  int a = 0, b = 0;
  if (active) {
    if (rows_first) {
      a = (int)(idx / chir);
      b = (int)(idx % chir);
    } else {
      b = (int)(idx / chil);
      a = (int)(idx % chil);
    }
  }
  const int D2 = d * d;
  cx<T> v[VMAX];
  if (active) {
    const z64* th = theta + (size_t)a * D2 * chir + b;
#pragma unroll
    for (int x = 0; x < VMAX; ++x) {
      if (x >= D2) break;
      const z64 tv = th[(size_t)x * chir];
      v[x] = cx<T>{T(tv.re), T(tv.im)};
    }
  }
  for (int u = 0; u < cpt; ++u) {
    const int ls = g0 + u;
    const int slot = c0 + ls;
    if (ls >= cnt || (nlimit && slot >= *nlimit)) break;  // uniform over the block
    const int c = list ? list[slot] : slot;
    cx<T>* o = out + (size_t)ls * stride;
    if (ldk > k) {
      const int pad = ldk - k;
      const size_t np = (size_t)m * pad, nth = (size_t)gridDim.x * blockDim.x;
      for (size_t e = idx; e < np; e += nth) o[(e / pad) * ldk + k + e % pad] = cx<T>{T(0), T(0)};
    }
    if (!active) continue;
    const cx<T>* q = qall + (size_t)c * D2 * D2;
    for (int y = 0; y < D2; ++y) {
      const int s1p = y / d, s2p = y - s1p * d;
      cx<T> acc = {T(0), T(0)};
#pragma unroll
      for (int x = 0; x < VMAX; ++x) {
        if (x >= D2) break;
        acc = cadd(acc, cmul(q[y * D2 + x], v[x]));
      }
      const size_t row = rows_first ? (size_t)a * d + s1p : (size_t)s2p * chir + b;
      const size_t col = rows_first ? (size_t)s2p * chir + b : (size_t)a * d + s1p;
      o[row * ldk + col] = acc;
    }
  }
}

// Purity tiles in FP64 (window re-score): for candidate slot `ls` of the chunk, tile (I, J),
// I <= J, of rho = N N^H over the k columns, on MFMA (16x16x4 FP64), four real products per
// complex product.  The NW waves form two rows of NW / 2: each owns BL x (2 BL / (NW / 2))
// 16x16 blocks of the TT x TT tile (TT = 32 * BL); instantiated with four waves, two workgroups
// per CU.  Operands are staged through registers: chunk c + 1 is fetched while chunk c is
// multiplied, then transposed into LDS (re and im planes, k-major).  The FP32 path uses
// k_gram_purity_dl below.  The epilogue writes sum |rho_tile|^2 (doubled off the diagonal) and
// the tile's trace to partial[slot][tile].
template <typename T, int BL, int NW>
__global__ __launch_bounds__(64 * NW, 2) void k_gram_purity(int m, int k, const cx<T>* __restrict__ nbase, size_t stride,
                                                     int c0, int cnt, const int* __restrict__ nlimit, int ntp,
                                                     double* __restrict__ partial) {
  typedef typename AccT<T>::type acc_t;
  constexpr int TT = 32 * BL, KC = 16, PAD = TT + 4;
  constexpr int NT = 64 * NW, WC = NW / 2;          // threads; waves along the columns (two rows)
  constexpr int BLR = BL, BLC = 2 * BL / WC;         // 16x16 blocks per wave: rows, columns
  // XCD-aware order: workgroup L runs on XCD L mod 8, so the ntp tiles of one candidate are
  // given consecutive slots of one XCD and share its L2 (candidates are padded to a multiple
  // of 8; the padding exits at once).
  const int L = blockIdx.x;
  const int xcd = L & 7, xslot = L >> 3;
  const int cg = xslot / ntp, tile = xslot - cg * ntp;
  const int ls = cg * 8 + xcd;
  const int slot = c0 + ls;
  if (ls >= cnt || (nlimit && slot >= *nlimit)) return;
  const cx<T>* N = nbase + (size_t)ls * stride;
  const int nt = (m + TT - 1) / TT;
  int I, J;
  tile_pair(tile, nt, I, J);
  // two LDS stages: chunk c + 1 is fetched into registers while chunk c is multiplied,
  // then stored into the other stage; one barrier per chunk
  __shared__ T As[2][2][KC][PAD];
  __shared__ T Bs[2][2][KC][PAD];
  __shared__ double red[NT];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wr = (w / WC) * (TT / 2), wc = (w % WC) * (TT / WC);
  // re and im accumulated directly (B holds -Im)
  acc_t accr[BLR][BLC], acci[BLR][BLC];
  for (int i = 0; i < BLR; ++i)
    for (int j = 0; j < BLC; ++j)
      for (int q = 0; q < 4; ++q) {
        accr[i][j][q] = T(0);
        acci[i][j][q] = T(0);
      }
  const int r0 = I * TT, q0 = J * TT;
  constexpr int U = TT * KC / NT;
  cx<T> pa[U], pb[U];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = t + NT * u;
      const int row = e / KC, kk = e % KC;
      const int col = k0 + kk;
      pa[u] = cx<T>{T(0), T(0)};
      pb[u] = cx<T>{T(0), T(0)};
      if (col < k) {
        if (r0 + row < m) pa[u] = N[(size_t)(r0 + row) * k + col];
        if (q0 + row < m) pb[u] = N[(size_t)(q0 + row) * k + col];
      }
    }
  };
  auto stash = [&](int sg) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = t + NT * u;
      const int row = e / KC, kk = e % KC;
      As[sg][0][kk][row] = pa[u].re;
      As[sg][1][kk][row] = pa[u].im;
      Bs[sg][0][kk][row] = pb[u].re;
      Bs[sg][1][kk][row] = -pb[u].im;
    }
  };
  fetch(0);
  stash(0);
  __syncthreads();
  int sg = 0;
  for (int k0 = 0; k0 < k; k0 += KC) {
    const bool more = k0 + KC < k;
    if (more) fetch(k0 + KC);
#pragma unroll
    for (int kk = 0; kk < KC; kk += 4) {
      const int ka = kk + (lane >> 4);
      T ar[BLR], ai[BLR], br[BLC], bi[BLC];
      for (int i = 0; i < BLR; ++i) {
        ar[i] = As[sg][0][ka][wr + i * 16 + (lane & 15)];
        ai[i] = As[sg][1][ka][wr + i * 16 + (lane & 15)];
      }
      for (int j = 0; j < BLC; ++j) {
        br[j] = Bs[sg][0][ka][wc + j * 16 + (lane & 15)];
        bi[j] = Bs[sg][1][ka][wc + j * 16 + (lane & 15)];
      }
      for (int i = 0; i < BLR; ++i)
        for (int j = 0; j < BLC; ++j) {
          accr[i][j] = mfma_t(ar[i], br[j], accr[i][j]);
          accr[i][j] = mfma_t(-ai[i], bi[j], accr[i][j]);
          acci[i][j] = mfma_t(ar[i], bi[j], acci[i][j]);
          acci[i][j] = mfma_t(ai[i], br[j], acci[i][j]);
        }
    }
    if (more) stash(sg ^ 1);
    __syncthreads();
    sg ^= 1;
  }
  double pur = 0.0, tr = 0.0;
  const double wgt = (I == J) ? 1.0 : 2.0;
  for (int i = 0; i < BLR; ++i)
    for (int j = 0; j < BLC; ++j)
      for (int q = 0; q < 4; ++q) {
        const int row = r0 + wr + i * 16 + mfma_row<T>(lane, q);
        const int col = q0 + wc + j * 16 + (lane & 15);
        if (row < m && col < m) {
          const double re = (double)accr[i][j][q], im = (double)acci[i][j][q];
          pur += wgt * (re * re + im * im);
          if (I == J && row == col) tr += re;
        }
      }
  pur = block_sum(pur, red);
  tr = block_sum(tr, red);
  if (t == 0) {
    partial[((size_t)slot * ntp + tile) * 2 + 0] = pur;
    partial[((size_t)slot * ntp + tile) * 2 + 1] = tr;
  }
}

// ------------------------------------------------------------------ split-BF16 scoring
// Each complex entry x of M_c is held as four BF16 planes: hi = bf16(Re x), lo = bf16(Re x - hi),
// and the same for Im x, so Re x = hi + lo to about 2^-16 relative.  A product of two such
// numbers keeps hi*hi + hi*lo + lo*hi (the lo*lo term is below the representation error); the
// Gram entries then carry a relative error of order 2^-16 and the FP64 window re-score decides.
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned short us8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ bf8 bf8_neg(bf8 x) {
  return __builtin_bit_cast(bf8, __builtin_bit_cast(us8, x) ^ (unsigned short)0x8000);
}
__device__ __forceinline__ f4 mfma_bf(bf8 a, bf8 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// M_c = reshape(Q_c Theta) (as k_gen_rotated<float>) written as planes [Re hi, Re lo, Im hi, Im lo],
// each m x k row-major BF16 with leading dimension ldk >= k (columns k..ldk-1 written as zeros);
// candidate slot ls at out + ls * stride (stride = 4 m ldk elements); cpt candidates per
// thread, as in k_gen_rotated.
template <int DD>
__global__ __launch_bounds__(256) void k_gen_rotated_bf16(int d_rt, int chil, int chir, const z64* __restrict__ theta,
                                                          const c32* __restrict__ qall, const int* __restrict__ list,
                                                          int c0, int cnt, const int* __restrict__ nlimit,
                                                          __bf16* __restrict__ out, size_t stride, int ldk,
                                                          int cpt) {
  const int d = DD > 0 ? DD : d_rt;
  constexpr int VMAX = DD > 0 ? DD * DD : kMaxD * kMaxD;
  const bool rows_first = chil * d <= d * chir;
  const int k = rows_first ? d * chir : chil * d;
  const int m = rows_first ? chil * d : d * chir;
  const int g0 = blockIdx.y * cpt;  // first candidate of this block's group
  if (g0 >= cnt || (nlimit && c0 + g0 >= *nlimit)) return;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool active = idx < (size_t)chil * chir;
  int a = 0, b = 0;
  if (active) {
    if (rows_first) {
      a = (int)(idx / chir);
      b = (int)(idx % chir);
    } else {
      b = (int)(idx / chil);
      a = (int)(idx % chil);
    }
  }
  const int D2 = d * d;
  c32 v[VMAX];
  if (active) {
    const z64* th = theta + (size_t)a * D2 * chir + b;
#pragma unroll
    for (int x = 0; x < VMAX; ++x) {
      if (x >= D2) break;
      const z64 tv = th[(size_t)x * chir];
      v[x] = c32{(float)tv.re, (float)tv.im};
    }
  }
  const size_t plane = (size_t)m * ldk;
  for (int u = 0; u < cpt; ++u) {
    const int ls = g0 + u;
    const int slot = c0 + ls;
    if (ls >= cnt || (nlimit && slot >= *nlimit)) break;  // uniform over the block
    const int c = list ? list[slot] : slot;
    __bf16* o = out + (size_t)ls * stride;
    if (ldk > k) {  // zero pad columns k..ldk-1 of every row of the four planes
      const int pad = ldk - k;
      const size_t np = (size_t)m * pad, nth = (size_t)gridDim.x * blockDim.x;
      for (size_t e = idx; e < np; e += nth) {
        const size_t at = (e / pad) * ldk + k + e % pad;
        for (int pl = 0; pl < 4; ++pl) o[pl * plane + at] = (__bf16)0.f;
      }
    }
    if (!active) continue;
    const c32* q = qall + (size_t)c * D2 * D2;
    for (int y = 0; y < D2; ++y) {
      const int s1p = y / d, s2p = y - s1p * d;
      c32 acc = {0.f, 0.f};
#pragma unroll
      for (int x = 0; x < VMAX; ++x) {
        if (x >= D2) break;
        acc = cadd(acc, cmul(q[y * D2 + x], v[x]));
      }
      const size_t row = rows_first ? (size_t)a * d + s1p : (size_t)s2p * chir + b;
      const size_t col = rows_first ? (size_t)s2p * chir + b : (size_t)a * d + s1p;
      const size_t e = row * ldk + col;
      const __bf16 rh = (__bf16)acc.re, ih = (__bf16)acc.im;
      o[e] = rh;
      o[plane + e] = (__bf16)(acc.re - (float)rh);
      o[2 * plane + e] = ih;
      o[3 * plane + e] = (__bf16)(acc.im - (float)ih);
    }
  }
}

// FP32 Gram purity with direct-to-LDS operand loads.  The rotated matrices arrive with rows
// padded by zero columns to a multiple of 16 (the zeros add nothing to rho), so k % 16 == 0.
// 128 x 128 tiles in eight waves (two rows of four, 64 x 32 each: two waves per SIMD, so one
// wave's LDS waits overlap the other's MFMAs); XCD-aware order and epilogue as in
// k_gram_purity.  Three real products per complex product (a quarter fewer MFMAs than four):
// T1 = Ar Br^T, T2 = Ai Bi^T with Bi = -Im B, T3 = (Ar + Ai)(Br + Bi)^T; re = T1 - T2,
// im = T3 - T1 - T2.
// Every 16-column chunk of a row is eight aligned 16-byte units (two complex values each), so
// the chunk of an operand tile (128 rows) is 16 blocks of 8 rows x 8 units, and one
// global_load_lds_dwordx4 of a wave moves a block straight into LDS, lane l filling the l-th
// 16-byte slot.  Lane l loads row 8b + (l >> 3), unit (l & 7) ^ (l >> 3): the units of a row are
// XOR-swizzled across its block so that the 16 rows read by one MFMA lane group fall in distinct
// banks.  Rows at or beyond m read row m - 1 (they only feed products outside the m x m result,
// which the epilogue drops).  The k order inside a chunk is permuted the same way for both
// operands: at MFMA step s lane group g takes k = 4g + s, so a lane reads its four k values of a
// row as two 16-byte units.  The next chunk streams into the other LDS stage while this one is
// multiplied: no register staging, one wait and one barrier per chunk.  (Staging through
// registers, as k_gram_purity does, peaked at 121 TFLOP/s at m = k = 768; this kernel at 140.)
__device__ __forceinline__ int dl_slot(int r, int ku) { return (r >> 3) * 64 + ((r & 7) << 3) + (ku ^ (r & 7)); }

typedef __attribute__((address_space(3))) void lds_void;

__global__ __launch_bounds__(512, 1) void k_gram_purity_dl(int m, int k, const c32* __restrict__ nbase, size_t stride,
                                                         int c0, int cnt, const int* __restrict__ nlimit, int ntp,
                                                         double* __restrict__ partial) {
  constexpr int TT = 128, NT = 512, WC = 4, BLR = 4, BLC = 2;
  const int L = blockIdx.x;
  const int xcd = L & 7, xslot = L >> 3;
  const int cg = xslot / ntp, tile = xslot - cg * ntp;
  const int ls = cg * 8 + xcd;
  const int slot = c0 + ls;
  if (ls >= cnt || (nlimit && slot >= *nlimit)) return;
  const c32* N = nbase + (size_t)ls * stride;
  const int nt = (m + TT - 1) / TT;
  int I, J;
  tile_pair(tile, nt, I, J);
  // two stages of both operands, 1024 16-byte slots (16 KB) each
  __shared__ float4 A0[1024], B0[1024], A1[1024], B1[1024];
  __shared__ double red[NT];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wr = (w / WC) * (TT / 2), wc = (w % WC) * (TT / WC);
  const int r0 = I * TT, q0 = J * TT;
  // wave w moves blocks w and w + 8 of each operand
  const int lr = lane >> 3, lku = (lane & 7) ^ lr;
  const c32* ga0 = N + (size_t)min(r0 + w * 8 + lr, m - 1) * k + 2 * lku;
  const c32* ga1 = N + (size_t)min(r0 + (w + 8) * 8 + lr, m - 1) * k + 2 * lku;
  const c32* gb0 = N + (size_t)min(q0 + w * 8 + lr, m - 1) * k + 2 * lku;
  const c32* gb1 = N + (size_t)min(q0 + (w + 8) * 8 + lr, m - 1) * k + 2 * lku;
  f4 accr[BLR][BLC], acci[BLR][BLC], acc3[BLR][BLC];
  for (int i = 0; i < BLR; ++i)
    for (int j = 0; j < BLC; ++j)
      for (int q = 0; q < 4; ++q) {
        accr[i][j][q] = 0.f;
        acci[i][j][q] = 0.f;
        acc3[i][j][q] = 0.f;
      }
  const int g = lane >> 4, rl = lane & 15;
  auto compute = [&](const float4* As, const float4* Bs) {
    float ar[BLR][4], ai[BLR][4], br[BLC][4], bi[BLC][4];
#pragma unroll
    for (int i = 0; i < BLR; ++i) {
      const int row = wr + i * 16 + rl;
      const float4 u0 = As[dl_slot(row, 2 * g)], u1 = As[dl_slot(row, 2 * g + 1)];
      ar[i][0] = u0.x;
      ai[i][0] = u0.y;
      ar[i][1] = u0.z;
      ai[i][1] = u0.w;
      ar[i][2] = u1.x;
      ai[i][2] = u1.y;
      ar[i][3] = u1.z;
      ai[i][3] = u1.w;
    }
#pragma unroll
    for (int j = 0; j < BLC; ++j) {
      const int row = wc + j * 16 + rl;
      const float4 u0 = Bs[dl_slot(row, 2 * g)], u1 = Bs[dl_slot(row, 2 * g + 1)];
      br[j][0] = u0.x;
      bi[j][0] = -u0.y;
      br[j][1] = u0.z;
      bi[j][1] = -u0.w;
      br[j][2] = u1.x;
      bi[j][2] = -u1.y;
      br[j][3] = u1.z;
      bi[j][3] = -u1.w;
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      float sa[BLR], sb[BLC];
      for (int i = 0; i < BLR; ++i) sa[i] = ar[i][s] + ai[i][s];
      for (int j = 0; j < BLC; ++j) sb[j] = br[j][s] + bi[j][s];
      for (int i = 0; i < BLR; ++i)
        for (int j = 0; j < BLC; ++j) {
          accr[i][j] = mfma_t(ar[i][s], br[j][s], accr[i][j]);
          acci[i][j] = mfma_t(ai[i][s], bi[j][s], acci[i][j]);
          acc3[i][j] = mfma_t(sa[i], sb[j], acc3[i][j]);
        }
    }
  };
  // The scheduling barriers keep the loads ahead of the products and every product ahead of the
  // wait for the next chunk (left alone, the compiler sinks the loads below the products).
  auto issue = [&](float4* As, float4* Bs, int k0) {
    __builtin_amdgcn_global_load_lds((const void*)(ga0 + k0), (lds_void*)(As + w * 64), 16, 0, 0);
    __builtin_amdgcn_global_load_lds((const void*)(ga1 + k0), (lds_void*)(As + (w + 8) * 64), 16, 0, 0);
    __builtin_amdgcn_global_load_lds((const void*)(gb0 + k0), (lds_void*)(Bs + w * 64), 16, 0, 0);
    __builtin_amdgcn_global_load_lds((const void*)(gb1 + k0), (lds_void*)(Bs + (w + 8) * 64), 16, 0, 0);
    __builtin_amdgcn_sched_barrier(0);
  };
  auto settle = [&]() {
    __builtin_amdgcn_sched_barrier(0);
    __builtin_amdgcn_s_waitcnt(0);  // this wave's loads have landed in LDS
    __syncthreads();                // ... and every other wave's
  };
  const int nch = k / 16;
  issue(A0, B0, 0);
  settle();
  int c = 0;
  for (; c + 2 <= nch; c += 2) {
    issue(A1, B1, (c + 1) * 16);
    compute(A0, B0);
    settle();
    if (c + 2 < nch) issue(A0, B0, (c + 2) * 16);
    compute(A1, B1);
    settle();
  }
  if (c < nch) compute(A0, B0);
  double pur = 0.0, tr = 0.0;
  const double wgt = (I == J) ? 1.0 : 2.0;
  for (int i = 0; i < BLR; ++i)
    for (int j = 0; j < BLC; ++j)
      for (int q = 0; q < 4; ++q) {
        const int row = r0 + wr + i * 16 + mfma_row<float>(lane, q);
        const int col = q0 + wc + j * 16 + (lane & 15);
        if (row < m && col < m) {
          const double t1 = (double)accr[i][j][q], t2 = (double)acci[i][j][q], t3 = (double)acc3[i][j][q];
          const double re = t1 - t2, im = t3 - t1 - t2;
          pur += wgt * (re * re + im * im);
          if (I == J && row == col) tr += re;
        }
      }
  pur = block_sum(pur, red);
  tr = block_sum(tr, red);
  if (t == 0) {
    partial[((size_t)slot * ntp + tile) * 2 + 0] = pur;
    partial[((size_t)slot * ntp + tile) * 2 + 1] = tr;
  }
}

// Purity tiles from the BF16 planes: tile (I, J), I <= J, of rho = M M^H (128 x 128 per
// workgroup, four waves of 4 x 4 16x16 blocks, v_mfma_f32_16x16x32_bf16).  Per 32-wide
// k chunk, a lane holds 8 consecutive k of one row per plane: A rows from tile I, B rows from
// tile J (same layout, rho[r][c] = sum_k M[r][k] conj(M[c][k])):
//   Re rho += Rh Rh + Rh Rl + Rl Rh + Ih Ih + Ih Il + Il Ih
//   Im rho += Ih Rh + Ih Rl + Il Rh - Rh Ih - Rh Il - Rl Ih.
// The planes arrive with rows padded by zero columns to a multiple of 32, so k % 32 == 0 and
// every chunk of a row is four aligned 16-byte groups.  LDS rows are 64 bytes; group g of row r
// sits in slot g ^ ((r >> 2) & 3), so the 16 rows read by a quarter-wave hit disjoint banks.
// Chunks are loaded straight into LDS: wave w moves plane w of each panel, one
// global_load_lds_dwordx4 per 16 rows (lane l fills the l-th 16-byte slot: row l >> 2, slot
// l & 3), and the next chunk streams into the other stage while this one is multiplied (one
// wait and one barrier per chunk).  Rows at or beyond m read row m - 1; they only feed results
// outside the m x m Gram.  XCD-aware workgroup order as in k_gram_purity.
constexpr int BT = 128, BKC = 32;
__global__ __launch_bounds__(256) void k_gram_purity_bf16(int m, int k, const __bf16* __restrict__ nbase,
                                                          size_t stride, int c0, int cnt,
                                                          const int* __restrict__ nlimit, int ntp,
                                                          double* __restrict__ partial) {
  const int L = blockIdx.x;
  const int xcd = L & 7, xslot = L >> 3;
  const int cg = xslot / ntp, tile = xslot - cg * ntp;
  const int ls = cg * 8 + xcd;
  const int slot = c0 + ls;
  if (ls >= cnt || (nlimit && slot >= *nlimit)) return;
  const __bf16* N = nbase + (size_t)ls * stride;
  const size_t plane = (size_t)m * k;
  const int nt = (m + BT - 1) / BT;
  int I, J;
  tile_pair(tile, nt, I, J);
  const bool diag = (I == J);
  // two stages of [panel A/B][plane][row][32 k as four 16-byte groups]
  __shared__ us8 S0[2][4][BT][4];
  __shared__ us8 S1[2][4][BT][4];
  __shared__ double red[256];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wr = (w >> 1) * (BT / 2), wc = (w & 1) * (BT / 2);
  f4 accr[4][4], acci[4][4];
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j)
      for (int q = 0; q < 4; ++q) {
        accr[i][j][q] = 0.f;
        acci[i][j][q] = 0.f;
      }
  const int r0 = I * BT, q0 = J * BT;
  // loader lane: row (lane >> 2) of a 16-row block, slot lane & 3 holding group slot ^ ((row >> 2) & 3)
  const int lrow = lane >> 2, lgrp = (lane & 3) ^ ((lrow >> 2) & 3);
  const __bf16* pA = N + (size_t)w * plane + 8 * lgrp;
  auto issue = [&](us8 (*Sx)[4][BT][4], int k0) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int row = 16 * u + lrow;
      __builtin_amdgcn_global_load_lds((const void*)(pA + (size_t)min(r0 + row, m - 1) * k + k0),
                                       (lds_void*)&Sx[0][w][16 * u][0], 16, 0, 0);
      if (!diag)
        __builtin_amdgcn_global_load_lds((const void*)(pA + (size_t)min(q0 + row, m - 1) * k + k0),
                                         (lds_void*)&Sx[1][w][16 * u][0], 16, 0, 0);
    }
    __builtin_amdgcn_sched_barrier(0);
  };
  auto settle = [&]() {
    __builtin_amdgcn_sched_barrier(0);
    __builtin_amdgcn_s_waitcnt(0);  // this wave's loads have landed in LDS
    __syncthreads();                // ... and every other wave's
  };
  const int bpan = diag ? 0 : 1;
  const int g = lane >> 4, rr = lane & 15;
  auto compute = [&](us8 (*Sx)[4][BT][4]) {
    bf8 A[4][6], B[4][4];  // A: [block i][Rh, Rl, Ih, Il, -Rh, -Rl]; B: [block j][Rh, Rl, Ih, Il]
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int row = wc + j * 16 + rr;
      const int slotg = g ^ ((row >> 2) & 3);
#pragma unroll
      for (int pl = 0; pl < 4; ++pl) B[j][pl] = __builtin_bit_cast(bf8, Sx[bpan][pl][row][slotg]);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int row = wr + i * 16 + rr;
      const int slotg = g ^ ((row >> 2) & 3);
#pragma unroll
      for (int pl = 0; pl < 4; ++pl) A[i][pl] = __builtin_bit_cast(bf8, Sx[0][pl][row][slotg]);
      A[i][4] = bf8_neg(A[i][0]);
      A[i][5] = bf8_neg(A[i][1]);
    }
    // term-major order: consecutive MFMAs write different accumulators
    constexpr int TA[12] = {0, 0, 1, 2, 2, 3, 2, 2, 3, 4, 4, 5};
    constexpr int TB[12] = {0, 1, 0, 2, 3, 2, 0, 1, 0, 2, 3, 2};
#pragma unroll
    for (int term = 0; term < 12; ++term) {
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          if (term < 6)
            accr[i][j] = mfma_bf(A[i][TA[term]], B[j][TB[term]], accr[i][j]);
          else
            acci[i][j] = mfma_bf(A[i][TA[term]], B[j][TB[term]], acci[i][j]);
        }
    }
  };
  const int nch = k / BKC;
  issue(S0, 0);
  settle();
  int c = 0;
  for (; c + 2 <= nch; c += 2) {
    issue(S1, (c + 1) * BKC);
    compute(S0);
    settle();
    if (c + 2 < nch) issue(S0, (c + 2) * BKC);
    compute(S1);
    settle();
  }
  if (c < nch) compute(S0);
  double pur = 0.0, tr = 0.0;
  const double wgt = diag ? 1.0 : 2.0;
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j)
      for (int q = 0; q < 4; ++q) {
        const int row = r0 + wr + i * 16 + mfma_row_f32(lane, q);
        const int col = q0 + wc + j * 16 + (lane & 15);
        if (row < m && col < m) {
          const double re = (double)accr[i][j][q], im = (double)acci[i][j][q];
          pur += wgt * (re * re + im * im);
          if (diag && row == col) tr += re;
        }
      }
  pur = block_sum(pur, red);
  tr = block_sum(tr, red);
  if (t == 0) {
    partial[((size_t)slot * ntp + tile) * 2 + 0] = pur;
    partial[((size_t)slot * ntp + tile) * 2 + 1] = tr;
  }
}

__global__ void k_score_reduce(int ntp, const int* __restrict__ nlimit, int count, const double* __restrict__ partial,
                               double* __restrict__ s2) {
  int slot = blockIdx.x * blockDim.x + threadIdx.x;
  int lim = nlimit ? *nlimit : count;
  if (slot >= lim || slot >= count) return;
  double pur = 0.0, tr = 0.0;
  for (int i = 0; i < ntp; ++i) {
    pur += partial[((size_t)slot * ntp + i) * 2 + 0];
    tr += partial[((size_t)slot * ntp + i) * 2 + 1];
  }
  s2[slot] = -log(pur / (tr * tr));
}

// ===================================================================================== selection
__global__ __launch_bounds__(1024) void k_select(int count, const double* __restrict__ s2, double tol,
                                                 DevStatus* st) {
  __shared__ double red[1024];
  __shared__ int redi[1024];
  const int t = threadIdx.x;
  double mn = DBL_MAX;
  for (int i = t; i < count; i += 1024) mn = fmin(mn, s2[i]);
  red[t] = mn;
  __syncthreads();
  for (int off = 512; off > 0; off >>= 1) {
    if (t < off) red[t] = fmin(red[t], red[t + off]);
    __syncthreads();
  }
  const double smin = red[0];
  int best = 0x7fffffff;
  for (int i = t; i < count; i += 1024)
    if (s2[i] <= smin + tol && i < best) best = i;
  redi[t] = best;
  __syncthreads();
  for (int off = 512; off > 0; off >>= 1) {
    if (t < off) redi[t] = min(redi[t], redi[t + off]);
    __syncthreads();
  }
  if (t == 0) {
    st->cstar = redi[0];
    st->s2min = smin;
  }
}

__global__ __launch_bounds__(1024) void k_window(int count, const double* __restrict__ s2lp, double window,
                                                 int* __restrict__ list, DevStatus* st) {
  __shared__ double red[1024];
  __shared__ int cnt[1024];
  const int t = threadIdx.x;
  double mn = DBL_MAX;
  for (int i = t; i < count; i += 1024) mn = fmin(mn, s2lp[i]);
  red[t] = mn;
  __syncthreads();
  for (int off = 512; off > 0; off >>= 1) {
    if (t < off) red[t] = fmin(red[t], red[t + off]);
    __syncthreads();
  }
  const double lim = red[0] + window;
  // contiguous ranges per thread keep the list in ascending order
  const int per = (count + 1023) / 1024;
  const int b0 = t * per, b1 = min(count, b0 + per);
  int my = 0;
  for (int i = b0; i < b1; ++i)
    if (s2lp[i] <= lim) ++my;
  cnt[t] = my;
  __syncthreads();
  if (t == 0) {
    int run = 0;
    for (int i = 0; i < 1024; ++i) {
      int v = cnt[i];
      cnt[i] = run;
      run += v;
    }
    st->nwindow = run;
    st->smin_lp = red[0];
  }
  __syncthreads();
  int pos = cnt[t];
  for (int i = b0; i < b1; ++i)
    if (s2lp[i] <= lim) list[pos++] = i;
}

__global__ __launch_bounds__(1024) void k_select_window(const int* __restrict__ list, const double* __restrict__ s2w,
                                                        double tol, DevStatus* st) {
  __shared__ double red[1024];
  __shared__ int redi[1024];
  const int t = threadIdx.x;
  const int nw = st->nwindow;
  double mn = DBL_MAX;
  for (int i = t; i < nw; i += 1024) mn = fmin(mn, s2w[i]);
  red[t] = mn;
  __syncthreads();
  for (int off = 512; off > 0; off >>= 1) {
    if (t < off) red[t] = fmin(red[t], red[t + off]);
    __syncthreads();
  }
  const double smin = red[0];
  int best = 0x7fffffff;
  for (int i = t; i < nw; i += 1024)
    if (s2w[i] <= smin + tol && list[i] < best) best = list[i];
  redi[t] = best;
  __syncthreads();
  for (int off = 512; off > 0; off >>= 1) {
    if (t < off) redi[t] = min(redi[t], redi[t + off]);
    __syncthreads();
  }
  if (t == 0) {
    st->cstar = redi[0];
    st->s2min = smin;
  }
}

// ===================================================================================== dense helpers
__device__ __forceinline__ z64 tau_pow(int p, int d) {
  double ang = M_PI * (double)p / (double)d;
  return z64{cos(ang), sin(ang)};
}

__global__ void k_apply_weyl_dense(int n, int d, long long D, const int* __restrict__ x, const int* __restrict__ z,
                                   int p, const z64* __restrict__ in, z64* __restrict__ out, int accumulate,
                                   z64 coeff) {
  long long y = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (y >= D) return;
  // digits of y, site 0 most significant
  long long rem = y, src = 0, mul = 1;
  int ph = 0;
  for (int i = n - 1; i >= 0; --i) {
    int yi = (int)(rem % d);
    rem /= d;
    int si = (yi - x[i] + d) % d;
    ph += z[i] * si;
    src += si * mul;
    mul *= d;
  }
  z64 f = tau_pow((p + 2 * (ph % d)) % (2 * d), d);
  z64 v = cmul(cmul(coeff, f), in[src]);
  out[y] = accumulate ? cadd(out[y], v) : v;
}

__global__ void k_clifford_dense(int n, int d, long long D, const int* __restrict__ a_idx,
                                 const int8_t* __restrict__ b_dig, const int* __restrict__ p_x,
                                 const z64* __restrict__ mvec, const z64* __restrict__ s0, z64* __restrict__ out) {
  long long y = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (y >= D) return;
  int yd[32];
  long long rem = y;
  for (int i = n - 1; i >= 0; --i) {
    yd[i] = (int)(rem % d);
    rem /= d;
  }
  z64 acc = {0.0, 0.0};
  for (long long xi = 0; xi < D; ++xi) {
    z64 mv = mvec[xi];
    if (mv.re == 0.0 && mv.im == 0.0) continue;
    long long a = a_idx[xi];
    const int8_t* bd = b_dig + xi * n;
    long long src = 0, mul = 1;
    int ph = 0;
    for (int i = n - 1; i >= 0; --i) {
      int ai = (int)(a % d);
      a /= d;
      int si = (yd[i] - ai + d) % d;
      ph += bd[i] * si;
      src += si * mul;
      mul *= d;
    }
    z64 f = tau_pow((p_x[xi] + 2 * (ph % d)) % (2 * d), d);
    acc = cadd(acc, cmul(mv, cmul(f, s0[src])));
  }
  out[y] = acc;
}

__global__ void k_scale(z64* v, size_t count, z64 f) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) v[i] = cmul(v[i], f);
}

__global__ void k_norm2(const z64* __restrict__ v, size_t count, double* out) {
  __shared__ double red[1024];
  double s = 0.0;
  for (size_t i = threadIdx.x; i < count; i += 1024) s += cabs2(v[i]);
  double r = block_sum(s, red);
  if (threadIdx.x == 0) *out = r;
}

}  // namespace

// ===================================================================================== launchers
void launch_mpo_site(hipStream_t s, int kind, int d, int chil, int chir, int dx, int dz, const MpoCoeff& co,
                     const z64* in, z64* out) {
  int ol = (kind == 1 || kind == 2) ? d * chil : chil;
  int orr = (kind == 0 || kind == 1) ? d * chir : chir;
  size_t total = (size_t)ol * d * orr;
  hipLaunchKernelGGL(k_mpo_site, dim3(blocks_for(total, 256)), dim3(256), 0, s, kind, d, chil, chir, dx, dz, co, in,
                     out);
  GC_LAUNCH_CHECK();
}

void launch_mpo_sum_site(hipStream_t s, int kind, int d, int J, int chil, int chir, const MpoTerms& terms,
                         const z64* in, z64* out) {
  GC_CHECK(J >= 1 && J <= kMaxGateTerms, GCAMPS_EINVAL, "MPO bond out of range");
  const int ol = (kind == 1 || kind == 2) ? J * chil : chil;
  const int orr = (kind == 0 || kind == 1) ? J * chir : chir;
  const size_t total = (size_t)ol * d * orr;
  hipLaunchKernelGGL(k_mpo_sum_site, dim3(blocks_for(total, 256)), dim3(256), 0, s, kind, d, J, chil, chir, terms, in,
                     out);
  GC_LAUNCH_CHECK();
}

void launch_apply_q(hipStream_t s, int d, int chil, int chir, const DevStatus* st, const z64* qmats, z64* theta) {
  size_t total = (size_t)chil * chir;
  hipLaunchKernelGGL(k_apply_q, dim3(blocks_for(total, 128)), dim3(128), 0, s, d, chil, chir, st, qmats, theta);
  GC_LAUNCH_CHECK();
}

void launch_rotate_copy(hipStream_t s, int d, int chil, int chir, int c, const z64* qmats, const z64* theta,
                        z64* out) {
  const size_t total = (size_t)chil * chir;
  hipLaunchKernelGGL(k_rotate_copy, dim3(blocks_for(total, 128)), dim3(128), 0, s, d, chil, chir, c, qmats, theta,
                     out);
  GC_LAUNCH_CHECK();
}

// Candidates per generator thread for full-set chunks of `first` candidates: the tuner's pick per
// (precision, d, chi_l, chi_r), timed on the first chunk (gen(c0, cnt, cpt) launches the generator).
template <typename Gen>
int gen_cpt(hipStream_t s, int prec, int d, int chil, int chir, const int* nlimit, int first, const Gen& gen) {
  if (nlimit || first < kGenMinChunk) return kGenCands;  // such chunks take one candidate per thread
  return tuned_choice(s, "gen_cpt", prec, d, chil, chir, kGenCpt, (int)(sizeof(kGenCpt) / sizeof(kGenCpt[0])),
                      kGenCands, [&](int cpt) { gen(0, first, cpt); });
}

void launch_score(hipStream_t s, int prec, int d, int chil, int chir, const z64* theta, const z64* q64, const c32* q32,
                  const int* list, int count, const int* nlimit, double* s2, double* partial, size_t partial_cap,
                  void* nbuf, size_t nbuf_bytes, hipEvent_t* evs, int evcap, int* evused, const z64* replica_tables) {
  if (evused) *evused = 0;
  if (count <= 0) return;
  if (prec == GCAMPS_SCORE_REPLICA) GC_CHECK(list == nullptr && nlimit == nullptr, GCAMPS_EINVAL,
                                             "replica scoring takes the full candidate set");
  const bool rows_first = chil * d <= d * chir;
  const int m = rows_first ? chil * d : d * chir;
  const int k = rows_first ? d * chir : chil * d;
  if (m <= SMALL_M) {
    if (prec == GCAMPS_SCORE_FP64 || prec == GCAMPS_SCORE_REPLICA)
      hipLaunchKernelGGL(k_score_small<double>, dim3(count), dim3(SMALL_THREADS), 0, s, d, chil, chir, theta, q64,
                         q32, list, nlimit, s2);
    else
      hipLaunchKernelGGL(k_score_small<float>, dim3(count), dim3(SMALL_THREADS), 0, s, d, chil, chir, theta, q64, q32,
                         list, nlimit, s2);
    GC_LAUNCH_CHECK();
    return;
  }
  if (prec == GCAMPS_SCORE_REPLICA) {
    GC_CHECK(replica_tables != nullptr, GCAMPS_EINVAL, "replica scoring without candidate tables");
    launch_score_replica(s, d, chil, chir, theta, replica_tables, count, s2, nbuf, nbuf_bytes);
    return;
  }
  if (prec == GCAMPS_SCORE_BF16) {
    const int nt = (m + BT - 1) / BT;
    const int ntp = nt * (nt + 1) / 2;
    GC_CHECK((size_t)count * ntp * 2 <= partial_cap, GCAMPS_ECAPACITY, "scoring partial buffer too small");
    const int ldk = (k + BKC - 1) / BKC * BKC;  // rows padded with zeros to whole 32-column chunks
    const size_t stride = 4 * (size_t)m * ldk;  // BF16 elements per candidate (four planes)
    const int chunk = (int)std::min<size_t>((size_t)count, nbuf_bytes / (stride * sizeof(__bf16)));
    GC_CHECK(chunk >= 1, GCAMPS_ECAPACITY, "rotated-matrix buffer too small");
    __bf16* nb = reinterpret_cast<__bf16*>(nbuf);
    auto gen = [&](int c0, int cnt, int cpt) {
      const dim3 gg(blocks_for((size_t)chil * chir, 256), (cnt + cpt - 1) / cpt);
      if (d == 3)
        hipLaunchKernelGGL((k_gen_rotated_bf16<3>), gg, dim3(256), 0, s, d, chil, chir, theta, q32, list, c0, cnt,
                           nlimit, nb, stride, ldk, cpt);
      else if (d == 2)
        hipLaunchKernelGGL((k_gen_rotated_bf16<2>), gg, dim3(256), 0, s, d, chil, chir, theta, q32, list, c0, cnt,
                           nlimit, nb, stride, ldk, cpt);
      else
        hipLaunchKernelGGL((k_gen_rotated_bf16<0>), gg, dim3(256), 0, s, d, chil, chir, theta, q32, list, c0, cnt,
                           nlimit, nb, stride, ldk, cpt);
      GC_LAUNCH_CHECK();
    };
    const int cpt_full = gen_cpt(s, prec, d, chil, chir, nlimit, std::min(chunk, count), gen);
    for (int c0 = 0; c0 < count; c0 += chunk) {
      const int cnt = std::min(chunk, count - c0);
      const int cpt = (!nlimit && cnt >= kGenMinChunk) ? cpt_full : 1;
      const dim3 gp((unsigned)ntp * ((cnt + 7) / 8) * 8);
      const int ev = (evs && evused && 2 * (*evused) + 1 < evcap) ? 2 * (*evused) : -1;
      gen(c0, cnt, cpt);
      if (ev >= 0) GC_HIP(hipEventRecord(evs[ev], s));
      hipLaunchKernelGGL(k_gram_purity_bf16, gp, dim3(256), 0, s, m, ldk, nb, stride, c0, cnt, nlimit, ntp, partial);
      if (ev >= 0) GC_HIP(hipEventRecord(evs[ev + 1], s));
      GC_LAUNCH_CHECK();
      if (ev >= 0) ++(*evused);
    }
    hipLaunchKernelGGL(k_score_reduce, dim3(blocks_for(count, 128)), dim3(128), 0, s, ntp, nlimit, count, partial, s2);
    GC_LAUNCH_CHECK();
    return;
  }
  const int TT = (prec == GCAMPS_SCORE_FP64) ? 64 : 128;
  const int nt = (m + TT - 1) / TT;
  const int ntp = nt * (nt + 1) / 2;
  GC_CHECK((size_t)count * ntp * 2 <= partial_cap, GCAMPS_ECAPACITY, "scoring partial buffer too small");
  const size_t elem = (prec == GCAMPS_SCORE_FP64) ? sizeof(z64) : sizeof(c32);
  // FP32 rows are padded with zero columns to a multiple of 16 for k_gram_purity_dl
  const int ldk = (prec == GCAMPS_SCORE_FP64) ? k : (k + 15) / 16 * 16;
  const size_t stride = (size_t)m * ldk;
  const int chunk = (int)std::min<size_t>((size_t)count, nbuf_bytes / (stride * elem));
  GC_CHECK(chunk >= 1, GCAMPS_ECAPACITY, "rotated-matrix buffer too small");

  auto gen = [&](int c0, int cnt, int cpt) {
    const dim3 gg(blocks_for((size_t)chil * chir, 256), (cnt + cpt - 1) / cpt);
    if (prec == GCAMPS_SCORE_FP64) {
      z64* nb = reinterpret_cast<z64*>(nbuf);
      if (d == 3)
        hipLaunchKernelGGL((k_gen_rotated<double, 3>), gg, dim3(256), 0, s, d, chil, chir, theta, q64, list, c0, cnt,
                           nlimit, nb, stride, ldk, cpt);
      else if (d == 2)
        hipLaunchKernelGGL((k_gen_rotated<double, 2>), gg, dim3(256), 0, s, d, chil, chir, theta, q64, list, c0, cnt,
                           nlimit, nb, stride, ldk, cpt);
      else
        hipLaunchKernelGGL((k_gen_rotated<double, 0>), gg, dim3(256), 0, s, d, chil, chir, theta, q64, list, c0, cnt,
                           nlimit, nb, stride, ldk, cpt);
    } else {
      c32* nb = reinterpret_cast<c32*>(nbuf);
      if (d == 3)
        hipLaunchKernelGGL((k_gen_rotated<float, 3>), gg, dim3(256), 0, s, d, chil, chir, theta, q32, list, c0, cnt,
                           nlimit, nb, stride, ldk, cpt);
      else if (d == 2)
        hipLaunchKernelGGL((k_gen_rotated<float, 2>), gg, dim3(256), 0, s, d, chil, chir, theta, q32, list, c0, cnt,
                           nlimit, nb, stride, ldk, cpt);
      else
        hipLaunchKernelGGL((k_gen_rotated<float, 0>), gg, dim3(256), 0, s, d, chil, chir, theta, q32, list, c0, cnt,
                           nlimit, nb, stride, ldk, cpt);
    }
    GC_LAUNCH_CHECK();
  };
  const int cpt_full = gen_cpt(s, prec, d, chil, chir, nlimit, std::min(chunk, count), gen);
  for (int c0 = 0; c0 < count; c0 += chunk) {
    const int cnt = std::min(chunk, count - c0);
    const int cpt = (!nlimit && cnt >= kGenMinChunk) ? cpt_full : 1;
    const dim3 gp((unsigned)ntp * ((cnt + 7) / 8) * 8);
    const int ev = (evs && evused && 2 * (*evused) + 1 < evcap) ? 2 * (*evused) : -1;
    gen(c0, cnt, cpt);
    if (prec == GCAMPS_SCORE_FP64) {
      z64* nb = reinterpret_cast<z64*>(nbuf);
      if (ev >= 0) GC_HIP(hipEventRecord(evs[ev], s));
      hipLaunchKernelGGL((k_gram_purity<double, 2, 4>), gp, dim3(256), 0, s, m, k, nb, stride, c0, cnt, nlimit, ntp,
                         partial);
      if (ev >= 0) GC_HIP(hipEventRecord(evs[ev + 1], s));
    } else {
      c32* nb = reinterpret_cast<c32*>(nbuf);
      if (ev >= 0) GC_HIP(hipEventRecord(evs[ev], s));
      hipLaunchKernelGGL(k_gram_purity_dl, gp, dim3(512), 0, s, m, ldk, nb, stride, c0, cnt, nlimit, ntp, partial);
      if (ev >= 0) GC_HIP(hipEventRecord(evs[ev + 1], s));
    }
    GC_LAUNCH_CHECK();
    if (ev >= 0) ++(*evused);
  }
  hipLaunchKernelGGL(k_score_reduce, dim3(blocks_for(count, 128)), dim3(128), 0, s, ntp, nlimit, count, partial, s2);
  GC_LAUNCH_CHECK();
}

void launch_select(hipStream_t s, int count, const double* s2, double tie_tol, DevStatus* st) {
  hipLaunchKernelGGL(k_select, dim3(1), dim3(1024), 0, s, count, s2, tie_tol, st);
  GC_LAUNCH_CHECK();
}

void launch_window(hipStream_t s, int count, const double* s2lp, double window, int* list, DevStatus* st) {
  hipLaunchKernelGGL(k_window, dim3(1), dim3(1024), 0, s, count, s2lp, window, list, st);
  GC_LAUNCH_CHECK();
}

void launch_select_window(hipStream_t s, const int* list, const double* s2win, double tie_tol, DevStatus* st) {
  hipLaunchKernelGGL(k_select_window, dim3(1), dim3(1024), 0, s, list, s2win, tie_tol, st);
  GC_LAUNCH_CHECK();
}

void launch_apply_weyl_dense(hipStream_t s, int n, int d, long long D, const int* x, const int* z, int p,
                             const z64* in, z64* out, int accumulate, z64 coeff) {
  hipLaunchKernelGGL(k_apply_weyl_dense, dim3(blocks_for((size_t)D, 256)), dim3(256), 0, s, n, d, D, x, z, p, in,
                     out, accumulate, coeff);
  GC_LAUNCH_CHECK();
}

void launch_clifford_dense(hipStream_t s, int n, int d, long long D, const int* a_idx, const int8_t* b_dig,
                           const int* p_x, const z64* mvec, const z64* s0, z64* out) {
  hipLaunchKernelGGL(k_clifford_dense, dim3(blocks_for((size_t)D, 128)), dim3(128), 0, s, n, d, D, a_idx, b_dig, p_x,
                     mvec, s0, out);
  GC_LAUNCH_CHECK();
}

void launch_scale(hipStream_t s, z64* v, size_t count, z64 f) {
  hipLaunchKernelGGL(k_scale, dim3(blocks_for(count, 256)), dim3(256), 0, s, v, count, f);
  GC_LAUNCH_CHECK();
}

void launch_norm2(hipStream_t s, const z64* v, size_t count, double* out) {
  hipLaunchKernelGGL(k_norm2, dim3(1), dim3(1024), 0, s, v, count, out);
  GC_LAUNCH_CHECK();
}

}  // namespace gc
