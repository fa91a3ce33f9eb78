// Dense FP64 complex linear algebra for the MPS factorisations (§2.4: truncation by SVD).
//
// * k_zgemm / k_zgemm_ks: C = alpha op(A) op(B) on 32x32 tiles with v_mfma_f64_16x16x4 (a
//   complex product is four real MFMAs into a real and an imaginary accumulator).
// * Hermitian eigen-decomposition by two-sided Jacobi rotations: a single-workgroup kernel that
//   keeps the whole matrix in LDS (m <= kSmallEig) and a block-Jacobi scheme for larger m
//   (pairs of 16-blocks solved as 32x32 sub-problems in LDS, the rotations applied to the matrix
//   and the eigenvector accumulator as 32x32 MFMA tile products).
// * k_trunc: descending sort of squared singular values and the truncation rule.
// * k_emit: writes the two factors of a split in the requested orientation.
#include <cfloat>
#include <cstring>

#include "kernels.h"

namespace gc {

typedef double d4 __attribute__((ext_vector_type(4)));

namespace {

// ===================================================================================== GEMM
// Two forms, both on 32 x 32 output tiles (a 768 x 768 product has 576 of them, so that every
// CU gets work where 64 x 64 tiles left 40% of the chip idle).  K advances in chunks of 16;
// each chunk is fetched into registers while the previous one is multiplied, then stored into
// the other LDS stage (one barrier per chunk).  A complex product is four real MFMAs into a real
// and an imaginary accumulator.  Hermitian products (herm: M == N and op(B) = op(A)^H) compute
// the upper triangle, diagonal included, and write its mirror.
constexpr int GT = 32, GK = 16, GLD = GT + 4;

// Output element (row, col) of a Hermitian or general product, with alpha and accumulate.
__device__ __forceinline__ void gemm_store(z64* __restrict__ C, int ldc, int M, int N, int row, int col, double sr,
                                           double si, z64 alpha, int accumulate, int herm) {
  if (row >= M || col >= N || (herm && row > col)) return;
  z64 v = {alpha.re * sr - alpha.im * si, alpha.re * si + alpha.im * sr};
  if (accumulate) v = cadd(v, C[(size_t)row * ldc + col]);
  C[(size_t)row * ldc + col] = v;
  if (herm && row < col) C[(size_t)col * ldc + row] = cconj(v);
}

// Element e of a 32-row (or 32-column) operand tile times KC k values, as (row or column, k):
// k fastest when LAYOUT is 0, the row or column fastest when it is 1.  Each operand takes the
// order in which consecutive threads read consecutive addresses: A as is and B transposed are
// contiguous along k (layout 0), A transposed and B as is along the row or column (layout 1).
template <int LAYOUT, int KC>
__device__ __forceinline__ void tile_elem(int e, int& rc, int& kk) {
  if (LAYOUT == 0) {
    rc = e / KC;
    kk = e % KC;
  } else {
    rc = e % GT;
    kk = e / GT;
  }
}
template <int OP>
__device__ __forceinline__ z64 load_a(const z64* __restrict__ A, int lda, int M, int K, int gr, int gk) {
  z64 v = {0.0, 0.0};
  if (gr < M && gk < K) {
    if (OP == 0) {
      v = A[(size_t)gr * lda + gk];
    } else {
      v = A[(size_t)gk * lda + gr];
      v.im = -v.im;
    }
  }
  return v;
}
template <int OP>
__device__ __forceinline__ z64 load_b(const z64* __restrict__ B, int ldb, int N, int K, int gc, int gk) {
  z64 v = {0.0, 0.0};
  if (gc < N && gk < K) {
    if (OP == 0) {
      v = B[(size_t)gk * ldb + gc];
    } else {
      v = B[(size_t)gc * ldb + gk];
      v.im = -v.im;
    }
  }
  return v;
}

// Four waves, each a 16 x 16 quadrant of the tile, over every K chunk.
template <int OPA, int OPB>
__global__ __launch_bounds__(256) void k_zgemm(int M, int N, int K, const z64* __restrict__ A, int lda,
                                               const z64* __restrict__ B, int ldb, z64* __restrict__ C, int ldc,
                                               z64 alpha, int accumulate, int herm) {
  const int m0 = blockIdx.y * GT, n0 = blockIdx.x * GT;
  if (herm && m0 >= n0 + GT) return;  // entirely below the diagonal
  __shared__ double As[2][2][GK][GLD];  // [stage][re, im][k][row]
  __shared__ double Bs[2][2][GK][GLD];  // [stage][re, im][k][col]
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wr = (w >> 1) * 16, wc = (w & 1) * 16;
  d4 accr = {0, 0, 0, 0}, acci = {0, 0, 0, 0};
  z64 ra[2], rb[2];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      int r, kk;
      tile_elem<OPA, GK>(t + 256 * i, r, kk);
      ra[i] = load_a<OPA>(A, lda, M, K, m0 + r, k0 + kk);
      tile_elem<OPB == 0 ? 1 : 0, GK>(t + 256 * i, r, kk);
      rb[i] = load_b<OPB>(B, ldb, N, K, n0 + r, k0 + kk);
    }
  };
  auto stash = [&](int s) {
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      int r, kk;
      tile_elem<OPA, GK>(t + 256 * i, r, kk);
      As[s][0][kk][r] = ra[i].re;
      As[s][1][kk][r] = ra[i].im;
      tile_elem<OPB == 0 ? 1 : 0, GK>(t + 256 * i, r, kk);
      Bs[s][0][kk][r] = rb[i].re;
      Bs[s][1][kk][r] = rb[i].im;
    }
  };
  const int nch = (K + GK - 1) / GK;
  fetch(0);
  stash(0);
  __syncthreads();
  for (int c = 0; c < nch; ++c) {
    const int s = c & 1;
    if (c + 1 < nch) fetch((c + 1) * GK);
#pragma unroll
    for (int kk = 0; kk < GK; kk += 4) {
      const int ka = kk + (lane >> 4);
      const double ar = As[s][0][ka][wr + (lane & 15)], ai = As[s][1][ka][wr + (lane & 15)];
      const double br = Bs[s][0][ka][wc + (lane & 15)], bi = Bs[s][1][ka][wc + (lane & 15)];
      accr = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, br, accr, 0, 0, 0);
      accr = __builtin_amdgcn_mfma_f64_16x16x4f64(-ai, bi, accr, 0, 0, 0);
      acci = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, bi, acci, 0, 0, 0);
      acci = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, br, acci, 0, 0, 0);
    }
    if (c + 1 < nch) stash(s ^ 1);
    __syncthreads();
  }
  for (int q = 0; q < 4; ++q)
    gemm_store(C, ldc, M, N, m0 + wr + mfma_row_f64(lane, q), n0 + wc + (lane & 15), accr[q], acci[q], alpha,
               accumulate, herm);
}

// Eight waves for products with few tiles: wave group g (waves 4g..4g+3, one 16 x 16 quadrant
// each) takes chunk 2p + g of every chunk pair p, and group 1 hands its sums to group 0 through
// LDS at the end (two partial sums per element, added in a fixed order).
template <int OPA, int OPB>
__global__ __launch_bounds__(512) void k_zgemm_ks(int M, int N, int K, const z64* __restrict__ A, int lda,
                                                  const z64* __restrict__ B, int ldb, z64* __restrict__ C, int ldc,
                                                  z64 alpha, int accumulate, int herm) {
  const int m0 = blockIdx.y * GT, n0 = blockIdx.x * GT;
  if (herm && m0 >= n0 + GT) return;
  __shared__ double As[2][2][2][GK][GLD];  // [stage][group][re, im][k][row]
  __shared__ double Bs[2][2][2][GK][GLD];
  __shared__ double Xr[4][4][64], Xi[4][4][64];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6, grp = w >> 2, wl = w & 3;
  const int wr = (wl >> 1) * 16, wc = (wl & 1) * 16;
  d4 accr = {0, 0, 0, 0}, acci = {0, 0, 0, 0};
  z64 ra[2], rb[2];
  auto fetch = [&](int k0) {  // a chunk pair: 32 rows x 32 k values of each operand
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      int r, kk;
      tile_elem<OPA, 2 * GK>(t + 512 * i, r, kk);
      ra[i] = load_a<OPA>(A, lda, M, K, m0 + r, k0 + kk);
      tile_elem<OPB == 0 ? 1 : 0, 2 * GK>(t + 512 * i, r, kk);
      rb[i] = load_b<OPB>(B, ldb, N, K, n0 + r, k0 + kk);
    }
  };
  auto stash = [&](int s) {
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      int r, kk;
      tile_elem<OPA, 2 * GK>(t + 512 * i, r, kk);
      As[s][kk / GK][0][kk % GK][r] = ra[i].re;
      As[s][kk / GK][1][kk % GK][r] = ra[i].im;
      tile_elem<OPB == 0 ? 1 : 0, 2 * GK>(t + 512 * i, r, kk);
      Bs[s][kk / GK][0][kk % GK][r] = rb[i].re;
      Bs[s][kk / GK][1][kk % GK][r] = rb[i].im;
    }
  };
  const int npair = (K + 2 * GK - 1) / (2 * GK);
  fetch(0);
  stash(0);
  __syncthreads();
  for (int c = 0; c < npair; ++c) {
    const int s = c & 1;
    if (c + 1 < npair) fetch((c + 1) * 2 * GK);
#pragma unroll
    for (int kk = 0; kk < GK; kk += 4) {
      const int ka = kk + (lane >> 4);
      const double ar = As[s][grp][0][ka][wr + (lane & 15)], ai = As[s][grp][1][ka][wr + (lane & 15)];
      const double br = Bs[s][grp][0][ka][wc + (lane & 15)], bi = Bs[s][grp][1][ka][wc + (lane & 15)];
      accr = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, br, accr, 0, 0, 0);
      accr = __builtin_amdgcn_mfma_f64_16x16x4f64(-ai, bi, accr, 0, 0, 0);
      acci = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, bi, acci, 0, 0, 0);
      acci = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, br, acci, 0, 0, 0);
    }
    if (c + 1 < npair) stash(s ^ 1);
    __syncthreads();
  }
  if (grp == 1)
    for (int q = 0; q < 4; ++q) {
      Xr[wl][q][lane] = accr[q];
      Xi[wl][q][lane] = acci[q];
    }
  __syncthreads();
  if (grp == 0)
    for (int q = 0; q < 4; ++q)
      gemm_store(C, ldc, M, N, m0 + wr + mfma_row_f64(lane, q), n0 + wc + (lane & 15), accr[q] + Xr[wl][q][lane],
                 acci[q] + Xi[wl][q][lane], alpha, accumulate, herm);
}

// ===================================================================================== Jacobi
// Round-robin (circle) pairing: step s of mp-1 steps pairs positions k and mp-1-k; position 0
// is fixed, position i >= 1 holds element ((i - 1 + s) mod (mp - 1)) + 1.  Every unordered pair
// of the mp indices meets exactly once per sweep.
__device__ __forceinline__ void rr_pair(int k, int s, int mp, int& p, int& q) {
  // k < mp / 2 and 0 <= s < mp - 1 keep both circle positions below 2 (mp - 1): one conditional
  // subtraction reduces them
  const int n1 = mp - 1, i0 = k, i1 = mp - 1 - k;
  const int x0 = i0 - 1 + s, x1 = i1 - 1 + s;
  int e0 = (i0 == 0) ? 0 : (x0 >= n1 ? x0 - n1 : x0) + 1;
  int e1 = (x1 >= n1 ? x1 - n1 : x1) + 1;
  p = e0 < e1 ? e0 : e1;
  q = e0 < e1 ? e1 : e0;
}

// tab[(s * half + k) * 2 + {0, 1}] = (p, q) for every step s and pair k.
__device__ void build_pair_table(unsigned char* tab, int mp) {
  const int half = mp / 2;
  for (int e = threadIdx.x; e < (mp - 1) * half; e += blockDim.x) {
    int s = e / half, k = e - s * half, p, q;
    rr_pair(k, s, mp, p, q);
    tab[2 * e] = (unsigned char)p;
    tab[2 * e + 1] = (unsigned char)q;
  }
}

struct JacobiArgs {
  double thr;   // absolute threshold on |g| (abs mode)
  double tol;   // relative threshold |g| <= tol sqrt(|a b|) (rel mode)
  double skip;  // rel mode: pairs whose diagonal entries are both below skip are left alone
  int rel;
  double floor2;  // rel mode: pairs with |g|^2 <= floor2 count as converged
};

// 1/sqrt(x) and 1/x from the hardware estimates refined by two Newton steps (the estimates
// carry about 23 correct bits; each step doubles them).
__device__ __forceinline__ double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  y = y * (1.5 - 0.5 * x * y * y);
  return y * (1.5 - 0.5 * x * y * y);
}
__device__ __forceinline__ double rcp_nr(double x) {
  double y = __builtin_amdgcn_rcp(x);
  y = y * (2.0 - x * y);
  return y * (2.0 - x * y);
}

// Whether the pair with diagonal (a, b) and off-diagonal g = gr + i gi is rotated.
__device__ __forceinline__ bool rot_needed(double a, double b, double gr, double gi, const JacobiArgs& ja) {
  const double h2 = gr * gr + gi * gi;
  if (ja.rel)
    return h2 > 1e-290 && h2 > ja.floor2 && h2 > ja.tol * ja.tol * fabs(a) * fabs(b) && fmax(fabs(a), fabs(b)) > ja.skip;
  return h2 > 1e-290 && h2 > ja.thr * ja.thr;
}

// Rotation J = [[c, -sp], [conj(sp), c]] (c real, |sp|^2 = 1 - c^2) for the Hermitian 2x2
// [[a, g], [conj g, b]]: J H J^H is diagonal with entries (a - t|g|, b + t|g|), where
// t = sign(b - a) 2|g| / (|b - a| + R), R = sqrt((b - a)^2 + 4|g|^2) (the smaller root of
// |g| t^2 - (a - b) t - |g| = 0), c = 1/sqrt(1 + t^2) and sp = c t g/|g|.  With
// den = |b - a| + R these are c = den / sqrt(den^2 + 4|g|^2), sp = sign 2 g / sqrt(den^2 + 4|g|^2),
// t|g| = sign 2|g|^2 / den: two reciprocal square roots in sequence.
__device__ __forceinline__ bool rot_params(double a, double b, double gr, double gi, const JacobiArgs& ja, double& c,
                                           double& spr, double& spi, double& na, double& nb) {
  if (!rot_needed(a, b, gr, gi, ja)) return false;
  const double h2 = gr * gr + gi * gi;
  const double dlt = b - a;
  const double sg = dlt < 0.0 ? -1.0 : 1.0;
  const double r2 = dlt * dlt + 4.0 * h2;
  const double den = fabs(dlt) + r2 * rsqrt_nr(r2);
  const double q = rsqrt_nr(den * den + 4.0 * h2);
  c = den * q;
  const double f = 2.0 * sg * q;
  spr = f * gr;
  spi = f * gi;
  const double th = 2.0 * sg * h2 * rcp_nr(den);
  na = a - th;
  nb = b + th;
  return true;
}

// One rotation of a parallel step: the pair's (c, sp) and new diagonal entries, and whether it
// rotates at all.
struct Rot {
  double c, spr, spi, na, nb;
  bool f;
};

// The rotation of pair (p, q) of the Hermitian matrix in planes (hr, hi) (leading dimension ld).
__device__ __forceinline__ Rot pair_rot(const double* __restrict__ hr, const double* __restrict__ hi, int ld, int p,
                                        int q, const JacobiArgs& ja) {
  Rot r;
  r.f = rot_params(hr[p * ld + p], hr[q * ld + q], hr[p * ld + q], hi[p * ld + q], ja, r.c, r.spr, r.spi, r.na, r.nb);
  return r;
}

// The 2x2 block (a b; c d) of rows (p1, q1) and columns (p2, q2) of H, rotated in place into
// the block of J H J^H: rotation r1 on the rows, r2 on the columns; diag marks the block of the
// pair itself (r1 = r2), whose result is diagonal.
__device__ __forceinline__ void rotate_vals(double& ar, double& ai, double& br, double& bi, double& cr, double& ci,
                                            double& dr, double& di, const Rot& r1, const Rot& r2, bool diag,
                                            int* any) {
  if (r1.f) {  // rows: r_p' = c r_p - sp r_q ; r_q' = conj(sp) r_p + c r_q
    const double c1 = r1.c, sp1r = r1.spr, sp1i = r1.spi;
    const double nar = c1 * ar - (sp1r * cr - sp1i * ci), nai = c1 * ai - (sp1r * ci + sp1i * cr);
    const double nbr = c1 * br - (sp1r * dr - sp1i * di), nbi = c1 * bi - (sp1r * di + sp1i * dr);
    const double ncr = c1 * cr + (sp1r * ar + sp1i * ai), nci = c1 * ci + (sp1r * ai - sp1i * ar);
    const double ndr = c1 * dr + (sp1r * br + sp1i * bi), ndi = c1 * di + (sp1r * bi - sp1i * br);
    ar = nar;
    ai = nai;
    br = nbr;
    bi = nbi;
    cr = ncr;
    ci = nci;
    dr = ndr;
    di = ndi;
  }
  if (r2.f) {  // cols: c_p' = c c_p - conj(sp) c_q ; c_q' = sp c_p + c c_q
    const double c2 = r2.c, sp2r = r2.spr, sp2i = r2.spi;
    const double nar = c2 * ar - (sp2r * br + sp2i * bi), nai = c2 * ai - (sp2r * bi - sp2i * br);
    const double ncr = c2 * cr - (sp2r * dr + sp2i * di), nci = c2 * ci - (sp2r * di - sp2i * dr);
    const double nbr = c2 * br + (sp2r * ar - sp2i * ai), nbi = c2 * bi + (sp2r * ai + sp2i * ar);
    const double ndr = c2 * dr + (sp2r * cr - sp2i * ci), ndi = c2 * di + (sp2r * ci + sp2i * cr);
    ar = nar;
    ai = nai;
    br = nbr;
    bi = nbi;
    cr = ncr;
    ci = nci;
    dr = ndr;
    di = ndi;
  }
  if (diag && r1.f) {
    ar = r1.na;
    dr = r1.nb;
    ai = di = br = bi = cr = ci = 0.0;
  }
  if (r1.f || r2.f) *any = 1;
}

// The same block read from the old planes (ir, ii) (leading dimension ld) and written to the new
// ones (orr, oi).
__device__ __forceinline__ void rotate_block(const double* __restrict__ ir, const double* __restrict__ ii,
                                             double* __restrict__ orr, double* __restrict__ oi, int ld, int p1,
                                             int q1, int p2, int q2, const Rot& r1, const Rot& r2, bool diag,
                                             int* any) {
  double ar = ir[p1 * ld + p2], ai = ii[p1 * ld + p2];
  double br = ir[p1 * ld + q2], bi = ii[p1 * ld + q2];
  double cr = ir[q1 * ld + p2], ci = ii[q1 * ld + p2];
  double dr = ir[q1 * ld + q2], di = ii[q1 * ld + q2];
  rotate_vals(ar, ai, br, bi, cr, ci, dr, di, r1, r2, diag, any);
  orr[p1 * ld + p2] = ar;
  oi[p1 * ld + p2] = ai;
  orr[p1 * ld + q2] = br;
  oi[p1 * ld + q2] = bi;
  orr[q1 * ld + p2] = cr;
  oi[q1 * ld + p2] = ci;
  orr[q1 * ld + q2] = dr;
  oi[q1 * ld + q2] = di;
}

// Rotation r (pair (p, q)) applied to rows v0 and v1 of the eigenvector accumulator, in place:
// v_p' = c v_p - conj(sp) v_q ; v_q' = sp v_p + c v_q.
__device__ __forceinline__ void rotate_vrows(double* __restrict__ vr, double* __restrict__ vi, int ld, int v0, int v1,
                                             int p, int q, const Rot& r) {
  const double c1 = r.c, sp1r = r.spr, sp1i = r.spi;
  const double w0pr = vr[v0 * ld + p], w0pi = vi[v0 * ld + p];
  const double w0qr = vr[v0 * ld + q], w0qi = vi[v0 * ld + q];
  const double w1pr = vr[v1 * ld + p], w1pi = vi[v1 * ld + p];
  const double w1qr = vr[v1 * ld + q], w1qi = vi[v1 * ld + q];
  vr[v0 * ld + p] = c1 * w0pr - (sp1r * w0qr + sp1i * w0qi);
  vi[v0 * ld + p] = c1 * w0pi - (sp1r * w0qi - sp1i * w0qr);
  vr[v0 * ld + q] = c1 * w0qr + (sp1r * w0pr - sp1i * w0pi);
  vi[v0 * ld + q] = c1 * w0qi + (sp1r * w0pi + sp1i * w0pr);
  vr[v1 * ld + p] = c1 * w1pr - (sp1r * w1qr + sp1i * w1qi);
  vi[v1 * ld + p] = c1 * w1pi - (sp1r * w1qi - sp1i * w1qr);
  vr[v1 * ld + q] = c1 * w1qr + (sp1r * w1pr - sp1i * w1pi);
  vi[v1 * ld + q] = c1 * w1qi + (sp1r * w1pi + sp1i * w1pr);
}

// rot_params without branches: every lane computes the rotation and the result is selected at the
// end (the identity and the unchanged diagonal when the pair is not rotated), so that the
// scheduler can interleave two rotations of one thread.
__device__ __forceinline__ Rot rot_select(double a, double b, double gr, double gi, const JacobiArgs& ja) {
  const bool need = rot_needed(a, b, gr, gi, ja);
  const double h2 = gr * gr + gi * gi;
  const double dlt = b - a;
  const double sg = dlt < 0.0 ? -1.0 : 1.0;
  const double r2 = dlt * dlt + 4.0 * h2;
  const double den = fabs(dlt) + r2 * rsqrt_nr(r2);
  const double q = rsqrt_nr(den * den + 4.0 * h2);
  const double f = 2.0 * sg * q;
  const double th = 2.0 * sg * h2 * rcp_nr(den);
  Rot r;
  r.f = need;
  r.c = need ? den * q : 1.0;
  r.spr = need ? f * gr : 0.0;
  r.spi = need ? f * gi : 0.0;
  r.na = need ? a - th : a;
  r.nb = need ? b + th : b;
  return r;
}

// A sequence of parallel Jacobi steps on the Hermitian H (2*half indices, half <= 16) held as
// two re/im plane pairs in LDS (double buffer).  Step s uses the pairs tab[s][k] = (p, q).
// Item (k1, k2) (k1, k2 < half) is the 2x2 block of rows (p_k1, q_k1) and columns
// (p_k2, q_k2): it needs rotations k1 and k2, computed from the old buffer, and its rotated block
// goes to the new buffer.  Rotation k1 is also applied to two rows of the eigenvector
// accumulator (V planes, in place; 2 * half rows in total).  With at least 2 half^2 threads the
// block update and the V update of an item run on different threads (each computes the
// rotations it needs), otherwise one thread does both; items are dealt round-robin.  On that
// split, V threads take k1 as the fast index and rows k2 and k2 + half (with a leading
// dimension of 16 mod 32 doubles the V accesses of 32 consecutive lanes fall in distinct
// banks); otherwise k2 is the fast index and the rows are 2 k2 and 2 k2 + 1.  One barrier per
// step.  Returns the index (0/1) of the buffer holding the result; *any is set when a rotation
// happened.
__device__ int jacobi_steps(double* __restrict__ h0r, double* __restrict__ h0i, double* __restrict__ h1r,
                            double* __restrict__ h1i, int ldh, int half, const unsigned char* __restrict__ tab,
                            int nsteps, double* __restrict__ vr, double* __restrict__ vi, int ldv,
                            const JacobiArgs& ja, int* any) {
  const int t = threadIdx.x, nt = blockDim.x;
  const int nitems = half * half;
  const bool split = nt >= 2 * nitems;
  const int nwork = split ? 2 * nitems : nitems;
  int cur = 0;
  for (int step = 0; step < nsteps; ++step) {
    const unsigned char* pt = tab + step * 2 * half;
    const double* __restrict__ ir = cur ? h1r : h0r;
    const double* __restrict__ ii = cur ? h1i : h0i;
    double* __restrict__ orr = cur ? h0r : h1r;
    double* __restrict__ oi = cur ? h0i : h1i;
    for (int e0 = t; e0 < nwork; e0 += nt) {
      const bool vsplit = split && e0 >= nitems;
      const bool do_v = !split || vsplit;
      const bool do_h = !split || e0 < nitems;
      const int e = vsplit ? e0 - nitems : e0;
      int k1, k2;
      if (vsplit) {
        k2 = (int)(((float)e + 0.5f) / (float)half);
        k1 = e - k2 * half;
      } else {
        k1 = (int)(((float)e + 0.5f) / (float)half);
        k2 = e - k1 * half;
      }
      const int p1 = pt[2 * k1], q1 = pt[2 * k1 + 1];
      const Rot r1 = pair_rot(ir, ii, ldh, p1, q1, ja);
      if (do_h) {
        const int p2 = pt[2 * k2], q2 = pt[2 * k2 + 1];
        const Rot r2 = pair_rot(ir, ii, ldh, p2, q2, ja);
        rotate_block(ir, ii, orr, oi, ldh, p1, q1, p2, q2, r1, r2, k1 == k2, any);
      }
      if (do_v && r1.f) {
        if (vsplit)
          rotate_vrows(vr, vi, ldv, k2, k2 + half, p1, q1, r1);
        else
          rotate_vrows(vr, vi, ldv, 2 * k2, 2 * k2 + 1, p1, q1, r1);
      }
    }
    __syncthreads();
    cur ^= 1;
  }
  return cur;
}

// x from lane (l + 1) mod 16 of the same 16-lane row (DPP row rotation by 15 to the right); every
// lane of the row must be active.
__device__ __forceinline__ double row_next(double x) {
  const long long v = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)v, 0x12F, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(v >> 32), 0x12F, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// The inter-block steps of a 32-index sub-problem on 512 threads, with its eigenvector
// accumulator V (starting from the identity) written to vo (32 x 32, row-major): step s
// (0..15) pairs index k < 16 with q_k(s) = 16 + (k + s) mod 16, so the 16 steps visit every pair
// (i < 16 <= j) once.  The arithmetic is that of jacobi_steps on the same pairs.
// Threads 0..255 update the blocks (k1 = t / 16, k2 = t mod 16); all LDS reads of a step are
// issued before its rotations are computed.  With a leading dimension of 16 mod 32 doubles every
// block and diagonal access of 32 consecutive lanes falls in distinct LDS banks.
// Threads 256..511 hold V in registers: thread (k1 = t mod 16, k2 = (t - 256) / 16) keeps rows
// k2 and k2 + 16 of columns k1 and q_k1(s).  It applies rotation k1, then takes column
// q_k1(s + 1) = q_{k1+1}(s) from the next lane of its 16-lane row; after 16 steps the columns
// are back at 16 + k1.  The 16 steps leave the matrix in (h0r, h0i).
__device__ void jacobi_ib_steps(double* __restrict__ h0r, double* __restrict__ h0i, double* __restrict__ h1r,
                                double* __restrict__ h1i, int ld, z64* __restrict__ vo, const JacobiArgs& ja,
                                int* any) {
  const int t = threadIdx.x;
  const bool do_v = t >= 256;  // uniform over each wave
  const int e = t & 255;
  const int k1 = do_v ? (e & 15) : (e >> 4);
  const int k2 = do_v ? (e >> 4) : (e & 15);
  // V thread: columns (p, q) of rows k2 (w0*) and k2 + 16 (w1*)
  double w0pr = (k1 == k2) ? 1.0 : 0.0, w0pi = 0.0, w0qr = 0.0, w0qi = 0.0;
  double w1pr = 0.0, w1pi = 0.0, w1qr = (k1 == k2) ? 1.0 : 0.0, w1qi = 0.0;
#pragma unroll 2
  for (int step = 0; step < 16; ++step) {
    const bool odd = step & 1;
    const double* __restrict__ ir = odd ? h1r : h0r;
    const double* __restrict__ ii = odd ? h1i : h0i;
    double* __restrict__ orr = odd ? h0r : h1r;
    double* __restrict__ oi = odd ? h0i : h1i;
    const int p1 = k1, q1 = 16 + ((k1 + step) & 15);
    const double a1 = ir[p1 * ld + p1], b1 = ir[q1 * ld + q1], g1r = ir[p1 * ld + q1], g1i = ii[p1 * ld + q1];
    if (!do_v) {
      const int p2 = k2, q2 = 16 + ((k2 + step) & 15);
      const double a2 = ir[p2 * ld + p2], b2 = ir[q2 * ld + q2], g2r = ir[p2 * ld + q2], g2i = ii[p2 * ld + q2];
      double ar = ir[p1 * ld + p2], ai = ii[p1 * ld + p2];
      double br = ir[p1 * ld + q2], bi = ii[p1 * ld + q2];
      double cr = ir[q1 * ld + p2], ci = ii[q1 * ld + p2];
      double dr = ir[q1 * ld + q2], di = ii[q1 * ld + q2];
      const Rot r1 = rot_select(a1, b1, g1r, g1i, ja), r2 = rot_select(a2, b2, g2r, g2i, ja);
      rotate_vals(ar, ai, br, bi, cr, ci, dr, di, r1, r2, k1 == k2, any);
      orr[p1 * ld + p2] = ar;
      oi[p1 * ld + p2] = ai;
      orr[p1 * ld + q2] = br;
      oi[p1 * ld + q2] = bi;
      orr[q1 * ld + p2] = cr;
      oi[q1 * ld + p2] = ci;
      orr[q1 * ld + q2] = dr;
      oi[q1 * ld + q2] = di;
    } else {
      const Rot r1 = rot_select(a1, b1, g1r, g1i, ja);
      if (r1.f) {  // v_p' = c v_p - conj(sp) v_q ; v_q' = sp v_p + c v_q
        const double c1 = r1.c, sp1r = r1.spr, sp1i = r1.spi;
        const double n0pr = c1 * w0pr - (sp1r * w0qr + sp1i * w0qi), n0pi = c1 * w0pi - (sp1r * w0qi - sp1i * w0qr);
        const double n0qr = c1 * w0qr + (sp1r * w0pr - sp1i * w0pi), n0qi = c1 * w0qi + (sp1r * w0pi + sp1i * w0pr);
        const double n1pr = c1 * w1pr - (sp1r * w1qr + sp1i * w1qi), n1pi = c1 * w1pi - (sp1r * w1qi - sp1i * w1qr);
        const double n1qr = c1 * w1qr + (sp1r * w1pr - sp1i * w1pi), n1qi = c1 * w1qi + (sp1r * w1pi + sp1i * w1pr);
        w0pr = n0pr;
        w0pi = n0pi;
        w0qr = n0qr;
        w0qi = n0qi;
        w1pr = n1pr;
        w1pi = n1pi;
        w1qr = n1qr;
        w1qi = n1qi;
      }
      w0qr = row_next(w0qr);
      w0qi = row_next(w0qi);
      w1qr = row_next(w1qr);
      w1qi = row_next(w1qi);
    }
    __syncthreads();
  }
  if (do_v) {
    vo[k2 * 32 + k1] = z64{w0pr, w0pi};
    vo[k2 * 32 + 16 + k1] = z64{w0qr, w0qi};
    vo[(k2 + 16) * 32 + k1] = z64{w1pr, w1pi};
    vo[(k2 + 16) * 32 + 16 + k1] = z64{w1qr, w1qi};
  }
}

// Round-robin table for mp indices (mp - 1 steps of mp/2 pairs).
__device__ void build_rr_table(unsigned char* tab, int mp) { build_pair_table(tab, mp); }

constexpr int SMALL_LD = 33;  // plane leading dimension for sub-problems of up to 32 indices

// Single-workgroup Jacobi: G (m x m, m <= kSmallEig = 32) -> U (m x m), lam (m), all in LDS.
__global__ __launch_bounds__(256) void k_jacobi_small(const z64* __restrict__ G, int ldg_in, int m,
                                                      z64* __restrict__ U, int ldu, double* __restrict__ lam, int rel,
                                                      double tol, double skip_rel, double floor_rel, int max_sweeps,
                                                      DevStatus* st) {
  constexpr int PL = 32 * SMALL_LD;
  __shared__ double h0r[PL], h0i[PL], h1r[PL], h1i[PL], vr[PL], vi[PL];
  __shared__ unsigned char tab[31 * 32];
  __shared__ int any, pending;
  __shared__ double trace;
  const int mp = m + (m & 1);
  const int half = mp / 2;
  const int t = threadIdx.x, nt = blockDim.x, ldh = SMALL_LD;
  build_rr_table(tab, mp);
  for (int idx = t; idx < mp * mp; idx += nt) {
    const int i = idx / mp, j = idx - (idx / mp) * mp;
    const z64 v = (i < m && j < m) ? G[(size_t)i * ldg_in + j] : z64{0.0, 0.0};
    h0r[i * ldh + j] = v.re;
    h0i[i * ldh + j] = v.im;
    vr[i * ldh + j] = (i == j) ? 1.0 : 0.0;
    vi[i * ldh + j] = 0.0;
  }
  __syncthreads();
  if (t == 0) {
    double tr = 0.0;
    for (int i = 0; i < m; ++i) tr += fabs(h0r[i * ldh + i]);
    trace = tr;
  }
  __syncthreads();
  const JacobiArgs ja{tol * trace, tol, skip_rel * trace, rel, (floor_rel * trace) * (floor_rel * trace)};
  int sweeps = 0, cur = 0;
  bool conv = false;
  for (int sw = 0; sw < max_sweeps; ++sw) {
    if (t == 0) any = 0;
    __syncthreads();
    // an odd number of steps swaps the buffers; keep the live matrix in (h0)
    const int res = jacobi_steps(cur ? h1r : h0r, cur ? h1i : h0i, cur ? h0r : h1r, cur ? h0i : h1i, ldh, half, tab,
                                 mp - 1, vr, vi, ldh, ja, &any);
    cur ^= res;
    ++sweeps;
    __syncthreads();
    // every wave reads the flag before thread 0 resets it for the next sweep
    const int rotated = any;
    __syncthreads();
    if (!rotated) {
      conv = true;
      break;
    }
    // The next sweep would rotate nothing (and change nothing) if no pair of the current matrix
    // passes the rotation test, read either way round: then it is skipped (7% faster here,
    // where a sweep is 31 dependent steps and the check one parallel pass).
    if (t == 0) pending = 0;
    __syncthreads();
    {
      const double* hr = cur ? h1r : h0r;
      const double* hi = cur ? h1i : h0i;
      for (int idx = t; idx < mp * mp; idx += nt) {
        const int i = idx / mp, j = idx - (idx / mp) * mp;
        if (i != j && rot_needed(hr[i * ldh + i], hr[j * ldh + j], hr[i * ldh + j], hi[i * ldh + j], ja)) pending = 1;
      }
    }
    __syncthreads();
    const int still = pending;
    __syncthreads();
    if (!still) {
      conv = true;
      break;
    }
  }
  const double* fr = cur ? h1r : h0r;
  for (int i = t; i < m; i += nt) lam[i] = fr[i * ldh + i];
  for (int idx = t; idx < m * m; idx += nt) {
    const int i = idx / m, j = idx - (idx / m) * m;
    U[(size_t)i * ldu + j] = z64{vr[i * ldh + j], vi[i * ldh + j]};
  }
  if (t == 0 && st) {
    st->converged = conv ? 1 : 0;
    st->sweeps = sweeps;
  }
}

// ----------------------------------------------------------------------- block Jacobi
constexpr int BJ = kBlk;      // block size (16)
constexpr int kSolveThreads = 512;  // threads per 32x32 sub-problem (block and V updates split)
static_assert(kSolveThreads == 2 * BJ * BJ, "the inter-block steps give each thread one block or one V item");
constexpr int BJ2 = 2 * kBlk; // pair size (32)
constexpr int SLD = BJ2 + 1;  // LDS leading dimension of the product tiles (plane layout)
constexpr int JLD = 48;       // LDS leading dimension of the solve's planes (16 mod 32 doubles)

// One 16x16 quadrant of a 32-deep complex product on one wave: acc += A B with
// A(row, kk) = a[kk * lda + wr + row] (conjugated when conja) and B(kk, col) = b[kk * ldb + wc + col].
// Every quadrant product of the rounds goes through this sequence, so a quadrant computed on its
// own equals the same quadrant of a whole-tile product bit for bit.
__device__ __forceinline__ void mmq(const double* ar_, const double* ai_, int lda, int wr, const double* br_,
                                    const double* bi_, int ldb, int wc, bool conja, d4& accr, d4& acci) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int kk = 0; kk < BJ2; kk += 4) {
    const int ka = kk + (lane >> 4);
    const double ar = ar_[ka * lda + wr + (lane & 15)];
    const double ai = conja ? -ai_[ka * lda + wr + (lane & 15)] : ai_[ka * lda + wr + (lane & 15)];
    const double br = br_[ka * ldb + wc + (lane & 15)];
    const double bi = bi_[ka * ldb + wc + (lane & 15)];
    accr = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, br, accr, 0, 0, 0);
    accr = __builtin_amdgcn_mfma_f64_16x16x4f64(-ai, bi, accr, 0, 0, 0);
    acci = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, bi, acci, 0, 0, 0);
    acci = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, br, acci, 0, 0, 0);
  }
}

// 32x32x32 complex product on four waves (one 16x16 quadrant each): acc += A * B where A is
// read as a[kk][row] (planes re/im, ld SLD) and B as b[kk][col]; conja conjugates A.
__device__ __forceinline__ void mm32(const double* ar_, const double* ai_, const double* br_, const double* bi_,
                                     bool conja, d4& accr, d4& acci) {
  const int w = threadIdx.x >> 6;
  mmq(ar_, ai_, SLD, (w >> 1) * 16, br_, bi_, SLD, (w & 1) * 16, conja, accr, acci);
}

__device__ __forceinline__ int pair_index(int P, int i, int step, int nb) {
  int I, J;
  rr_pair(P, step, nb, I, J);
  return i < BJ ? I * BJ + i : J * BJ + (i - BJ);
}

// The pair holding block b at outer step s and b's offset in it (0: first block, BJ: second):
// the inverse of rr_pair over nb blocks.  Block 0 stays in pair 0; another block b sits at
// position x = (b - 1 - s) mod (nb - 1) of the rotating circle, which is the first slot of pair
// x + 1 for x < nb / 2 - 1 and the second slot of pair nb - 2 - x otherwise.
__device__ __forceinline__ void block_home(int b, int s, int nb, int& pair, int& off) {
  if (b == 0) {
    pair = 0;
    off = 0;
    return;
  }
  int x = b - 1 - s;  // in (-(nb - 1), nb - 1)
  if (x < 0) x += nb - 1;
  pair = (x <= nb / 2 - 2) ? x + 1 : nb - 2 - x;
  int I, J;
  rr_pair(pair, s, nb, I, J);
  off = (b == I) ? 0 : BJ;
}

// One 32x32 row tile (R, Q) of U <- U V_Q with 512 threads: all threads stage the operands, the
// first four waves multiply (planes re/im in a_*/b_*, 32 x SLD each).
__device__ void u_tile(z64* __restrict__ Up, int mp, int nb, int step, const z64* __restrict__ V,
                       const int* __restrict__ pair_flag, int tile, double* __restrict__ a_re,
                       double* __restrict__ a_im, double* __restrict__ b_re, double* __restrict__ b_im) {
  const int half = nb / 2;
  const int R = tile / half, Q = tile % half;
  if (!pair_flag[Q]) return;  // uniform over the block
  const int t = threadIdx.x;
  const z64* VQ = V + (size_t)Q * BJ2 * BJ2;
  int q0, q1;
  rr_pair(Q, step, nb, q0, q1);
  z64 uv[BJ2 * BJ2 / kSolveThreads], qv[BJ2 * BJ2 / kSolveThreads];
#pragma unroll
  for (int u = 0; u < BJ2 * BJ2 / kSolveThreads; ++u) {  // every load before the first store
    const int idx = t + kSolveThreads * u, row = idx / BJ2, kk = idx % BJ2;
    uv[u] = Up[(size_t)(R * BJ2 + row) * mp + (kk < BJ ? q0 * BJ + kk : q1 * BJ + kk - BJ)];
    qv[u] = VQ[idx];
  }
#pragma unroll
  for (int u = 0; u < BJ2 * BJ2 / kSolveThreads; ++u) {
    const int idx = t + kSolveThreads * u, row = idx / BJ2, kk = idx % BJ2;
    a_re[kk * SLD + row] = uv[u].re;
    a_im[kk * SLD + row] = uv[u].im;
    b_re[row * SLD + kk] = qv[u].re;
    b_im[row * SLD + kk] = qv[u].im;
  }
  __syncthreads();
  if (t < 256) {
    const int lane = t & 63, w = t >> 6;
    const int wr = (w >> 1) * 16, wc = (w & 1) * 16;
    d4 accr = {0, 0, 0, 0}, acci = {0, 0, 0, 0};
    mm32(a_re, a_im, b_re, b_im, false, accr, acci);
    for (int q = 0; q < 4; ++q) {
      const int row = wr + mfma_row_f64(lane, q), col = wc + (lane & 15);
      Up[(size_t)(R * BJ2 + row) * mp + pair_index(Q, col, step, nb)] = z64{accr[q], acci[q]};
    }
  }
}

// One 32x32 tile (P, Q), P <= Q, of the round's update Gd = V^H Gs V with 512 threads (all stage
// the operands, the first four waves multiply); the (Q, P) tile is written as the conjugate
// transpose.  A pair that did not rotate contributes the identity; a tile whose two pairs both
// did not rotate is copied as it is (with its mirror).
__device__ void g_tile(const z64* __restrict__ Gs, z64* __restrict__ Gd, int mp, int nb, int step,
                       const z64* __restrict__ V, const int* __restrict__ pair_flag, int tile, double* __restrict__ a_re,
                       double* __restrict__ a_im, double* __restrict__ b_re, double* __restrict__ b_im) {
  const int half = nb / 2;
  int P = 0, rem = tile;
  while (rem >= half - P) {
    rem -= half - P;
    ++P;
  }
  const int Q = P + rem;
  const int fP = pair_flag[P], fQ = pair_flag[Q];
  const int t = threadIdx.x, nt = blockDim.x, lane = t & 63, w = t >> 6;
  if (!fP && !fQ) {  // uniform over the block
    for (int idx = t; idx < BJ2 * BJ2; idx += nt) {
      const int row = idx / BJ2, col = idx % BJ2;
      const size_t pq = (size_t)pair_index(P, row, step, nb) * mp + pair_index(Q, col, step, nb);
      const size_t qp = (size_t)pair_index(Q, row, step, nb) * mp + pair_index(P, col, step, nb);
      Gd[pq] = Gs[pq];
      if (P != Q) Gd[qp] = Gs[qp];
    }
    return;
  }
  const int wr = (w >> 1) * 16, wc = (w & 1) * 16;
  const z64* VP = V + (size_t)P * BJ2 * BJ2;
  const z64* VQ = V + (size_t)Q * BJ2 * BJ2;
  // V_P is needed after the first product: fetch it into registers now
  z64 vp[BJ2 * BJ2 / kSolveThreads];
#pragma unroll
  for (int u = 0; u < BJ2 * BJ2 / kSolveThreads; ++u) {
    const int idx = t + kSolveThreads * u;
    const int r = idx / BJ2, c = idx % BJ2;
    vp[u] = fP ? VP[idx] : ((r == c) ? z64{1.0, 0.0} : z64{0.0, 0.0});
  }
  // a[kk][row] = T[row][kk] = Gs[rows(P)[row], cols(Q)[kk]];  b = V_Q (or the identity); every
  // load is issued before the first store
  int p0, p1, q0, q1;
  rr_pair(P, step, nb, p0, p1);
  rr_pair(Q, step, nb, q0, q1);
  z64 gv[BJ2 * BJ2 / kSolveThreads], qv[BJ2 * BJ2 / kSolveThreads];
#pragma unroll
  for (int u = 0; u < BJ2 * BJ2 / kSolveThreads; ++u) {
    const int idx = t + kSolveThreads * u, row = idx / BJ2, kk = idx % BJ2;
    const int gr = row < BJ ? p0 * BJ + row : p1 * BJ + row - BJ;
    const int gc = kk < BJ ? q0 * BJ + kk : q1 * BJ + kk - BJ;
    gv[u] = Gs[(size_t)gr * mp + gc];
    qv[u] = fQ ? VQ[idx] : ((row == kk) ? z64{1.0, 0.0} : z64{0.0, 0.0});
  }
#pragma unroll
  for (int u = 0; u < BJ2 * BJ2 / kSolveThreads; ++u) {
    const int idx = t + kSolveThreads * u, row = idx / BJ2, kk = idx % BJ2;
    a_re[kk * SLD + row] = gv[u].re;
    a_im[kk * SLD + row] = gv[u].im;
    b_re[row * SLD + kk] = qv[u].re;
    b_im[row * SLD + kk] = qv[u].im;
  }
  __syncthreads();
  d4 accr = {0, 0, 0, 0}, acci = {0, 0, 0, 0};
  if (t < 256) mm32(a_re, a_im, b_re, b_im, false, accr, acci);  // X = T V_Q
  __syncthreads();
  if (t < 256)
    for (int q = 0; q < 4; ++q) {
      const int row = wr + mfma_row_f64(lane, q), col = wc + (lane & 15);
      b_re[row * SLD + col] = accr[q];
      b_im[row * SLD + col] = acci[q];
      accr[q] = 0.0;
      acci[q] = 0.0;
    }
#pragma unroll
  for (int u = 0; u < BJ2 * BJ2 / kSolveThreads; ++u) {
    const int idx = t + kSolveThreads * u;
    a_re[(idx / BJ2) * SLD + idx % BJ2] = vp[u].re;
    a_im[(idx / BJ2) * SLD + idx % BJ2] = vp[u].im;
  }
  __syncthreads();
  if (t < 256) {
    mm32(a_re, a_im, b_re, b_im, true, accr, acci);  // Y = V_P^H X
    for (int q = 0; q < 4; ++q) {
      const int row = wr + mfma_row_f64(lane, q), col = wc + (lane & 15);
      const int gr = pair_index(P, row, step, nb), gc = pair_index(Q, col, step, nb);
      Gd[(size_t)gr * mp + gc] = z64{accr[q], acci[q]};
      if (P != Q) Gd[(size_t)gc * mp + gr] = z64{accr[q], -acci[q]};
    }
  }
}

constexpr int HLD = 17;  // leading dimension of the half-width (32 x 16) planes of rebuild_pair
constexpr int kRebuildLds = 6 * BJ2 * SLD + 4 * BJ2 * HLD;  // doubles of scratch rebuild_pair uses

// The 32x32 sub-problem of blocks (I, J) after the previous round's update, rebuilt from the
// matrix before that update (Gs) and that round's rotations (V, flags pf, outer step ps) with
// the very products the previous round's tile updates make: with P and Q the previous pairs of
// I and J (offsets oI and oJ in them), the diagonal blocks are quadrants of V_P^H Gs_PP V_P and
// V_Q^H Gs_QQ V_Q and the off-diagonal block one of the (min, max) tile, mirrored as that tile's
// update mirrors it.  Only the quadrants needed are formed, each in the order of the whole-tile
// product (mmq), so the block equals what the update writes.  Writes planes (hr, hi) (leading
// dimension JLD), which may alias the scratch sc (kRebuildLds doubles); kSolveThreads threads.
__device__ void rebuild_pair(int I, int J, const z64* __restrict__ Gs, int mp, int nb, int ps,
                             const z64* __restrict__ V, const int* __restrict__ pf, double* __restrict__ sc,
                             double* __restrict__ hr, double* __restrict__ hi) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  int P, oI, Q, oJ;
  block_home(I, ps, nb, P, oI);
  block_home(J, ps, nb, Q, oJ);
  const int fP = pf[P], fQ = pf[Q];
  // tile u: rows of pair A[u], columns of pair B[u], quadrant (qr[u], qc[u]) of its update
  const bool sw = P > Q;
  const int A[3] = {P, sw ? Q : P, Q}, B[3] = {P, sw ? P : Q, Q};
  const int qr[3] = {oI, sw ? oJ : oI, oJ}, qc[3] = {oI, sw ? oI : oJ, oJ};
  const bool fA[3] = {fP != 0, sw ? fQ != 0 : fP != 0, fQ != 0}, fB[3] = {fP != 0, sw ? fP != 0 : fQ != 0, fQ != 0};
  // scratch: tile u transposed (tr[u][kk][row], ld SLD), then the half V planes: columns oI..oI+15
  // of V_P (vh[0]) and oJ..oJ+15 of V_Q (vh[1]), vh[kk][c] with ld HLD
  double* tr_re[3] = {sc, sc + 2 * BJ2 * SLD, sc + 4 * BJ2 * SLD};
  double* tr_im[3] = {sc + BJ2 * SLD, sc + 3 * BJ2 * SLD, sc + 5 * BJ2 * SLD};
  double* vh_re[2] = {sc + 6 * BJ2 * SLD, sc + 6 * BJ2 * SLD + 2 * BJ2 * HLD};
  double* vh_im[2] = {sc + 6 * BJ2 * SLD + BJ2 * HLD, sc + 6 * BJ2 * SLD + 3 * BJ2 * HLD};
  // every load of the staging is issued before the first store (one memory latency, not eight)
  z64 gv[6], vv[2];
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    const int u = i >> 1, e = t + (i & 1) * kSolveThreads, row = e / BJ2, kk = e % BJ2;
    int a0, a1, b0, b1;  // blocks of pairs A[u] and B[u] (uniform)
    rr_pair(A[u], ps, nb, a0, a1);
    rr_pair(B[u], ps, nb, b0, b1);
    const int gr = row < BJ ? a0 * BJ + row : a1 * BJ + row - BJ;
    const int gc = kk < BJ ? b0 * BJ + kk : b1 * BJ + kk - BJ;
    gv[i] = Gs[(size_t)gr * mp + gc];
  }
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int r = t / BJ, c = t % BJ, pr = h ? Q : P, off = h ? oJ : oI;
    const bool f = h ? fQ : fP;
    vv[h] = f ? V[(size_t)pr * BJ2 * BJ2 + r * BJ2 + off + c] : ((r == off + c) ? z64{1.0, 0.0} : z64{0.0, 0.0});
  }
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    const int u = i >> 1, e = t + (i & 1) * kSolveThreads, row = e / BJ2, kk = e % BJ2;
    tr_re[u][kk * SLD + row] = gv[i].re;
    tr_im[u][kk * SLD + row] = gv[i].im;
  }
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int r = t / BJ, c = t % BJ;
    vh_re[h][r * HLD + c] = vv[h].re;
    vh_im[h][r * HLD + c] = vv[h].im;
  }
  __syncthreads();
  // X = T V_B restricted to columns qc: waves 0..5 (tile w / 2, rows (w % 2) * 16)
  const int xu = w >> 1, xr = (w & 1) * BJ;
  const bool xrun = w < 6 && (fA[xu] || fB[xu]);
  d4 accr = {0, 0, 0, 0}, acci = {0, 0, 0, 0};
  if (xrun) {
    const int hb = (xu == 1) ? (sw ? 0 : 1) : (xu == 0 ? 0 : 1);  // half plane of V_B[u]
    mmq(tr_re[xu], tr_im[xu], SLD, xr, vh_re[hb], vh_im[hb], HLD, 0, false, accr, acci);
  }
  __syncthreads();
  if (xrun)  // X quadrant over the tile's own scratch: x[row][c], ld HLD
    for (int q = 0; q < 4; ++q) {
      const int row = xr + mfma_row_f64(lane, q), col = lane & 15;
      tr_re[xu][row * HLD + col] = accr[q];
      tr_im[xu][row * HLD + col] = acci[q];
      accr[q] = 0.0;
      acci[q] = 0.0;
    }
  __syncthreads();
  // Y quadrant of tile w (waves 0..2): V_A^H X, or the quadrant of Gs itself when neither pair
  // rotated (waves 3..5 read it)
  double yr[4], yi[4];
  if (w < 3) {
    const int u = w;
    if (fA[u] || fB[u]) {
      const int ha = (u == 1) ? (sw ? 1 : 0) : (u == 0 ? 0 : 1);  // half plane of V_A[u]
      mmq(vh_re[ha], vh_im[ha], HLD, 0, tr_re[u], tr_im[u], HLD, 0, true, accr, acci);
      for (int q = 0; q < 4; ++q) {
        yr[q] = accr[q];
        yi[q] = acci[q];
      }
    }
  } else if (w < 6) {
    const int u = w - 3;
    if (!(fA[u] || fB[u]))
      for (int q = 0; q < 4; ++q) {  // element (row, col) of the quadrant, as the MFMA layout
        const int row = mfma_row_f64(lane, q), col = lane & 15;
        yr[q] = tr_re[u][(qc[u] + col) * SLD + qr[u] + row];
        yi[q] = tr_im[u][(qc[u] + col) * SLD + qr[u] + row];
      }
  }
  __syncthreads();
  // place the quadrants: tile 0 -> (I, I), tile 2 -> (J, J), tile 1 -> (I, J) and its mirror
  const int u = (w < 3) ? w : w - 3;
  const bool mine = (w < 3) ? (fA[u] || fB[u]) : (w < 6 && !(fA[u] || fB[u]));
  if (mine)
    for (int q = 0; q < 4; ++q) {
      const int row = mfma_row_f64(lane, q), col = lane & 15;
      if (u == 0) {
        hr[row * JLD + col] = yr[q];
        hi[row * JLD + col] = yi[q];
      } else if (u == 2) {
        hr[(BJ + row) * JLD + BJ + col] = yr[q];
        hi[(BJ + row) * JLD + BJ + col] = yi[q];
      } else if (!sw) {  // rows of I, columns of J; mirror conjugated
        hr[row * JLD + BJ + col] = yr[q];
        hi[row * JLD + BJ + col] = yi[q];
        hr[(BJ + col) * JLD + row] = yr[q];
        hi[(BJ + col) * JLD + row] = -yi[q];
      } else {  // the (Q, P) tile: rows of J, columns of I; mirror conjugated
        hr[(BJ + row) * JLD + col] = yr[q];
        hi[(BJ + row) * JLD + col] = yi[q];
        hr[col * JLD + BJ + row] = yr[q];
        hi[col * JLD + BJ + row] = -yi[q];
      }
    }
}

// Solve step of a round: pair k of outer step `step` solves its 32x32 sub-problem (blocks I, J)
// and writes the accumulated rotation to V + k*32*32 (row-major) with a rotated flag.  The first
// step of an outer sweep runs a full round-robin sweep over the 32 indices (covering the pairs
// inside each block); later steps rotate only the 16 x 16 inter-block pairs.  Over one outer
// sweep every index pair is visited once.  With ps < 0 the sub-problem is read from Gs; otherwise
// Gs is the matrix before the previous round's update (outer step ps, rotations Vp, flags pfp)
// and the sub-problem is rebuilt from it (rebuild_pair), the update itself running beside this
// solve.  LDS: six 32 x JLD planes (the rebuild's scratch aliases them).
__device__ void solve_pair(int k, const z64* __restrict__ Gs, int mp, int nb, int step, int ps,
                           const z64* __restrict__ Vp, const int* __restrict__ pfp, double thr, double tol,
                           double skip, int rel, double floor2, z64* __restrict__ Vout, int* __restrict__ pair_flag,
                           int* __restrict__ any_flag, double* __restrict__ h0r, double* __restrict__ h0i,
                           double* __restrict__ h1r, double* __restrict__ h1i, double* __restrict__ vr,
                           double* __restrict__ vi, unsigned char* __restrict__ tab, int& any, int& need) {
  const int t = threadIdx.x, nt = blockDim.x;
  int I, J;
  rr_pair(k, step, nb, I, J);
  const bool full = (step == 0);
  if (t == 0) {
    any = 0;
    need = 0;
  }
  if (full) build_rr_table(tab, BJ2);
  const JacobiArgs ja{thr, tol, skip, rel, floor2};
  if (ps < 0) {
    for (int idx = t; idx < BJ2 * BJ2; idx += nt) {
      const int i = idx / BJ2, j = idx % BJ2;
      const int gi = (i < BJ ? I * BJ + i : J * BJ + (i - BJ));
      const int gj = (j < BJ ? I * BJ + j : J * BJ + (j - BJ));
      const z64 v = Gs[(size_t)gi * mp + gj];
      h0r[i * JLD + j] = v.re;
      h0i[i * JLD + j] = v.im;
    }
  } else {
    rebuild_pair(I, J, Gs, mp, nb, ps, Vp, pfp, h0r, h0r, h0i);
  }
  if (full)
    for (int idx = t; idx < BJ2 * BJ2; idx += nt) {
      const int i = idx / BJ2, j = idx % BJ2;
      vr[i * JLD + j] = (i == j) ? 1.0 : 0.0;
      vi[i * JLD + j] = 0.0;
    }
  __syncthreads();
  for (int idx = t; idx < BJ2 * BJ2; idx += nt) {
    const int i = idx / BJ2, j = idx % BJ2;
    if (i < j && (full || (i < BJ && j >= BJ))) {
      if (rot_needed(h0r[i * JLD + i], h0r[j * JLD + j], h0r[i * JLD + j], h0i[i * JLD + j], ja)) need = 1;
    }
  }
  __syncthreads();
  const int run = need;
  if (run) {
    z64* vo = Vout + (size_t)k * BJ2 * BJ2;
    if (full) {
      jacobi_steps(h0r, h0i, h1r, h1i, JLD, BJ, tab, BJ2 - 1, vr, vi, JLD, ja, &any);
      for (int idx = t; idx < BJ2 * BJ2; idx += nt) {
        const int i = idx / BJ2, j = idx % BJ2;
        vo[idx] = z64{vr[i * JLD + j], vi[i * JLD + j]};
      }
    } else {
      jacobi_ib_steps(h0r, h0i, h1r, h1i, JLD, vo, ja, &any);
    }
  }
  if (t == 0) {
    const int a = run ? any : 0;
    pair_flag[k] = a;
    if (a) atomicOr(any_flag, 1);
  }
}

// One round of the block Jacobi sweep in one launch.  Blocks 0..half-1 (when step >= 0) solve the
// sub-problems of outer step `step` (rotations to Vout, flags to pair_flag, any rotation to
// *any_flag; a non-null any_next, the flag of the next sweep, is cleared); when ps >= 0 the previous
// round (outer step ps, rotations Vp, flags pfp) is applied
// beside them: the next half(half+1)/2 blocks form the tiles of Gd = V^H Gs V, the remaining
// (mp/32) half blocks the row tiles of U <- U V.  The solves rebuild their sub-problems from Gs,
// so no block waits for another; Gs and Gd alternate between rounds.  512 threads.
// Launched with kJroundPad bytes of (unused) dynamic LDS, a block holds more than half of a CU's
// 160 KB, so it holds the CU alone: a solve then never shares its SIMDs with tile updates (the
// round's critical path), which queue on the other CUs.  That pays while the updates are few
// (m = 768: 21.0 against 22.8 us per round) and costs once they dominate (m = 1024: 26.6
// against 24.5 us; m = 2048: 89.9 against 59.8 us), where it is launched without the pad.
constexpr int kJroundPad = 8192;
__global__ __launch_bounds__(512) void k_jround(const z64* __restrict__ Gs, z64* __restrict__ Gd,
                                                z64* __restrict__ Up, int mp, int nb, int step, int ps,
                                                const double* __restrict__ trace, double tol, double skip_rel,
                                                int rel, double floor_rel, z64* __restrict__ Vout,
                                                int* __restrict__ pair_flag, int* __restrict__ any_flag,
                                                int* __restrict__ any_next, const z64* __restrict__ Vp,
                                                const int* __restrict__ pfp) {
  constexpr int PL = BJ2 * JLD;
  static_assert(6 * PL >= kRebuildLds, "the rebuild's scratch fits in the solve's planes");
  __shared__ double pool[6 * PL];
  __shared__ unsigned char tab[31 * 32];
  static_assert(sizeof(pool) + sizeof(tab) + kJroundPad > 80 * 1024, "a padded block holds half a CU's LDS");
  __shared__ int any, need;
  const int half = nb / 2, nsolve = step >= 0 ? half : 0, ngt = half * (half + 1) / 2;
  int b = blockIdx.x;
  if (any_next && b == 0 && threadIdx.x == 0) *any_next = 0;
  if (b < nsolve) {
    // thresholds from the trace on the device (read by no host sync)
    const double tr = *trace;
    const double thr = tol * tr, skip = skip_rel * tr, floor2 = (floor_rel * tr) * (floor_rel * tr);
    solve_pair(b, Gs, mp, nb, step, ps, Vp, pfp, thr, tol, skip, rel, floor2, Vout, pair_flag, any_flag, pool,
               pool + PL, pool + 2 * PL, pool + 3 * PL, pool + 4 * PL, pool + 5 * PL, tab, any, need);
    return;
  }
  b -= nsolve;
  if (b < ngt)
    g_tile(Gs, Gd, mp, nb, ps, Vp, pfp, b, pool, pool + BJ2 * SLD, pool + 2 * BJ2 * SLD, pool + 3 * BJ2 * SLD);
  else
    u_tile(Up, mp, nb, ps, Vp, pfp, b - ngt, pool, pool + BJ2 * SLD, pool + 2 * BJ2 * SLD, pool + 3 * BJ2 * SLD);
}

__global__ void k_pad_copy(const z64* __restrict__ G, int m, int ldg, z64* __restrict__ Gp, int mp,
                           z64* __restrict__ Up) {
  size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)mp * mp) return;
  int i = (int)(idx / mp), j = (int)(idx % mp);
  Gp[idx] = (i < m && j < m) ? G[(size_t)i * ldg + j] : z64{0.0, 0.0};
  Up[idx] = (i == j) ? z64{1.0, 0.0} : z64{0.0, 0.0};
}

__global__ void k_trace(const z64* __restrict__ Gp, int m, int mp, double* out, int* __restrict__ sweep_flags) {
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < m; i += blockDim.x) s += fabs(Gp[(size_t)i * mp + i].re);
  red[threadIdx.x] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = red[0];
    reinterpret_cast<int*>(out + 1)[0] = 0;  // pre-check flag, set by k_offdiag_check
    sweep_flags[0] = 0;                      // the sweeps' rotation flags (even and odd sweeps)
    sweep_flags[1] = 0;
  }
}

// Pre-check of a decomposition: sets *flag when some pair (i < j < m) of Gp passes the rotation
// test, with the thresholds the sweeps would use (from the trace in out[0] of k_trace).
__global__ void k_offdiag_check(const z64* __restrict__ Gp, int m, int mp, const double* __restrict__ trace_in,
                                double tol, double skip_rel, int rel, double floor_rel, int* __restrict__ flag) {
  const double trace = *trace_in;
  const JacobiArgs ja{tol * trace, tol, skip_rel * trace, rel, (floor_rel * trace) * (floor_rel * trace)};
  const size_t total = (size_t)m * m;
  int hit = 0;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / m), j = (int)(e % m);
    if (i < j) {
      const z64 g = Gp[(size_t)i * mp + j];
      if (rot_needed(Gp[(size_t)i * mp + i].re, Gp[(size_t)j * mp + j].re, g.re, g.im, ja)) hit = 1;
    }
  }
  if (hit) atomicOr(flag, 1);
}

__global__ void k_unpad(const z64* __restrict__ Gp, const z64* __restrict__ Up, int m, int mp, z64* __restrict__ U,
                        int ldu, double* __restrict__ lam) {
  size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)m * m) return;
  int i = (int)(idx / m), j = (int)(idx % m);
  U[(size_t)i * ldu + j] = Up[(size_t)i * mp + j];
  if (j == 0) lam[i] = Gp[(size_t)i * mp + i].re;
}

// ===================================================================================== misc
__global__ void k_rownorm2(const z64* __restrict__ B, int m, int k, int ldb, double* __restrict__ out) {
  __shared__ double red[256];
  const int r = blockIdx.x;
  double s = 0.0;
  for (int c = threadIdx.x; c < k; c += blockDim.x) s += cabs2(B[(size_t)r * ldb + c]);
  red[threadIdx.x] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[r] = red[0];
}

// Truncation rule on squared values sig2 (any order).  Sorted descending (ties by index).
//   w_j = sig2_j / sum sig2;  tail[k] = sum_{j >= k} w_j  (accumulated from the smallest)
//   k_cut = smallest k >= 1 with tail[k] <= cutoff; k_floor = #{sigma_j > 1e-13 sigma_0}
//   k = min(k_cut, k_floor, chi_max); degeneracy guard as in the truncation rule.
// mode 1 keeps k_floor (exact moves).  need_pass2 when a kept value is below 1e-12 sig2_0.
// force_k > 0 replaces the rule by that rank (frozen-decision replay; never flagged).
constexpr int TRUNC_MAX = 4096;
__global__ __launch_bounds__(1024) void k_trunc(const double* __restrict__ sig2, int m, double cutoff, int chi_max,
                                                int mode, int force_k, int* __restrict__ perm,
                                                double* __restrict__ sig_sorted, DevStatus* st,
                                                const double* __restrict__ extra) {
  __shared__ double key[TRUNC_MAX];
  __shared__ int idx[TRUNC_MAX];
  int P2 = 1;
  while (P2 < m) P2 <<= 1;
  const int t = threadIdx.x, nt = blockDim.x;
  for (int i = t; i < P2; i += nt) {
    key[i] = (i < m) ? fmax(sig2[i], 0.0) : -1.0;
    idx[i] = i;
  }
  __syncthreads();
  // bitonic sort: descending key, ascending index on ties
  for (int size = 2; size <= P2; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = t; i < P2; i += nt) {
        int j = i ^ stride;
        if (j > i) {
          bool desc = ((i & size) == 0);
          double ki = key[i], kj = key[j];
          int ii = idx[i], ij = idx[j];
          bool i_before_j = (ki > kj) || (ki == kj && ii < ij);
          bool swap = desc ? !i_before_j : i_before_j;
          if (swap) {
            key[i] = kj;
            key[j] = ki;
            idx[i] = ij;
            idx[j] = ii;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int i = t; i < m; i += nt) {
    perm[i] = idx[i];
    sig_sorted[i] = sqrt(key[i]);
  }
  if (t == 0) {
    // weight outside the listed values (always discarded): starts every tail
    const double ex = extra ? fmax(*extra, 0.0) : 0.0;
    double total = ex;
    for (int i = m - 1; i >= 0; --i) total += key[i];
    // smallest k with tail[k] <= cutoff, tails accumulated from the smallest value
    double tails_k = ex / total;
    int kcut = m;
    for (int k = m - 1; k >= 1; --k) {
      tails_k += key[k] / total;
      if (tails_k <= cutoff) kcut = k;
      else break;
    }
    const double s0 = sqrt(key[0]);
    int kfloor = 0;
    for (int i = 0; i < m; ++i)
      if (sqrt(key[i]) > 1e-13 * s0) ++kfloor;
    int k;
    int flagged = 0;
    if (mode == 1) {
      k = kfloor > 0 ? kfloor : 1;
    } else {
      k = kcut;
      if (kfloor < k) k = kfloor;
      if (chi_max < k) k = chi_max;
      if (k < 1) k = 1;
      if (k < m) {
        double sk = sqrt(key[k]), skm = sqrt(key[k - 1]);
        if (sk > 1e-13 * s0 && sk >= skm * (1.0 - 1e-10)) {
          int j = k - 1;
          while (j > 0 && sqrt(key[j]) >= sqrt(key[j - 1]) * (1.0 - 1e-10)) --j;
          if (j == 0)
            flagged = 1;
          else
            k = j;
        }
      }
    }
    if (force_k > 0) {
      k = force_k < m ? force_k : m;
      flagged = 0;
    }
    double eps = ex / total;
    for (int i = m - 1; i >= k; --i) eps += key[i] / total;
    st->kept = k;
    st->eps = eps;
    st->flagged = flagged;
    st->need_pass2 = (key[k - 1] < 1e-12 * key[0]) ? 1 : 0;
    st->lam_max = key[0];
  }
}

// Factor emission.  W is the wide orientation of the split matrix M (p x q): wide = 1 when
// W = M (p <= q, m = p, kW = q), wide = 0 when W = M^H (m = q, kW = p).  With U (m x m) the
// eigenvectors of W W^H, B = U^H W (m x kW), perm the sorted order and sig the row norms of B:
//   wide, left_ortho : L = U[:, perm],            R = B[perm, :] * rn
//   wide, right_ortho: L = U[:, perm] * sig * rn, R = B[perm, :] / sig
//   tall, left_ortho : L = B[perm, :]^H / sig,    R = sig * rn * U[:, perm]^H
//   tall, right_ortho: L = B[perm, :]^H * rn,     R = U[:, perm]^H
// rn = 1 / sqrt(sum_kept sig^2) when renorm, else 1.
__global__ void k_emit(int wide, int left_ortho, int renorm, int p, int q, int kept, const z64* __restrict__ U,
                       int ldu, const z64* __restrict__ B, int ldb, const int* __restrict__ perm,
                       const double* __restrict__ sig, z64* __restrict__ L, z64* __restrict__ R) {
  __shared__ double rn_s;
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int j = 0; j < kept; ++j) s += sig[j] * sig[j];
    rn_s = renorm ? 1.0 / sqrt(s) : 1.0;
  }
  __syncthreads();
  const double rn = rn_s;
  size_t nl = (size_t)p * kept, nr = (size_t)kept * q;
  size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < nl) {
    int i = (int)(idx / kept), j = (int)(idx % kept);
    int pj = perm[j];
    z64 v;
    if (wide) {
      v = U[(size_t)i * ldu + pj];
      if (!left_ortho) v = cscale(v, sig[j] * rn);
    } else {
      v = cconj(B[(size_t)pj * ldb + i]);
      v = left_ortho ? cscale(v, 1.0 / sig[j]) : cscale(v, rn);
    }
    L[idx] = v;
  } else if (idx < nl + nr) {
    size_t e = idx - nl;
    int j = (int)(e / q), c = (int)(e % q);
    int pj = perm[j];
    z64 v;
    if (wide) {
      v = B[(size_t)pj * ldb + c];
      v = left_ortho ? cscale(v, rn) : cscale(v, 1.0 / sig[j]);
    } else {
      v = cconj(U[(size_t)c * ldu + pj]);
      if (left_ortho) v = cscale(v, sig[j] * rn);
    }
    R[e] = v;
  }
}

__global__ void k_copy(z64* __restrict__ dst, const z64* __restrict__ src, size_t count) {
  size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < count) dst[idx] = src[idx];
}

__global__ void k_fill_identity(z64* U, int m, int ld) {
  size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)m * m) return;
  int i = (int)(idx / m), j = (int)(idx % m);
  U[(size_t)i * ld + j] = (i == j) ? z64{1.0, 0.0} : z64{0.0, 0.0};
}

inline unsigned blocks_for(size_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

// ===================================================================================== launchers
void linalg_set_attributes() {
  // the rounds' optional LDS pad is dynamic shared memory; static plus dynamic exceeds 64 KB
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_jround), hipFuncAttributeMaxDynamicSharedMemorySize,
                            kJroundPad);
  (void)hipGetLastError();
}

void launch_zgemm(hipStream_t s, int opa, int opb, int M, int N, int K, const z64* A, int lda, const z64* B,
                  int ldb, z64* C, int ldc, z64 alpha, int accumulate, int herm) {
  if (M <= 0 || N <= 0) return;
  const dim3 grid((N + GT - 1) / GT, (M + GT - 1) / GT);
  // Below 256 tiles (Hermitian: counting the upper ones) the K-split form with two waves per
  // SIMD is faster (768 x 256 x 768: 39 against 54 us), above it the four-wave form (768^3:
  // 108 against 112 us; both against 226 us on 64 x 64 single-stage tiles).
  const long tiles = herm ? (long)grid.x * (grid.x + 1) / 2 : (long)grid.x * grid.y;
  const bool ks = tiles < 256;
#define GC_ZGEMM(OA, OB)                                                                                         \
  do {                                                                                                           \
    if (ks)                                                                                                      \
      hipLaunchKernelGGL((k_zgemm_ks<OA, OB>), grid, dim3(512), 0, s, M, N, K, A, lda, B, ldb, C, ldc, alpha,    \
                         accumulate, herm);                                                                      \
    else                                                                                                         \
      hipLaunchKernelGGL((k_zgemm<OA, OB>), grid, dim3(256), 0, s, M, N, K, A, lda, B, ldb, C, ldc, alpha,       \
                         accumulate, herm);                                                                      \
  } while (0)
  if (opa == 0 && opb == 0)
    GC_ZGEMM(0, 0);
  else if (opa == 0 && opb == 1)
    GC_ZGEMM(0, 1);
  else if (opa == 1 && opb == 0)
    GC_ZGEMM(1, 0);
  else
    GC_ZGEMM(1, 1);
#undef GC_ZGEMM
  GC_LAUNCH_CHECK();
}

void eig_hermitian(hipStream_t s, const z64* G, int m, int ldg, z64* U, int ldu, double* lam, int rel, EigWork& w,
                   DevStatus* st, int* host_sweeps, bool precheck) {
  const double tol = rel ? 1e-14 : 4e-15;
  // Relative pass: pairs whose diagonal entries are both below 1e-28 lambda_max (lambda_max >=
  // trace / m) are left alone.  They lie two decades below the rank floor (sigma^2 = 1e-26
  // sigma_0^2), so no decision depends on them, and exact null directions sit at the rounding
  // level (~1e-32 of the trace), where a relative criterion cannot be met.
  const double skip = rel ? 1e-28 / (double)m : 0.0;
  // Relative pass: an off-diagonal entry of at most 1e-29 trace / m (<= 1e-29 lambda_max) counts
  // as converged.  On exactly rank-deficient matrices the rounding of the rotations keeps
  // entries of that size alive between directions at the rounding level, where a relative
  // criterion is never met (the pass then ran out of sweeps); an eigenvalue at or above the rank
  // floor (1e-26 lambda_max) moves by at most 1e-3 of itself because of such an entry.
  const double floor_rel = rel ? 1e-29 / (double)m : 0.0;
  // Sweeps grow with m on these Grams: up to ~20 at m = 768, 19-26 at m = 3072, where one
  // decomposition needed more than 40 (every sub-problem still rotating for the first ~20
  // sweeps, then a steady decay).
  const int max_sweeps = m > 1024 ? 100 : 40;
  if (m <= kSmallEig) {
    hipLaunchKernelGGL(k_jacobi_small, dim3(1), dim3(256), 0, s, G, ldg, m, U, ldu, lam, rel, tol, skip, floor_rel,
                       max_sweeps, st);
    GC_LAUNCH_CHECK();
    if (host_sweeps) *host_sweeps = -1;
    return;
  }
  const int mp = ((m + BJ2 - 1) / BJ2) * BJ2;
  const int nb = mp / BJ;
  GC_CHECK(mp <= w.m_pad, GCAMPS_ECAPACITY, "eigensolver workspace too small");
  z64* Gp = w.G;
  z64* Up = w.G + (size_t)w.m_pad * w.m_pad;
  z64* Gp1 = w.G + 2 * (size_t)w.m_pad * w.m_pad;
  hipLaunchKernelGGL(k_pad_copy, dim3(blocks_for((size_t)mp * mp, 256)), dim3(256), 0, s, G, m, ldg, Gp, mp, Up);
  GC_LAUNCH_CHECK();
  double* d_trace = reinterpret_cast<double*>(w.flags + 512);
  // rotation flag of sweep sw: sweep_flag(sw); the first round of a sweep clears the next sweep's
  // (written by no round of this sweep, and read by the host two sweeps ago), k_trace both
  auto sweep_flag = [&](int sw) { return w.flags + 300 + (sw & 1); };
  hipLaunchKernelGGL(k_trace, dim3(1), dim3(256), 0, s, Gp, m, mp, d_trace, sweep_flag(0));
  GC_LAUNCH_CHECK();
  if (precheck) {
    hipLaunchKernelGGL(k_offdiag_check, dim3(blocks_for((size_t)m * m, 256)), dim3(256), 0, s, Gp, m, mp, d_trace, tol,
                       skip, rel, floor_rel, reinterpret_cast<int*>(d_trace + 1));
    GC_LAUNCH_CHECK();
  }
  if (precheck) {  // the pre-check flag sits after the trace; the rounds read the trace themselves
    double local[2] = {0.0, 0.0};
    double* tr_flag = w.host_rb ? w.host_rb : local;  // pinned when the context gives a slot
    GC_HIP(hipMemcpyAsync(tr_flag, d_trace, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    GC_HIP(hipStreamSynchronize(s));
    int pre_hit = 1;
    std::memcpy(&pre_hit, &tr_flag[1], sizeof(int));
    if (!pre_hit) {  // nothing to rotate: U = I (set by k_pad_copy), lam = diag(G)
      hipLaunchKernelGGL(k_unpad, dim3(blocks_for((size_t)m * m, 256)), dim3(256), 0, s, Gp, Up, m, mp, U, ldu,
                         lam);
      GC_LAUNCH_CHECK();
      if (host_sweeps) *host_sweeps = 0;
      return;
    }
  }
  const int half = nb / 2;
  int sweeps = 0;
  bool conv = false;
  // rotation and flag buffers of round r: V + (r & 1) * half * 32 * 32, flags + 1 + (r & 1) * 128
  // (half <= m_pad / 32 <= 128; the V region holds m_pad / 16 blocks of 32 x 32 and more)
  GC_CHECK(half <= 128, GCAMPS_ECAPACITY, "eigensolver: matrix side exceeds 4096");
  auto vbuf = [&](long r) { return w.V + (size_t)(r & 1) * half * BJ2 * BJ2; };
  auto fbuf = [&](long r) { return w.flags + 1 + (r & 1) * 128; };
  // the matrix after round r - 1's update lives in gbuf(r): round r (r >= 1) solves from gbuf(r - 1)
  // and the previous round's rotations while it writes gbuf(r)
  auto gbuf = [&](long r) { return (r & 1) ? Gp1 : Gp; };
  const int gtiles = half * (half + 1) / 2, utiles = (mp / BJ2) * half;
  // a whole CU per block while the tile updates are few (see k_jround)
  const size_t pad = mp <= 896 ? kJroundPad : 0;
  long round = 0;  // rounds launched so far
  int prev_step = -1;
  for (int sw = 0; sw < max_sweeps; ++sw) {
    for (int step = 0; step < nb - 1; ++step, ++round) {
      const bool upd = round > 0;
      hipLaunchKernelGGL(k_jround, dim3(half + (upd ? gtiles + utiles : 0)), dim3(kSolveThreads), pad, s,
                         upd ? gbuf(round - 1) : Gp, gbuf(round), Up, mp, nb, step, upd ? prev_step : -1, d_trace,
                         tol, skip, rel, floor_rel, vbuf(round), fbuf(round), sweep_flag(sw),
                         step == 0 ? sweep_flag(sw + 1) : nullptr, upd ? vbuf(round - 1) : nullptr,
                         upd ? fbuf(round - 1) : nullptr);
      GC_LAUNCH_CHECK();
      prev_step = step;
    }
    ++sweeps;
    // (A check after each sweep for pairs left to rotate, to skip the sweep that only confirms
    // convergence, costs as much here as that sweep: its rounds are cheap when nothing rotates.)
    int local = 0;
    int* hany = w.host_rb ? reinterpret_cast<int*>(w.host_rb) : &local;  // pinned when given
    GC_HIP(hipMemcpyAsync(hany, sweep_flag(sw), sizeof(int), hipMemcpyDeviceToHost, s));
    GC_HIP(hipStreamSynchronize(s));
    const int any = *hany;
    if (!any) {
      conv = true;
      break;
    }
  }
  // the last round's update: G into gbuf(round), U in place
  hipLaunchKernelGGL(k_jround, dim3(gtiles + utiles), dim3(kSolveThreads), pad, s, gbuf(round - 1), gbuf(round), Up, mp,
                     nb, -1, prev_step, d_trace, tol, skip, rel, floor_rel, nullptr, nullptr, nullptr, nullptr,
                     vbuf(round - 1), fbuf(round - 1));
  GC_LAUNCH_CHECK();
  const z64* Gf = gbuf(round);
  hipLaunchKernelGGL(k_unpad, dim3(blocks_for((size_t)m * m, 256)), dim3(256), 0, s, Gf, Up, m, mp, U, ldu, lam);
  GC_LAUNCH_CHECK();
  GC_CHECK(conv, GCAMPS_ENUMERIC,
           std::string("block Jacobi eigensolver did not converge (m = ") + std::to_string(m) +
               (rel ? ", relative-accuracy pass)" : ", first pass)"));
  if (host_sweeps) *host_sweeps = sweeps;
}

void launch_rownorm2(hipStream_t s, const z64* B, int m, int k, int ldb, double* out) {
  if (m <= 0) return;
  hipLaunchKernelGGL(k_rownorm2, dim3(m), dim3(256), 0, s, B, m, k, ldb, out);
  GC_LAUNCH_CHECK();
}

void launch_trunc(hipStream_t s, const double* sig2, int m, double cutoff, int chi_max, int mode, int force_k,
                  int* perm, double* sig_sorted, DevStatus* st, const double* extra) {
  GC_CHECK(m <= TRUNC_MAX, GCAMPS_ECAPACITY, "truncation: matrix side exceeds 4096");
  hipLaunchKernelGGL(k_trunc, dim3(1), dim3(1024), 0, s, sig2, m, cutoff, chi_max, mode, force_k, perm, sig_sorted,
                     st, extra);
  GC_LAUNCH_CHECK();
}

void launch_emit(hipStream_t s, int wide, int left_ortho, int renorm, int p, int q, int kept, const z64* U, int ldu,
                 const z64* B, int ldb, const int* perm, const double* sig, z64* L, z64* R) {
  size_t total = (size_t)p * kept + (size_t)kept * q;
  hipLaunchKernelGGL(k_emit, dim3(blocks_for(total, 256)), dim3(256), 0, s, wide, left_ortho, renorm, p, q, kept, U,
                     ldu, B, ldb, perm, sig, L, R);
  GC_LAUNCH_CHECK();
}

void launch_copy(hipStream_t s, z64* dst, const z64* src, size_t count) {
  if (!count) return;
  hipLaunchKernelGGL(k_copy, dim3(blocks_for(count, 256)), dim3(256), 0, s, dst, src, count);
  GC_LAUNCH_CHECK();
}

void launch_fill_identity(hipStream_t s, z64* U, int m, int ld) {
  hipLaunchKernelGGL(k_fill_identity, dim3(blocks_for((size_t)m * m, 256)), dim3(256), 0, s, U, m, ld);
  GC_LAUNCH_CHECK();
}

}  // namespace gc
