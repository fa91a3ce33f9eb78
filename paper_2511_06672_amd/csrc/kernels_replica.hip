// Replica-tensor scoring of disentangler candidates: the Rényi-2 purity of Q_c Theta (§3, the
// entanglement of the rotated two-site tensor), rewritten so that the state and the candidate
// separate.  Exact up to rounding; the candidate enters only through a table built once per
// candidate set.
//
// Theta(a, t, b), t = (t1 t2) in [0, D), D = d^2.  Take the cut on the side of the smaller bond
// x (x = a when chi_l <= chi_r, else x = b) and let y be the other bond.  With
//   F(x t, x' t') = sum_y Theta(x t y) conj Theta(x' t' y)          (Hermitian, (X D) x (X D))
// the purity of the cut is
//   P_c = sum_{t t' u u'} W(t t', u u') V_c(t t', u u'),
//   W(t t', u u') = sum_{x x'} F(x t, x' t') F(x' u, x u').
// For the left cut (x = a) V_c = VL_c with
//   VL(t t', u u') = sum_{s1 s1'} aL(s1, s1'; t, t') aL(s1', s1; u, u'),
//   aL(s1, s1'; t, t') = sum_{s2} Q((s1 s2), t) conj Q((s1' s2), t');
// for the right cut (x = b) V_c = VR_c with the roles of the two qudits exchanged:
//   VR(t t', u u') = sum_{s2 s2'} aR(s2, s2'; t, t') aR(s2', s2; u, u'),
//   aR(s2, s2'; t, t') = sum_{s1} Q((s1 s2), t) conj Q((s1 s2'), t').
// S2_c = -ln(P_c / tr^2), tr = sum_{x t} F(x t, x t).
//
// Symmetry halves the pair sum: with B_{xx'}(t, t') = F(x t, x' t') one has
// F(x' u, x u') = conj B_{xx'}(u', u) and B_{x'x}(t, t') = conj B_{xx'}(t', t), so
//   W = A + A^T,  A = sum_{x < x'} b g^T + 1/2 sum_x b g^T,  b = vec B_{xx'}, g(u u') = conj B_{xx'}(u', u),
// and P_c = Re sum A o (V_c + V_c^T).  The tables hold Vs_c = V_c + V_c^T.
//
// Cost per bond: the Gram F ((X D)^2 Y / 2 complex MACs on the FP64 MFMA GEMM), the pair sum
// (X (X + 1) / 2 * D^4 complex MACs) and one D^4 dot product per candidate, against
// N_c * 4 m^2 k flop for scoring every candidate directly.
#include "kernels.h"

namespace gc {

namespace {

template <int DD>
__device__ __forceinline__ z64 v_entry(const z64* __restrict__ q, bool left, int t, int tp, int u, int up) {
  constexpr int D = DD * DD;
  z64 acc = {0.0, 0.0};
  for (int p = 0; p < DD; ++p)
    for (int pp = 0; pp < DD; ++pp) {
      z64 a1 = {0.0, 0.0}, a2 = {0.0, 0.0};
      for (int k = 0; k < DD; ++k) {
        const int sp = left ? p * DD + k : k * DD + p;
        const int spp = left ? pp * DD + k : k * DD + pp;
        a1 = cadd(a1, cmul(q[sp * D + t], cconj(q[spp * D + tp])));
        a2 = cadd(a2, cmul(q[spp * D + u], cconj(q[sp * D + up])));
      }
      acc = cadd(acc, cmul(a1, a2));
    }
  return acc;
}

// One thread per (candidate, entry e = r R + col): vl/vr[c R^2 + e] = V(r, col) + V(col, r).
template <int DD>
__global__ __launch_bounds__(256) void k_replica_tables(int count, const z64* __restrict__ qm, z64* __restrict__ vl,
                                                        z64* __restrict__ vr) {
  constexpr int D = DD * DD, R = D * D;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (e >= R * R || c >= count) return;
  const int r = e / R, col = e % R;
  const int t = r / D, tp = r % D, u = col / D, up = col % D;
  const z64* q = qm + (size_t)c * D * D;
  vl[(size_t)c * R * R + e] = cadd(v_entry<DD>(q, true, t, tp, u, up), v_entry<DD>(q, true, u, up, t, tp));
  vr[(size_t)c * R * R + e] = cadd(v_entry<DD>(q, false, t, tp, u, up), v_entry<DD>(q, false, u, up, t, tp));
}

// Right cut: Tr[(b D + t) chi_l + a] = Theta[(a D + t) chi_r + b], 32 x 32 tiles of (a, b) per t.
__global__ __launch_bounds__(256) void k_replica_transpose(int chil, int D, int chir, const z64* __restrict__ theta,
                                                           z64* __restrict__ tr) {
  __shared__ double sr[32][33], si[32][33];
  const int t = blockIdx.z;
  const int a0 = blockIdx.y * 32, b0 = blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int j = ty; j < 32; j += 8) {
    const int a = a0 + j, b = b0 + tx;
    if (a < chil && b < chir) {
      const z64 v = theta[((size_t)a * D + t) * chir + b];
      sr[j][tx] = v.re;
      si[j][tx] = v.im;
    }
  }
  __syncthreads();
  for (int j = ty; j < 32; j += 8) {
    const int b = b0 + j, a = a0 + tx;
    if (a < chil && b < chir) tr[((size_t)b * D + t) * chil + a] = z64{sr[tx][j], si[tx][j]};
  }
}

// Pair (x, x') with x <= x' from its rank p in row-major order of the upper triangle.
__device__ __forceinline__ void unrank_pair(long long p, int X, int& x, int& xp) {
  // offset(x) = x X - x (x - 1) / 2 pairs precede row x
  const double b = 2.0 * X + 1.0;
  int g = (int)floor((b - sqrt(b * b - 8.0 * (double)p)) * 0.5);
  g = max(0, min(g, X - 1));
  auto off = [X](long long r) { return r * X - r * (r - 1) / 2; };
  while (g > 0 && off(g) > p) --g;
  while (g + 1 < X && off(g + 1) <= p) ++g;
  x = g;
  xp = g + (int)(p - off(g));
}

// Partial sums of A over a contiguous range of pairs.  DD = 3: 243 threads own 3 x 9 entries of
// the 81 x 81 A; DD = 2: 256 threads own one entry of the 16 x 16 A.  Pairs are staged NB at a
// time in LDS as b = vec B_{xx'}; g is read from b by index transposition.  Row layout of the
// partial: 2 R^2 doubles (A as re, im) and the trace contribution, padded to 2 R^2 + 2.
template <int DD>
__global__ __launch_bounds__(256) void k_replica_pairs(int X, const z64* __restrict__ F, int ldf, long long npairs,
                                                       double* __restrict__ partial) {
  constexpr int D = DD * DD, R = D * D;
  constexpr int RP = DD == 3 ? 3 : 1, CP = DD == 3 ? 9 : 1;
  constexpr int NTC = R / CP, NACT = (R / RP) * NTC;
  constexpr int NB = 8;
  __shared__ double br[NB][R], bi[NB][R];
  __shared__ double wgt[NB];
  __shared__ int px[NB], pxp[NB];
  const int t = threadIdx.x;
  const bool active = t < NACT;
  const int tr = active ? t / NTC : 0, tc = active ? t % NTC : 0;
  double ar[RP][CP], ai[RP][CP];
  for (int i = 0; i < RP; ++i)
    for (int k = 0; k < CP; ++k) ar[i][k] = ai[i][k] = 0.0;
  int colT[CP];
  for (int k = 0; k < CP; ++k) {
    const int col = tc * CP + k;
    colT[k] = (col % D) * D + col / D;
  }
  double trace = 0.0;
  const long long p0 = npairs * blockIdx.x / gridDim.x, p1 = npairs * (blockIdx.x + 1) / gridDim.x;
  for (long long pb = p0; pb < p1; pb += NB) {
    const int nb = (int)min((long long)NB, p1 - pb);
    if (t < nb) {
      int x, xp;
      unrank_pair(pb + t, X, x, xp);
      px[t] = x;
      pxp[t] = xp;
      wgt[t] = (x == xp) ? 0.5 : 1.0;
    }
    __syncthreads();
    for (int e = t; e < nb * R; e += blockDim.x) {  // e = (t1, j, t2): runs of one row of F
      const int t1 = e / (nb * D), rem = e % (nb * D), j = rem / D, t2 = rem % D;
      const z64 v = F[(size_t)(px[j] * D + t1) * ldf + pxp[j] * D + t2];
      br[j][t1 * D + t2] = v.re;
      bi[j][t1 * D + t2] = v.im;
    }
    __syncthreads();
    if (active) {
      for (int j = 0; j < nb; ++j) {
        const double w = wgt[j];
        double xr[RP], xi[RP], gr[CP], gi[CP];
        for (int i = 0; i < RP; ++i) {
          xr[i] = w * br[j][tr * RP + i];
          xi[i] = w * bi[j][tr * RP + i];
        }
        for (int k = 0; k < CP; ++k) {
          gr[k] = br[j][colT[k]];
          gi[k] = -bi[j][colT[k]];
        }
        for (int i = 0; i < RP; ++i)
          for (int k = 0; k < CP; ++k) {
            ar[i][k] += xr[i] * gr[k] - xi[i] * gi[k];
            ai[i][k] += xr[i] * gi[k] + xi[i] * gr[k];
          }
      }
    }
    if (t == 0)
      for (int j = 0; j < nb; ++j)
        if (px[j] == pxp[j])
          for (int s = 0; s < D; ++s) trace += br[j][s * D + s];
    __syncthreads();
  }
  double* out = partial + (size_t)blockIdx.x * (2 * R * R + 2);
  if (active)
    for (int i = 0; i < RP; ++i)
      for (int k = 0; k < CP; ++k) {
        const int e = (tr * RP + i) * R + tc * CP + k;
        out[2 * e] = ar[i][k];
        out[2 * e + 1] = ai[i][k];
      }
  if (t == 0) {
    out[2 * R * R] = trace;
    out[2 * R * R + 1] = 0.0;
  }
}

__global__ __launch_bounds__(256) void k_replica_reduce(int nwg, int len, const double* __restrict__ partial,
                                                        double* __restrict__ out) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= len) return;
  double s = 0.0;
  for (int w = 0; w < nwg; ++w) s += partial[(size_t)w * len + e];
  out[e] = s;
}

// One workgroup per candidate: P_c = Re sum_e A[e] Vs_c[e]; s2 = -ln(P_c / tr^2).
__global__ __launch_bounds__(256) void k_replica_score(int R2, int count, const double* __restrict__ A,
                                                       const z64* __restrict__ vs, double* __restrict__ s2) {
  __shared__ double red[256];
  const int c = blockIdx.x, t = threadIdx.x;
  if (c >= count) return;
  const z64* v = vs + (size_t)c * R2;
  double p = 0.0;
  for (int e = t; e < R2; e += 256) p += A[2 * e] * v[e].re - A[2 * e + 1] * v[e].im;
  red[t] = p;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (t < off) red[t] += red[t + off];
    __syncthreads();
  }
  if (t == 0) {
    const double tr = A[2 * R2];
    s2[c] = -log(red[0] / (tr * tr));
  }
}

}  // namespace

size_t replica_table_elems(int d, int count) {
  const size_t D = (size_t)d * d;
  return 2 * (size_t)count * D * D * D * D;
}

size_t replica_scratch_bytes(int d, int chi_max) {
  const size_t D = (size_t)d * d, R2 = D * D * D * D;
  const size_t XD = (size_t)chi_max * D;
  const size_t f = XD * XD * sizeof(z64);
  const size_t th = (size_t)chi_max * D * chi_max * sizeof(z64);
  const size_t part = (size_t)kReplicaMaxWg * (2 * R2 + 2) * sizeof(double);
  const size_t a = (2 * R2 + 2) * sizeof(double);
  return align256(f) + align256(th) + align256(part) + align256(a);
}

void launch_replica_tables(hipStream_t s, int d, int count, const z64* qmats, z64* tables) {
  GC_CHECK(d == 2 || d == 3, GCAMPS_EUNSUPPORTED, "replica scoring is implemented for d = 2 and 3");
  const int D = d * d, R2 = D * D * D * D;
  z64* vl = tables;
  z64* vr = tables + (size_t)count * R2;
  const dim3 g((R2 + 255) / 256, count);
  if (d == 3)
    hipLaunchKernelGGL(k_replica_tables<3>, g, dim3(256), 0, s, count, qmats, vl, vr);
  else
    hipLaunchKernelGGL(k_replica_tables<2>, g, dim3(256), 0, s, count, qmats, vl, vr);
  GC_LAUNCH_CHECK();
}

void launch_score_replica(hipStream_t s, int d, int chil, int chir, const z64* theta, const z64* tables, int count,
                          double* s2, void* scratch, size_t scratch_bytes) {
  GC_CHECK(d == 2 || d == 3, GCAMPS_EUNSUPPORTED, "replica scoring is implemented for d = 2 and 3");
  if (count <= 0) return;
  const int D = d * d, R2 = D * D * D * D;
  const bool left = chil <= chir;
  const int X = left ? chil : chir, Y = left ? chir : chil;
  const size_t XD = (size_t)X * D;
  char* p = reinterpret_cast<char*>(scratch);
  z64* F = reinterpret_cast<z64*>(p);
  p += align256(XD * XD * sizeof(z64));
  z64* Tr = reinterpret_cast<z64*>(p);
  p += align256((size_t)chil * D * chir * sizeof(z64));
  double* part = reinterpret_cast<double*>(p);
  p += align256((size_t)kReplicaMaxWg * (2 * R2 + 2) * sizeof(double));
  double* A = reinterpret_cast<double*>(p);
  p += align256((2 * (size_t)R2 + 2) * sizeof(double));
  GC_CHECK((size_t)(p - reinterpret_cast<char*>(scratch)) <= scratch_bytes, GCAMPS_ECAPACITY,
           "replica scoring scratch too small");
  const z64* M = theta;  // (X D) x Y row-major
  if (!left) {
    const dim3 g((chir + 31) / 32, (chil + 31) / 32, D);
    hipLaunchKernelGGL(k_replica_transpose, g, dim3(256), 0, s, chil, D, chir, theta, Tr);
    GC_LAUNCH_CHECK();
    M = Tr;
  }
  launch_zgemm(s, 0, 1, (int)XD, (int)XD, Y, M, Y, M, Y, F, (int)XD, z64{1.0, 0.0}, 0, 1);
  const long long npairs = (long long)X * (X + 1) / 2;
  const int nwg = (int)std::max<long long>(1, std::min<long long>(kReplicaMaxWg, (npairs + 127) / 128));
  if (d == 3)
    hipLaunchKernelGGL(k_replica_pairs<3>, dim3(nwg), dim3(256), 0, s, X, F, (int)XD, npairs, part);
  else
    hipLaunchKernelGGL(k_replica_pairs<2>, dim3(nwg), dim3(256), 0, s, X, F, (int)XD, npairs, part);
  GC_LAUNCH_CHECK();
  const int len = 2 * R2 + 2;
  hipLaunchKernelGGL(k_replica_reduce, dim3((len + 255) / 256), dim3(256), 0, s, nwg, len, part, A);
  GC_LAUNCH_CHECK();
  const z64* vs = tables + (left ? 0 : (size_t)count * R2);
  hipLaunchKernelGGL(k_replica_score, dim3(count), dim3(256), 0, s, R2, count, A, vs, s2);
  GC_LAUNCH_CHECK();
}

}  // namespace gc
