// Bond-dimension criterion for disentanglers: the rank each candidate would leave on the bond.
//
// For candidate c, M_c = reshape(Q_c Theta) across the cut (the same matrix whose purity the
// Renyi-2 score uses, §3); its singular values go through the truncation rule of the split
// (cutoff on the discarded weight, rank floor 1e-13 sigma_0, chi_max, degeneracy guard), and the
// kept count is the candidate's bond dimension.  Deciding the rank floor needs singular values
// accurate relative to sigma_0 far below the FP64 resolution of a Gram matrix, so each candidate
// gets a one-sided (Hestenes) Jacobi SVD of M_c itself: rows are rotated pairwise until they are
// mutually orthogonal, and the singular values are the row norms.  One workgroup per candidate
// holds M_c (smaller side <= 32) in LDS.
#include <algorithm>
#include <cfloat>
#include <climits>

#include "kernels.h"

namespace gc {

namespace {

constexpr int kRankThreads = 256;

// Round-robin pairing of mp (even) rows: step s pairs positions k and mp-1-k; position 0 fixed.
__device__ __forceinline__ void rr_rows(int k, int s, int mp, int& p, int& q) {
  const int i0 = k, i1 = mp - 1 - k;
  const int e0 = (i0 == 0) ? 0 : ((i0 - 1 + s) % (mp - 1)) + 1;
  const int e1 = ((i1 - 1 + s) % (mp - 1)) + 1;
  p = e0 < e1 ? e0 : e1;
  q = e0 < e1 ? e1 : e0;
}

__global__ __launch_bounds__(kRankThreads) void k_cand_rank(int d, int chil, int chir, const z64* __restrict__ theta,
                                                            const z64* __restrict__ qm, int count, double cutoff,
                                                            int chi_max, int* __restrict__ rank_out) {
  extern __shared__ double lds[];
  __shared__ double s2v[32];
  __shared__ int rotated;
  const int c = blockIdx.x, t = threadIdx.x;
  if (c >= count) return;
  const int D2 = d * d;
  const bool rows_first = chil * d <= d * chir;
  const int m = rows_first ? chil * d : d * chir;
  const int k = rows_first ? d * chir : chil * d;
  const int mp = m + (m & 1);  // even row count (a padding row of zeros)
  double* mr = lds;
  double* mi = lds + (size_t)mp * k;
  const z64* q = qm + (size_t)c * D2 * D2;
  // M_c[(a s1'), (s2' b)] = sum_{s1 s2} Q[(s1' s2'), (s1 s2)] Theta[a, s1, s2, b]; rows are the
  // smaller side (the transpose otherwise: same singular values)
  for (int e = t; e < mp * k; e += kRankThreads) {
    const int r = e / k, col = e % k;
    double vr = 0.0, vi = 0.0;
    if (r < m) {
      int a, s1p, s2p, b;
      if (rows_first) {
        a = r / d;
        s1p = r % d;
        s2p = col / chir;
        b = col % chir;
      } else {
        s2p = r / chir;
        b = r % chir;
        a = col / d;
        s1p = col % d;
      }
      const z64* qrow = q + (s1p * d + s2p) * D2;
      for (int x = 0; x < D2; ++x) {
        const z64 qv = qrow[x];
        const z64 tv = theta[((size_t)a * D2 + x) * chir + b];
        vr += qv.re * tv.re - qv.im * tv.im;
        vi += qv.re * tv.im + qv.im * tv.re;
      }
    }
    mr[e] = vr;
    mi[e] = vi;
  }
  __syncthreads();
  // Hestenes sweeps: 16 threads per row pair (mp / 2 <= 16 pairs per step)
  const int grp = t >> 4, gl = t & 15;
  const int npairs = mp / 2;
  const double tol = 1e-15;
  for (int sweep = 0; sweep < 60; ++sweep) {
    if (t == 0) rotated = 0;
    __syncthreads();
    for (int step = 0; step < mp - 1; ++step) {
      if (grp < npairs) {
        int p, qq;
        rr_rows(grp, step, mp, p, qq);
        double al = 0.0, be = 0.0, gr = 0.0, gi = 0.0;
        for (int j = gl; j < k; j += 16) {
          const double pr = mr[p * k + j], pi = mi[p * k + j];
          const double qr = mr[qq * k + j], qi = mi[qq * k + j];
          al += pr * pr + pi * pi;
          be += qr * qr + qi * qi;
          gr += pr * qr + pi * qi;  // r_p conj(r_q)
          gi += pi * qr - pr * qi;
        }
        for (int off = 8; off > 0; off >>= 1) {
          al += __shfl_xor(al, off, 16);
          be += __shfl_xor(be, off, 16);
          gr += __shfl_xor(gr, off, 16);
          gi += __shfl_xor(gi, off, 16);
        }
        const double h2 = gr * gr + gi * gi;
        if (h2 > 1e-300 && h2 > tol * tol * al * be) {
          // J = [[c, -sp], [conj(sp), c]] diagonalises [[al, g], [conj g, be]]; rows <- J rows
          const double dlt = be - al;
          const double sg = dlt < 0.0 ? -1.0 : 1.0;
          const double den = fabs(dlt) + sqrt(dlt * dlt + 4.0 * h2);
          const double qn = 1.0 / sqrt(den * den + 4.0 * h2);
          const double cs = den * qn, spr = 2.0 * sg * qn * gr, spi = 2.0 * sg * qn * gi;
          for (int j = gl; j < k; j += 16) {
            const double pr = mr[p * k + j], pi = mi[p * k + j];
            const double qr = mr[qq * k + j], qi = mi[qq * k + j];
            mr[p * k + j] = cs * pr - (spr * qr - spi * qi);
            mi[p * k + j] = cs * pi - (spr * qi + spi * qr);
            mr[qq * k + j] = cs * qr + (spr * pr + spi * pi);
            mi[qq * k + j] = cs * qi + (spr * pi - spi * pr);
          }
          if (gl == 0) rotated = 1;
        }
      }
      __syncthreads();
    }
    const int any = rotated;
    __syncthreads();
    if (!any) break;
  }
  // singular values squared = row norms squared
  if (t < m) {
    double s = 0.0;
    for (int j = 0; j < k; ++j) s += mr[t * k + j] * mr[t * k + j] + mi[t * k + j] * mi[t * k + j];
    s2v[t] = s;
  }
  __syncthreads();
  if (t == 0) {
    double* key = s2v;
    for (int i = 1; i < m; ++i) {  // descending
      const double v = key[i];
      int j = i - 1;
      while (j >= 0 && key[j] < v) {
        key[j + 1] = key[j];
        --j;
      }
      key[j + 1] = v;
    }
    double total = 0.0;
    for (int i = m - 1; i >= 0; --i) total += key[i];
    int kk = m;  // the truncation rule of the split (cutoff, floor, chi_max, degeneracy guard)
    if (total > 0.0) {
      double tail = 0.0;
      int kcut = m;
      for (int j = m - 1; j >= 1; --j) {
        tail += key[j] / total;
        if (tail <= cutoff) kcut = j;
        else break;
      }
      const double s0 = sqrt(key[0]);
      int kfloor = 0;
      for (int i = 0; i < m; ++i)
        if (sqrt(key[i]) > 1e-13 * s0) ++kfloor;
      kk = min(kcut, min(kfloor, chi_max));
      if (kk < 1) kk = 1;
      if (kk < m) {
        const double sk = sqrt(key[kk]), skm = sqrt(key[kk - 1]);
        if (sk > 1e-13 * s0 && sk >= skm * (1.0 - 1e-10)) {
          int j = kk - 1;
          while (j > 0 && sqrt(key[j]) >= sqrt(key[j - 1]) * (1.0 - 1e-10)) --j;
          if (j > 0) kk = j;
        }
      }
    }
    rank_out[c] = kk;
  }
}

// c* = 0 unless some candidate leaves a smaller rank than the identity; then, among the
// candidates of the smallest rank, the lowest index with s2 <= min s2 + tol.
__global__ __launch_bounds__(1024) void k_select_rank(int count, const int* __restrict__ rank,
                                                      const double* __restrict__ s2, double tol, DevStatus* st) {
  __shared__ double red[1024];
  __shared__ int redi[1024];
  const int t = threadIdx.x;
  int rmin = INT_MAX;
  for (int i = t; i < count; i += 1024) rmin = min(rmin, rank[i]);
  redi[t] = rmin;
  __syncthreads();
  for (int off = 512; off > 0; off >>= 1) {
    if (t < off) redi[t] = min(redi[t], redi[t + off]);
    __syncthreads();
  }
  const int rbest = redi[0];
  __syncthreads();
  double mn = DBL_MAX;
  for (int i = t; i < count; i += 1024)
    if (rank[i] == rbest) mn = fmin(mn, s2[i]);
  red[t] = mn;
  __syncthreads();
  for (int off = 512; off > 0; off >>= 1) {
    if (t < off) red[t] = fmin(red[t], red[t + off]);
    __syncthreads();
  }
  const double smin = red[0];
  int best = INT_MAX;
  for (int i = t; i < count; i += 1024)
    if (rank[i] == rbest && s2[i] <= smin + tol && i < best) best = i;
  redi[t] = best;
  __syncthreads();
  for (int off = 512; off > 0; off >>= 1) {
    if (t < off) redi[t] = min(redi[t], redi[t + off]);
    __syncthreads();
  }
  if (t == 0) {
    st->cstar = (rbest < rank[0]) ? redi[0] : 0;
    st->s2min = smin;
  }
}

}  // namespace

void launch_cand_rank(hipStream_t s, int d, int chil, int chir, const z64* theta, const z64* qmats, int count,
                      double cutoff, int chi_max, int* rank_out) {
  const int m = std::min(chil * d, d * chir), k = std::max(chil * d, d * chir);
  const int mp = m + (m & 1);
  GC_CHECK(m <= kRankMaxM && (size_t)mp * k <= kRankMaxElems, GCAMPS_EUNSUPPORTED,
           "bond-dimension criterion: two-site matrix too large (smaller side <= 32, at most 8192 entries)");
  if (count <= 0) return;
  const size_t lds = 2 * (size_t)mp * k * sizeof(double);
  hipLaunchKernelGGL(k_cand_rank, dim3(count), dim3(kRankThreads), lds, s, d, chil, chir, theta, qmats, count, cutoff,
                     chi_max, rank_out);
  GC_LAUNCH_CHECK();
}

void launch_select_rank(hipStream_t s, int count, const int* rank, const double* s2, double tie_tol, DevStatus* st) {
  hipLaunchKernelGGL(k_select_rank, dim3(1), dim3(1024), 0, s, count, rank, s2, tie_tol, st);
  GC_LAUNCH_CHECK();
}

void rank_set_attributes() {
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_cand_rank), hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)(2 * kRankMaxElems * sizeof(double)));
  (void)hipGetLastError();
}

}  // namespace gc
