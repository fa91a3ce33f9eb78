// Rank-revealing reduction for the truncating splits of §2.4.
//
// A split of a two-site tensor after a disentangler (§3) factorises M = Q Theta, whose Gram
// G = W W^H (m x m, W the wide orientation of M) often has rank far below m: the rotated
// two-site tensor keeps the rank of the bond it came from.  Cholesky factorisation with
// diagonal pivoting, G = L L^H + S, takes one column per step with the largest remaining
// diagonal entry of the Schur complement S and stops once the trace of S is below a bound the
// truncation rule cannot see.  The r x r matrix L^H L then has the nonzero eigenvalues of
// L L^H, and with L^H L = Y diag(lam) Y^H the columns of L Y / sqrt(lam) are the corresponding
// eigenvectors of L L^H.  Every eigenvalue of G exceeds that of L L^H by at most tr S (S is
// positive semidefinite and both traces are exact), so the discarded weight counts tr S as
// discarded.  The eigensolver then works on an r x r matrix instead of m x m.
//
// k_pchol_panel runs NB pivot steps in one workgroup: the pivot is the largest remaining
// diagonal (lowest index on ties), the new column is the pivot row of the Schur complement
// (read from G, which holds the complement of all earlier panels) minus the contributions of
// this panel's earlier columns (held in registers), divided by the square root of the pivot.
// The host applies G <- G - L_p L_p^H for the panel's columns between panel launches.
#include <algorithm>
#include <climits>
#include <utility>

#include "kernels.h"

namespace gc {

namespace {

constexpr int kPcThreads = 512;

__global__ __launch_bounds__(256) void k_pchol_init(const z64* __restrict__ G, int m, int ldg,
                                                    double* __restrict__ dvec, int* __restrict__ pv,
                                                    PcState* __restrict__ stt) {
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < m; i += blockDim.x) {
    const double v = G[(size_t)i * ldg + i].re;
    dvec[i] = v;
    pv[i] = 0;
    s += fmax(v, 0.0);
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    stt->r = 0;
    stt->done = 0;
    stt->trace = red[0];
    stt->tres = red[0];
  }
}

// One panel of NB pivot steps; thread t owns rows t, t + 512, ..., t + (RPT - 1) 512.  One
// barrier per step: each wave posts its remaining trace, its pivot candidate and that row's
// entries in the panel's earlier columns; every thread then combines the eight posts in the same
// order.  The posting slots alternate between two sets by step parity, so a wave may post step
// jj + 1 while a slower one still reads step jj.
template <int RPT, int NB>
__global__ __launch_bounds__(kPcThreads) void k_pchol_panel(const z64* __restrict__ G, int m, int ldg,
                                                            double* __restrict__ dvec, int* __restrict__ pv,
                                                            z64* __restrict__ L, int ldl, PcState* __restrict__ stt,
                                                            double tol_rel) {
  constexpr int NW = kPcThreads / 64;
  __shared__ double w_sum[2][NW], w_max[2][NW];
  __shared__ int w_idx[2][NW];
  __shared__ z64 w_lp[2][NW][NB];
  if (stt->done) return;  // uniform: an earlier panel stopped
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int j0 = stt->r;
  const double stop = tol_rel * stt->trace;
  double dl[RPT];
  int pvl[RPT];
  z64 lp[RPT][NB];
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int i = t + q * kPcThreads;
    dl[q] = i < m ? dvec[i] : 0.0;
    pvl[q] = i < m ? pv[i] : 1;
#pragma unroll
    for (int c = 0; c < NB; ++c) lp[q][c] = z64{0.0, 0.0};
  }
  int jdone = 0;
  bool stopped = false;
  double tres = 0.0;
#pragma unroll
  for (int jj = 0; jj < NB; ++jj) {
    const int b = jj & 1;
    // remaining trace and the pivot (largest remaining diagonal, lowest index on ties)
    double ls = 0.0, lm = -1.0;
    int li = INT_MAX;
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      if (!pvl[q]) {
        const double v = fmax(dl[q], 0.0);
        ls += v;
        if (v > lm) {
          lm = v;
          li = t + q * kPcThreads;
        }
      }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      ls += __shfl_xor(ls, off, 64);
      const double om = __shfl_xor(lm, off, 64);
      const int oi = __shfl_xor(li, off, 64);
      if (om > lm || (om == lm && oi < li)) {
        lm = om;
        li = oi;
      }
    }
    // the wave's candidate row (owned by a thread of this wave) posts its panel entries
    if (li != INT_MAX && t == (li & (kPcThreads - 1))) {
#pragma unroll
      for (int q = 0; q < RPT; ++q)
        if (q == li / kPcThreads) {
#pragma unroll
          for (int c = 0; c < jj; ++c) w_lp[b][w][c] = lp[q][c];
        }
    }
    if (lane == 0) {
      w_sum[b][w] = ls;
      w_max[b][w] = lm;
      w_idx[b][w] = li;
    }
    __syncthreads();
    double tot = 0.0, dp = -1.0;
    int p = INT_MAX, pw = 0;
#pragma unroll
    for (int k = 0; k < NW; ++k) {
      tot += w_sum[b][k];
      const double mk = w_max[b][k];
      const int ik = w_idx[b][k];
      if (mk > dp || (mk == dp && ik < p)) {
        dp = mk;
        p = ik;
        pw = k;
      }
    }
    if (tot <= stop || !(dp > 0.0) || p >= m) {  // uniform across the workgroup
      tres = tot;
      stopped = true;
      break;
    }
    const z64* lpp = w_lp[b][pw];  // the pivot row's entries in this panel's earlier columns
    const double rp = sqrt(dp), irp = 1.0 / rp;
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int i = t + q * kPcThreads;
      z64 l = {0.0, 0.0};
      if (i < m && !pvl[q]) {
        if (i == p) {
          l = z64{rp, 0.0};
          pvl[q] = 1;
          dl[q] = 0.0;
        } else {
          const z64 g = G[(size_t)p * ldg + i];  // S[i, p] = conj(S[p, i])
          double sr = g.re, si = -g.im;
#pragma unroll
          for (int c = 0; c < jj; ++c) {  // - L[i, c] conj(L[p, c])
            const z64 a = lp[q][c], bb = lpp[c];
            sr -= a.re * bb.re + a.im * bb.im;
            si -= a.im * bb.re - a.re * bb.im;
          }
          l = z64{sr * irp, si * irp};
          dl[q] -= l.re * l.re + l.im * l.im;
        }
      }
      lp[q][jj] = l;
      if (i < m) L[(size_t)i * ldl + j0 + jj] = l;
    }
    jdone = jj + 1;
  }
  // columns this panel did not produce are zero, so the host's update of the panel is exact
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int i = t + q * kPcThreads;
    if (i < m) {
      for (int c = jdone; c < NB && j0 + c < ldl; ++c) L[(size_t)i * ldl + j0 + c] = z64{0.0, 0.0};
      dvec[i] = dl[q];
      pv[i] = pvl[q];
    }
  }
  if (t == 0) {
    stt->r = j0 + jdone;
    if (stopped) {
      stt->done = 1;
      stt->tres = tres;
    }
  }
}

// The factorisation ran through every row: nothing is left in the Schur complement.
__global__ void k_pchol_finish(PcState* __restrict__ stt) {
  stt->done = 1;
  stt->tres = 0.0;
}

// Columns of X (m x r, ld ldx) scaled to unit norm; one workgroup per column.
__global__ __launch_bounds__(256) void k_normalize_cols(z64* __restrict__ X, int m, int r, int ldx) {
  __shared__ double red[256];
  const int c = blockIdx.x;
  double s = 0.0;
  for (int i = threadIdx.x; i < m; i += blockDim.x) s += cabs2(X[(size_t)i * ldx + c]);
  red[threadIdx.x] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  const double f = red[0] > 0.0 ? 1.0 / sqrt(red[0]) : 0.0;
  for (int i = threadIdx.x; i < m; i += blockDim.x) X[(size_t)i * ldx + c] = cscale(X[(size_t)i * ldx + c], f);
}

// dst = f * src (m x r, ld ld).
__global__ void k_scaled_copy(z64* __restrict__ dst, const z64* __restrict__ src, size_t count, double f) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < count) dst[idx] = cscale(src[idx], f);
}

inline unsigned blocks_of(size_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

template <int RPT, int NB>
void run_panels(hipStream_t s, const z64* G, int m, int ldg, double* dvec, int* pv, z64* L, int ldl, PcState* stt,
                double tol_rel, int j0, int count) {
  for (int g = 0; g < count; ++g) {
    hipLaunchKernelGGL((k_pchol_panel<RPT, NB>), dim3(1), dim3(kPcThreads), 0, s, G, m, ldg, dvec, pv, L, ldl, stt,
                       tol_rel);
    GC_LAUNCH_CHECK();
    const int jc = j0 + g * NB;
    const int nbk = std::min(NB, m - jc);
    if (nbk > 0)  // Schur complement of the panel's columns: G <- G - L_p L_p^H
      launch_zgemm(s, 0, 1, m, m, nbk, L + jc, ldl, L + jc, ldl, const_cast<z64*>(G), ldg, z64{-1.0, 0.0}, 1, 1);
  }
}

}  // namespace

int pchol_reduce(hipStream_t s, z64* G, int m, int ldg, z64* L, int ldl, double tol_rel, int rmax, double* dvec,
                 int* pv, PcState* stt, PcState* host_state) {
  GC_CHECK(m >= 1 && m <= 4096 && ldl >= m, GCAMPS_ECAPACITY, "rank reduction: matrix side outside 1..4096");
  hipLaunchKernelGGL(k_pchol_init, dim3(1), dim3(256), 0, s, G, m, ldg, dvec, pv, stt);
  GC_LAUNCH_CHECK();
  // panel width times rows per thread at most 32 complex registers per thread (the panel
  // loop must unroll fully for the panel to stay in registers)
  const int rpt = (m + kPcThreads - 1) / kPcThreads;
  const int nb = rpt <= 2 ? 16 : rpt <= 4 ? 8 : 4;
  const int group = 4;  // panels launched between read-backs of the stop flag
  int j0 = 0;
  for (;;) {
    const int count = std::min(group, (m - j0 + nb - 1) / nb);
    if (rpt <= 1)
      run_panels<1, 16>(s, G, m, ldg, dvec, pv, L, ldl, stt, tol_rel, j0, count);
    else if (rpt <= 2)
      run_panels<2, 16>(s, G, m, ldg, dvec, pv, L, ldl, stt, tol_rel, j0, count);
    else if (rpt <= 4)
      run_panels<4, 8>(s, G, m, ldg, dvec, pv, L, ldl, stt, tol_rel, j0, count);
    else
      run_panels<8, 4>(s, G, m, ldg, dvec, pv, L, ldl, stt, tol_rel, j0, count);
    j0 += count * nb;
    GC_HIP(hipMemcpyAsync(host_state, stt, sizeof(PcState), hipMemcpyDeviceToHost, s));
    GC_HIP(hipStreamSynchronize(s));
    if (host_state->done || j0 >= m || host_state->r >= rmax) break;
  }
  if (!host_state->done && host_state->r >= m) {  // every row pivoted: the complement is empty
    hipLaunchKernelGGL(k_pchol_finish, dim3(1), dim3(1), 0, s, stt);
    GC_LAUNCH_CHECK();
    host_state->done = 1;
    host_state->tres = 0.0;
  }
  return host_state->r;
}

void launch_normalize_cols(hipStream_t s, z64* X, int m, int r, int ldx) {
  if (r <= 0) return;
  hipLaunchKernelGGL(k_normalize_cols, dim3(r), dim3(256), 0, s, X, m, r, ldx);
  GC_LAUNCH_CHECK();
}

void orthonormalize_cols(hipStream_t s, z64* X, z64* Xn, z64* S, int m, int r, int iters) {
  // Newton-Schulz steps toward the polar factor: X <- X (3 I - X^H X) / 2, X and Xn alternating
  // (ld r); the result ends in X.
  for (int it = 0; it < iters; ++it) {
    launch_zgemm(s, 1, 0, r, r, m, X, r, X, r, S, r, z64{1.0, 0.0}, 0, 1);
    const size_t cnt = (size_t)m * r;
    hipLaunchKernelGGL(k_scaled_copy, dim3(blocks_of(cnt, 256)), dim3(256), 0, s, Xn, X, cnt, 1.5);
    GC_LAUNCH_CHECK();
    launch_zgemm(s, 0, 0, m, r, r, X, r, S, r, Xn, r, z64{-0.5, 0.0}, 1, 0);
    std::swap(X, Xn);
  }
  if (iters & 1) launch_copy(s, Xn, X, (size_t)m * r);  // bring the last iterate back to the caller's X
}

}  // namespace gc
