// Kernels of the reverse sweep (gradient of an observable with respect to phase-gate angles).
//
// Adjoint convention: for a real loss L and a complex array X, Xbar = dL/d conj(X), so that
// dL = 2 Re sum conj(Xbar) dX.  The dense products of the reverse sweep use the GEMM of
// kernels_linalg; the kernels here are the elementwise and reduction steps around them:
// * factorisation adjoint helpers (kept-norm, gauge scalings, the renormalisation
//   projection, row/column gathers by the sort order, the kept/discarded mixing matrix);
// * the transpose of the MPO site map and the gradient of its coefficients;
// * Q^dagger applied to a two-site tensor.
#include "kernels.h"

namespace gc {

namespace {

inline unsigned nblocks(size_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

// Deterministic single-block sum of 1024 per-thread partials (fixed tree order).
__device__ double block_sum(double v, double* red) {
  const int t = threadIdx.x;
  red[t] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (t < s) red[t] += red[t + s];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// out[0] = rn = 1/sqrt(sum_{j<k} sig_j^2) (1 when !renorm), out[1] = 1/(rn^2) factor base
__global__ __launch_bounds__(1024) void k_kept_norm(const double* __restrict__ sig, int k, int renorm,
                                                    double* __restrict__ out) {
  __shared__ double red[1024];
  double v = 0.0;
  for (int j = threadIdx.x; j < k; j += blockDim.x) v += sig[j] * sig[j];
  const double tot = block_sum(v, red);
  if (threadIdx.x == 0) out[0] = renorm ? 1.0 / sqrt(tot) : 1.0;
}

// X[r][c] *= 1 / (sig[c]^2 rn^2) (cols = true) or 1 / (sig[r]^2 rn^2) (cols = false).
__global__ void k_inv_gram_scale(z64* __restrict__ X, int rows, int cols, int by_cols, const double* __restrict__ sig,
                                 const double* __restrict__ rnp) {
  size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)rows * cols) return;
  const int r = (int)(idx / cols), c = (int)(idx % cols);
  const double s = by_cols ? sig[c] : sig[r];
  const double rn = rnp[0];
  X[idx] = cscale(X[idx], 1.0 / (s * s * rn * rn));
}

// out[0] = Re sum conj(a) b
__global__ __launch_bounds__(1024) void k_dot_re(const z64* __restrict__ a, const z64* __restrict__ b, size_t count,
                                                 double* __restrict__ out) {
  __shared__ double red[1024];
  double v = 0.0;
  for (size_t i = threadIdx.x; i < count; i += blockDim.x) v += a[i].re * b[i].re + a[i].im * b[i].im;
  const double tot = block_sum(v, red);
  if (threadIdx.x == 0) out[0] = tot;
}

// Xbar = rn (Nbar - N dot)
__global__ void k_renorm_bwd(const z64* __restrict__ Nbar, const z64* __restrict__ N, size_t count,
                             const double* __restrict__ rnp, const double* __restrict__ dotp, z64* __restrict__ Xbar) {
  size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= count) return;
  const double rn = rnp[0], dt = dotp[0];
  Xbar[idx] = cscale(csub(Nbar[idx], cscale(N[idx], dt)), rn);
}

// dst[a][c] = src[perm[a]][c] for a < keep_rows, 0 for keep_rows <= a < m.
__global__ void k_gather_rows(const z64* __restrict__ src, const int* __restrict__ perm, int m, int cols,
                              int keep_rows, z64* __restrict__ dst) {
  size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)m * cols) return;
  const int a = (int)(idx / cols), c = (int)(idx % cols);
  dst[idx] = (a < keep_rows) ? src[(size_t)perm[a] * cols + c] : z64{0.0, 0.0};
}

// dst[r][a] = src[r][perm[a]] (m x m)
__global__ void k_gather_cols(const z64* __restrict__ src, const int* __restrict__ perm, int m,
                              z64* __restrict__ dst) {
  size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)m * m) return;
  const int r = (int)(idx / m), a = (int)(idx % m);
  dst[idx] = src[(size_t)r * m + perm[a]];
}

// Mixing of kept (index < k) and discarded rows in the sorted basis:
//   Zc[a][b] = (G1[a][b] + conj(G1[b][a])) / (s_kept^2 - s_discarded^2)  when exactly one of a, b < k,
// 0 otherwise (and 0 on an exact tie, where the derivative of the split does not exist).
__global__ void k_trunc_mix(const z64* __restrict__ G1, int m, int k, const double* __restrict__ sig,
                            z64* __restrict__ Zc) {
  size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)m * m) return;
  const int a = (int)(idx / m), b = (int)(idx % m);
  z64 v = {0.0, 0.0};
  if ((a < k) != (b < k)) {
    const int kept = a < k ? a : b, disc = a < k ? b : a;
    const double delta = sig[kept] * sig[kept] - sig[disc] * sig[disc];
    if (delta > 0.0) v = cscale(cadd(G1[idx], cconj(G1[(size_t)b * m + a])), 1.0 / delta);
  }
  Zc[idx] = v;
}

// Transpose of the MPO site map k_mpo_site: in_bar[al, src, be] from out_bar.  Term b of the
// map sends in[al, src, be] to out[., (src + b dx) mod d, .] with weight K_b^{[kind 0,3]}
// omega^{(b dz) src}.
__global__ void k_mpo_site_bwd(int kind, int d, int chil, int chir, int dx, int dz, MpoCoeff co,
                               const z64* __restrict__ obar, z64* __restrict__ ibar) {
  size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t total = (size_t)chil * d * chir;
  if (idx >= total) return;
  const int be = (int)(idx % chir);
  const int src = (int)((idx / chir) % d);
  const int al = (int)(idx / ((size_t)chir * d));
  const int orr = (kind == 0 || kind == 1) ? d * chir : chir;
  z64 acc = {0.0, 0.0};
  for (int b = 0; b < d; ++b) {
    const int a = (b * dx) % d, c = (b * dz) % d;
    const int s = (src + a) % d;
    z64 wgt = co.w[(c * src) % d];
    if (kind == 0 || kind == 3) wgt = cmul(co.k[b], wgt);
    size_t o;
    if (kind == 3)
      o = ((size_t)al * d + s) * orr + be;
    else if (kind == 0)
      o = ((size_t)al * d + s) * orr + (size_t)b * chir + be;
    else if (kind == 2)
      o = ((size_t)(b * chil + al) * d + s) * orr + be;
    else
      o = ((size_t)(b * chil + al) * d + s) * orr + (size_t)b * chir + be;
    acc = cadd(acc, cmulc(wgt, obar[o]));
  }
  ibar[idx] = acc;
}

// Gradient of the MPO coefficients at the first site (kind 0) or of a one-site MPO (kind 3):
//   Kbar_b = sum_e out_bar[e] conj(term_b[e]),  term_b = omega^{(b dz) src} in[al, src, be].
__global__ __launch_bounds__(1024) void k_mpo_coeff_bwd(int kind, int d, int chil, int chir, int dx, int dz,
                                                        MpoCoeff co, const z64* __restrict__ in,
                                                        const z64* __restrict__ obar, z64* __restrict__ kbar) {
  __shared__ double red[1024];
  double accr[kMaxD], acci[kMaxD];
  for (int b = 0; b < kMaxD; ++b) accr[b] = acci[b] = 0.0;
  const size_t total = (size_t)chil * d * chir;
  const int orr = (kind == 0) ? d * chir : chir;
  for (size_t idx = threadIdx.x; idx < total; idx += blockDim.x) {
    const int be = (int)(idx % chir);
    const int src = (int)((idx / chir) % d);
    const int al = (int)(idx / ((size_t)chir * d));
    const z64 v = in[idx];
    for (int b = 0; b < d; ++b) {
      const int a = (b * dx) % d, c = (b * dz) % d;
      const int s = (src + a) % d;
      const z64 term = cmul(co.w[(c * src) % d], v);
      const size_t o = (kind == 0) ? ((size_t)al * d + s) * orr + (size_t)b * chir + be
                                   : ((size_t)al * d + s) * orr + be;
      const z64 pr = cmulc(term, obar[o]);  // conj(term) * obar
      accr[b] += pr.re;
      acci[b] += pr.im;
    }
  }
  for (int b = 0; b < d; ++b) {
    const double r = block_sum(accr[b], red);
    const double i = block_sum(acci[b], red);
    if (threadIdx.x == 0) kbar[b] = z64{r, i};
  }
}

// theta <- Q_c^dagger theta on the physical pair of a (chil, d, d, chir) tensor.
__global__ void k_apply_qh(int d, int chil, int chir, int c, const z64* __restrict__ qm, z64* __restrict__ theta) {
  size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)chil * chir) return;
  const int a = (int)(idx / chir), b = (int)(idx % chir);
  const int D2 = d * d;
  const z64* q = qm + (size_t)c * D2 * D2;
  z64 v[kMaxD * kMaxD];
  for (int x = 0; x < D2; ++x) v[x] = theta[((size_t)a * D2 + x) * chir + b];
  for (int y = 0; y < D2; ++y) {
    z64 acc = {0.0, 0.0};
    for (int x = 0; x < D2; ++x) acc = cadd(acc, cmulc(q[x * D2 + y], v[x]));
    theta[((size_t)a * D2 + y) * chir + b] = acc;
  }
}

}  // namespace

void launch_kept_norm(hipStream_t s, const double* sig, int k, int renorm, double* out) {
  hipLaunchKernelGGL(k_kept_norm, dim3(1), dim3(1024), 0, s, sig, k, renorm, out);
  GC_LAUNCH_CHECK();
}
void launch_inv_gram_scale(hipStream_t s, z64* X, int rows, int cols, int by_cols, const double* sig,
                           const double* rn) {
  if (!rows || !cols) return;
  hipLaunchKernelGGL(k_inv_gram_scale, dim3(nblocks((size_t)rows * cols, 256)), dim3(256), 0, s, X, rows, cols,
                     by_cols, sig, rn);
  GC_LAUNCH_CHECK();
}
void launch_dot_re(hipStream_t s, const z64* a, const z64* b, size_t count, double* out) {
  hipLaunchKernelGGL(k_dot_re, dim3(1), dim3(1024), 0, s, a, b, count, out);
  GC_LAUNCH_CHECK();
}
void launch_renorm_bwd(hipStream_t s, const z64* Nbar, const z64* N, size_t count, const double* rn,
                       const double* dot, z64* Xbar) {
  if (!count) return;
  hipLaunchKernelGGL(k_renorm_bwd, dim3(nblocks(count, 256)), dim3(256), 0, s, Nbar, N, count, rn, dot, Xbar);
  GC_LAUNCH_CHECK();
}
void launch_gather_rows(hipStream_t s, const z64* src, const int* perm, int m, int cols, int keep_rows, z64* dst) {
  if (!m || !cols) return;
  hipLaunchKernelGGL(k_gather_rows, dim3(nblocks((size_t)m * cols, 256)), dim3(256), 0, s, src, perm, m, cols,
                     keep_rows, dst);
  GC_LAUNCH_CHECK();
}
void launch_gather_cols(hipStream_t s, const z64* src, const int* perm, int m, z64* dst) {
  hipLaunchKernelGGL(k_gather_cols, dim3(nblocks((size_t)m * m, 256)), dim3(256), 0, s, src, perm, m, dst);
  GC_LAUNCH_CHECK();
}
void launch_trunc_mix(hipStream_t s, const z64* G1, int m, int k, const double* sig, z64* Zc) {
  hipLaunchKernelGGL(k_trunc_mix, dim3(nblocks((size_t)m * m, 256)), dim3(256), 0, s, G1, m, k, sig, Zc);
  GC_LAUNCH_CHECK();
}
void launch_mpo_site_bwd(hipStream_t s, int kind, int d, int chil, int chir, int dx, int dz, const MpoCoeff& co,
                         const z64* obar, z64* ibar) {
  size_t total = (size_t)chil * d * chir;
  hipLaunchKernelGGL(k_mpo_site_bwd, dim3(nblocks(total, 256)), dim3(256), 0, s, kind, d, chil, chir, dx, dz, co,
                     obar, ibar);
  GC_LAUNCH_CHECK();
}
void launch_mpo_coeff_bwd(hipStream_t s, int kind, int d, int chil, int chir, int dx, int dz, const MpoCoeff& co,
                          const z64* in, const z64* obar, z64* kbar) {
  hipLaunchKernelGGL(k_mpo_coeff_bwd, dim3(1), dim3(1024), 0, s, kind, d, chil, chir, dx, dz, co, in, obar, kbar);
  GC_LAUNCH_CHECK();
}
void launch_apply_qh(hipStream_t s, int d, int chil, int chir, int c, const z64* qmats, z64* theta) {
  size_t total = (size_t)chil * chir;
  hipLaunchKernelGGL(k_apply_qh, dim3(nblocks(total, 128)), dim3(128), 0, s, d, chil, chir, c, qmats, theta);
  GC_LAUNCH_CHECK();
}

}  // namespace gc
