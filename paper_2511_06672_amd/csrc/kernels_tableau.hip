// Integer Z_d tableau kernels: Clifford layer update, disentangler right multiplication,
// and commutation of a Weyl operator through C (§2.2, §2.3, §2.3.1, §3).
//
// Device layout: row r of the 2n-row tableau has exponents tx[r*n + i], tz[r*n + i] for site
// i and phase tp[r] (power of tau, mod 2d).  Rows 0..n-1 are S_k = C Z_k C^dagger, rows
// n..2n-1 are D_k = C X_k C^dagger.  All arithmetic is exact integer arithmetic.
#include "kernels.h"

namespace gc {

namespace {

__device__ __forceinline__ int imod(int v, int m) {
  v %= m;
  return v < 0 ? v + m : v;
}

// Sum over the 64 lanes of a wavefront (every lane receives the total).
__device__ __forceinline__ int wave_sum(int v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__global__ void k_tableau_init(int n, int* tx, int* tz, int* tp) {
  int idx = blockIdx.x * blockDim.x + threadIdx.x;
  int total = 2 * n * n;
  if (idx < total) {
    int r = idx / n, i = idx % n;
    tx[idx] = (r >= n && r - n == i) ? 1 : 0;
    tz[idx] = (r < n && r == i) ? 1 : 0;
  }
  if (idx < 2 * n) tp[idx] = 0;
}

// One thread per tableau row; the words of a layer act on disjoint pairs and are applied
// in order.  lut entry: low 16 bits = image index, bits 16.. = tau-phase increment.
__global__ void k_tableau_layer(int n, int d, int count, const int* __restrict__ sites,
                                const uint32_t* __restrict__ luts, int* tx, int* tz, int* tp) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= 2 * n) return;
  const int D4 = d * d * d * d;
  int p = tp[r];
  for (int w = 0; w < count; ++w) {
    int a = sites[w], b = a + 1;
    int xa = tx[r * n + a], za = tz[r * n + a], xb = tx[r * n + b], zb = tz[r * n + b];
    int v = ((xa * d + za) * d + xb) * d + zb;
    uint32_t e = luts[(size_t)w * D4 + v];
    int img = (int)(e & 0xffffu);
    p = imod(p + (int)(e >> 16), 2 * d);
    tz[r * n + b] = img % d;
    tx[r * n + b] = (img / d) % d;
    tz[r * n + a] = (img / (d * d)) % d;
    tx[r * n + a] = img / (d * d * d);
  }
  tp[r] = p;
}

// Weyl string held by one wavefront: lane owns sites lane and lane + 64.
struct WaveWeyl {
  int x[2], z[2];
  int p;
};

__device__ __forceinline__ void ww_load(WaveWeyl& w, const int* tx, const int* tz, const int* tp, int row,
                                        int n, int lane) {
  for (int h = 0; h < 2; ++h) {
    int i = lane + 64 * h;
    w.x[h] = (i < n) ? tx[row * n + i] : 0;
    w.z[h] = (i < n) ? tz[row * n + i] : 0;
  }
  w.p = tp[row];
}

// w^e: exponents times e, phase e*p + 2 <x,z> e(e-1)/2
__device__ __forceinline__ WaveWeyl ww_pow(const WaveWeyl& w, int e, int d) {
  int xz = wave_sum(w.x[0] * w.z[0] + w.x[1] * w.z[1]);
  WaveWeyl o;
  for (int h = 0; h < 2; ++h) {
    o.x[h] = imod(e * w.x[h], d);
    o.z[h] = imod(e * w.z[h], d);
  }
  o.p = imod(e * w.p + 2 * imod(xz, d) * (e * (e - 1) / 2), 2 * d);
  return o;
}

// a * b: exponents add, phase p_a + p_b + 2 <z_a, x_b>
__device__ __forceinline__ void ww_mul(WaveWeyl& a, const WaveWeyl& b, int d) {
  int cross = wave_sum(a.z[0] * b.x[0] + a.z[1] * b.x[1]);
  for (int h = 0; h < 2; ++h) {
    a.x[h] = imod(a.x[h] + b.x[h], d);
    a.z[h] = imod(a.z[h] + b.z[h], d);
  }
  a.p = imod(a.p + b.p + 2 * imod(cross, d), 2 * d);
}

// C <- C Q^dagger at pair (site, site+1).  For each Pauli P of the pair the new row is
// C (Q^dagger P Q) C^dagger, i.e. the old rows multiplied out with the exponents of
// Q^dagger P Q = tau^q X_a^xa Z_a^za X_b^xb Z_b^zb in the order D_a, S_a, D_b, S_b.
__global__ void k_tableau_right_mult(int n, int d, int site, const DevStatus* st,
                                     const uint32_t* __restrict__ inv_luts, int* tx, int* tz, int* tp) {
  const int c = st->cstar;
  if (c == 0) return;
  const int lane = threadIdx.x;
  const int D4 = d * d * d * d;
  const uint32_t* lut = inv_luts + (size_t)c * D4;
  const int a = site, b = site + 1;
  WaveWeyl Sa, Sb, Da, Db;
  ww_load(Sa, tx, tz, tp, a, n, lane);
  ww_load(Sb, tx, tz, tp, b, n, lane);
  ww_load(Da, tx, tz, tp, n + a, n, lane);
  ww_load(Db, tx, tz, tp, n + b, n, lane);
  // targets: Z_a, Z_b, X_a, X_b  (index v = ((xa*d + za)*d + xb)*d + zb)
  const int tgt[4] = {d * d, 1, d * d * d, d};
  const int rows[4] = {a, b, n + a, n + b};
  WaveWeyl out[4];
  for (int t = 0; t < 4; ++t) {
    uint32_t e = lut[tgt[t]];
    int img = (int)(e & 0xffffu);
    int ezb = img % d, exb = (img / d) % d, eza = (img / (d * d)) % d, exa = img / (d * d * d);
    WaveWeyl acc;
    acc.x[0] = acc.x[1] = acc.z[0] = acc.z[1] = 0;
    acc.p = (int)(e >> 16);
    ww_mul(acc, ww_pow(Da, exa, d), d);
    ww_mul(acc, ww_pow(Sa, eza, d), d);
    ww_mul(acc, ww_pow(Db, exb, d), d);
    ww_mul(acc, ww_pow(Sb, ezb, d), d);
    out[t] = acc;
  }
  for (int t = 0; t < 4; ++t) {
    for (int h = 0; h < 2; ++h) {
      int i = lane + 64 * h;
      if (i < n) {
        tx[rows[t] * n + i] = out[t].x[h];
        tz[rows[t] * n + i] = out[t].z[h];
      }
    }
    if (lane == 0) tp[rows[t]] = out[t].p;
  }
}

// P = C^dagger W C for the target W = tau^{p_t} X^{x_t} Z^{z_t} (target layout: x[n], z[n], p).
// Exponents from the symplectic relations: delta_j = -lam(W, S_j), s_j = lam(W, D_j) with
// lam(u, v) = <z_u, x_v> - <x_u, z_v>.  The phase follows from multiplying the rows out:
// prod_j S_j^{s_j} D_j^{delta_j} = tau^q W(t), and P = W(delta, s, p_t - q + 2 <s, delta>).
__global__ void k_weyl_extract(int n, int d, const int* __restrict__ tx, const int* __restrict__ tz,
                               const int* __restrict__ tp, const int* __restrict__ target, DevWeyl* out,
                               int* err) {
  __shared__ int s_exp[kMaxN], d_exp[kMaxN];
  const int t = threadIdx.x;
  const int* tgx = target;
  const int* tgz = target + n;
  const int pt = target[2 * n];
  for (int j = t; j < n; j += blockDim.x) {
    int ls = 0, ld = 0;
    for (int i = 0; i < n; ++i) {
      ls += tgz[i] * tx[j * n + i] - tgx[i] * tz[j * n + i];
      ld += tgz[i] * tx[(n + j) * n + i] - tgx[i] * tz[(n + j) * n + i];
    }
    d_exp[j] = imod(-ls, d);
    s_exp[j] = imod(ld, d);
  }
  __syncthreads();
  if (t >= 64) return;
  const int lane = t;
  WaveWeyl acc;
  acc.x[0] = acc.x[1] = acc.z[0] = acc.z[1] = 0;
  acc.p = 0;
  for (int j = 0; j < n; ++j) {
    if (s_exp[j]) {
      WaveWeyl r;
      ww_load(r, tx, tz, tp, j, n, lane);
      ww_mul(acc, ww_pow(r, s_exp[j], d), d);
    }
    if (d_exp[j]) {
      WaveWeyl r;
      ww_load(r, tx, tz, tp, n + j, n, lane);
      ww_mul(acc, ww_pow(r, d_exp[j], d), d);
    }
  }
  int bad = 0;
  for (int h = 0; h < 2; ++h) {
    int i = lane + 64 * h;
    if (i < n && (acc.x[h] != imod(tgx[i], d) || acc.z[h] != imod(tgz[i], d))) bad = 1;
  }
  bad = wave_sum(bad);
  int sd = 0;
  for (int h = 0; h < 2; ++h) {
    int i = lane + 64 * h;
    if (i < n) sd += s_exp[i] * d_exp[i];
  }
  sd = wave_sum(sd);
  for (int h = 0; h < 2; ++h) {
    int i = lane + 64 * h;
    if (i < n) {
      out->x[i] = d_exp[i];
      out->z[i] = s_exp[i];
    }
  }
  if (lane == 0) {
    out->p = imod(pt - acc.p + 2 * imod(sd, d), 2 * d);
    int l = -1, r = -1;
    for (int i = 0; i < n; ++i)
      if (d_exp[i] || s_exp[i]) {
        if (l < 0) l = i;
        r = i;
      }
    out->l = l;
    out->r = r;
    *err = bad ? 1 : 0;
  }
}

}  // namespace

void launch_tableau_init(hipStream_t s, int n, int* tx, int* tz, int* tp) {
  int total = 2 * n * n;
  hipLaunchKernelGGL(k_tableau_init, dim3((total + 255) / 256), dim3(256), 0, s, n, tx, tz, tp);
  GC_LAUNCH_CHECK();
}

void launch_tableau_layer(hipStream_t s, int n, int d, int count, const int* sites, const uint32_t* luts,
                          int* tx, int* tz, int* tp) {
  hipLaunchKernelGGL(k_tableau_layer, dim3((2 * n + 127) / 128), dim3(128), 0, s, n, d, count, sites, luts,
                     tx, tz, tp);
  GC_LAUNCH_CHECK();
}

void launch_tableau_right_mult(hipStream_t s, int n, int d, int site, const DevStatus* st,
                               const uint32_t* inv_luts, int* tx, int* tz, int* tp) {
  hipLaunchKernelGGL(k_tableau_right_mult, dim3(1), dim3(64), 0, s, n, d, site, st, inv_luts, tx, tz, tp);
  GC_LAUNCH_CHECK();
}

void launch_weyl_extract(hipStream_t s, int n, int d, const int* tx, const int* tz, const int* tp,
                         const int* target, DevWeyl* out, int* err) {
  hipLaunchKernelGGL(k_weyl_extract, dim3(1), dim3(128), 0, s, n, d, tx, tz, tp, target, out, err);
  GC_LAUNCH_CHECK();
}

}  // namespace gc
