// Internal declarations shared by the HIP translation units of libgcamps.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/gcamps.h"

namespace gc {

// ----------------------------------------------------------------- complex types
template <typename T>
struct cx {
  T re, im;
};
using z64 = cx<double>;
using c32 = cx<float>;

template <typename T>
__host__ __device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__host__ __device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b) {  // conj(a) * b
  return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
template <typename T>
__host__ __device__ __forceinline__ cx<T> cadd(cx<T> a, cx<T> b) {
  return {a.re + b.re, a.im + b.im};
}
template <typename T>
__host__ __device__ __forceinline__ cx<T> csub(cx<T> a, cx<T> b) {
  return {a.re - b.re, a.im - b.im};
}
template <typename T>
__host__ __device__ __forceinline__ cx<T> cscale(cx<T> a, T s) {
  return {a.re * s, a.im * s};
}
template <typename T>
__host__ __device__ __forceinline__ cx<T> cconj(cx<T> a) {
  return {a.re, -a.im};
}
template <typename T>
__host__ __device__ __forceinline__ T cabs2(cx<T> a) {
  return a.re * a.re + a.im * a.im;
}

// ----------------------------------------------------------------- MFMA 16x16x4 accumulators
// Row of accumulator item q in lane `lane` (column is lane % 16).  Measured on gfx950:
// v_mfma_f64_16x16x4f64 places row 4q + lane/16, v_mfma_f32_16x16x4f32 row 4(lane/16) + q.
__device__ __forceinline__ int mfma_row_f64(int lane, int q) { return 4 * q + (lane >> 4); }
__device__ __forceinline__ int mfma_row_f32(int lane, int q) { return 4 * (lane >> 4) + q; }
template <typename T>
__device__ __forceinline__ int mfma_row(int lane, int q);
template <>
__device__ __forceinline__ int mfma_row<double>(int lane, int q) { return mfma_row_f64(lane, q); }
template <>
__device__ __forceinline__ int mfma_row<float>(int lane, int q) { return mfma_row_f32(lane, q); }

// ----------------------------------------------------------------- errors
struct Error {
  int code;
  std::string msg;
};
void set_error(const std::string& msg);

#define GC_HIP(call)                                                              \
  do {                                                                            \
    hipError_t e_ = (call);                                                       \
    if (e_ != hipSuccess)                                                         \
      throw ::gc::Error{GCAMPS_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)}; \
  } while (0)

#define GC_CHECK(cond, code, msg)                 \
  do {                                            \
    if (!(cond)) throw ::gc::Error{(code), (msg)}; \
  } while (0)

#define GC_LAUNCH_CHECK() GC_HIP(hipGetLastError())

// ----------------------------------------------------------------- limits
inline size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

constexpr int kMaxD = 7;
constexpr int kMaxGateTerms = 81;  // Weyl terms of a general gate (two qutrits: 3^4)
constexpr int kMaxN = 128;
constexpr double kNearTieLowp = 1e-4;  // smallest re-score window with FP32 / split-BF16 scoring
constexpr size_t kDenseMax = size_t(1) << 16;  // largest d^n of the dense (validation) state
constexpr int kSmallEig = 32;   // largest m handled by the single-workgroup eigensolver
// Truncating splits with kReduceMinM < m <= kReduceMaxM take the pivoted-Cholesky path: below,
// its fixed costs (panel launches, two more eigensolves) outweigh what it saves (measured on the
// headline workload: m = 81 0.95 against 0.62 ms, m = 243 3.1 against 2.1 ms); above, it is
// untested against the plain path's accuracy.
constexpr int kReduceMinM = 320;
constexpr int kReduceMaxM = 1024;
constexpr int kBlk = 16;        // block size of the multi-workgroup block Jacobi

// ----------------------------------------------------------------- device status block
// Written by the selection / truncation kernels, read back once per bond.
struct DevStatus {
  int32_t cstar;       // selected candidate
  int32_t kept;        // kept rank after truncation
  int32_t flagged;     // degenerate cut flag
  int32_t nwindow;     // FP32 mode: number of candidates re-scored in FP64
  int32_t converged;   // eigensolver convergence flag (1 = ok)
  int32_t need_pass2;  // factorisation needs the accurate second pass
  int32_t sweeps;      // eigensolver sweeps used
  int32_t pad;
  double eps;          // discarded relative weight
  double smin_lp;      // minimum low-precision score
  double s2min;        // minimum FP64 score
  double norm2;        // |Theta|^2 of the scored tensor
  double lam_max;      // largest Gram eigenvalue
  double pad2;
};

// Weyl string result of the commutation step (device layout).
struct DevWeyl {
  int32_t x[kMaxN];
  int32_t z[kMaxN];
  int32_t p;
  int32_t l, r;
  int32_t pad;
};

// ----------------------------------------------------------------- compiled words
// A two-qudit Clifford word compiled to its action on Weyl strings of the pair:
// lut[v] for v = ((xa*d + za)*d + xb)*d + zb packs the image (x'a, z'a, x'b, z'b)
// in the same base-d index and the tau-phase increment in bits 16..23.
struct CompiledWord {
  std::vector<uint32_t> fwd;  // U W U^dagger
  std::vector<uint32_t> inv;  // U^dagger W U
  std::vector<z64> mat;       // d^2 x d^2 unitary, row-major (row = s_a*d + s_b)
};
CompiledWord compile_word(int d, const gcamps_word& w);
// Generator words (application order) of an exhaustive two-qudit Clifford set, identity first.
std::vector<std::vector<uint8_t>> clifford_word_set(int d, int kind);

}  // namespace gc

// ----------------------------------------------------------------- candidate set
struct gcamps_candset {
  int d;
  int count;
  std::vector<gc::CompiledWord> words;
  uint64_t uid;
};
