// Launch wrappers of the HIP kernels (one definition per .hip translation unit).
#pragma once

#include "internal.h"

namespace gc {

// ------------------------------------------------------------------ tableau (kernels_tableau.hip)
// Device tableau: tx[2n*n], tz[2n*n], tp[2n] (row r, site i at r*n + i); exponents in [0,d),
// phases in [0,2d).
void launch_tableau_init(hipStream_t s, int n, int* tx, int* tz, int* tp);
void launch_tableau_layer(hipStream_t s, int n, int d, int count, const int* sites,
                          const uint32_t* luts, int* tx, int* tz, int* tp);
// C <- C Q^dagger for the candidate selected in st->cstar (no-op when 0).
void launch_tableau_right_mult(hipStream_t s, int n, int d, int site, const DevStatus* st,
                               const uint32_t* inv_luts, int* tx, int* tz, int* tp);
// P = C^dagger W C for the target W (x, z, p) held in `target`; result in out.
void launch_weyl_extract(hipStream_t s, int n, int d, const int* tx, const int* tz, const int* tp,
                         const int* target, DevWeyl* out, int* err);

// ------------------------------------------------------------------ dense linear algebra
// C = alpha * op(A) op(B) (+ C if accumulate); row-major, complex128; op 0 = N, 1 = conj-transpose.
// herm != 0: C is Hermitian (M == N, op(B) = op(A)^H): only the upper triangle is computed and
// mirrored.
void launch_zgemm(hipStream_t s, int opa, int opb, int M, int N, int K, const z64* A, int lda,
                  const z64* B, int ldb, z64* C, int ldc, z64 alpha, int accumulate, int herm);
// Hermitian eigen-decomposition by two-sided Jacobi.  G (m x m, ld ldg) is destroyed (holds
// the rotated matrix, padded to mp x mp with ld mp in the block variant); U (ld ldu) receives
// eigenvectors, lam the eigenvalues (unsorted).  rel: relative-accuracy criterion.
struct EigWork {
  z64* G;      // three padded m_pad x m_pad planes: matrix, accumulator, second matrix buffer
  z64* V;      // block rotations
  int* flags;  // device flags
  int m_pad;
  double* host_rb = nullptr;  // pinned host read-back slots (2 doubles); pageable locals when null
};
// Offsets in a context's pinned read-back block: device status, Cholesky state, eigensolver
// slots, conjugated Weyl string and its error flag.
constexpr size_t kRbStatus = 0, kRbPcState = 256, kRbEig = 512, kRbWeyl = 1024, kRbWeylErr = 2560, kRbBytes = 4096;
// precheck: test every pair against the rotation criterion first and return U = I, lam =
// diag(G) without a sweep when none qualifies (for matrices expected to be diagonal already,
// e.g. a Rayleigh-Ritz step; the result equals what one sweep that rotates nothing leaves).
void eig_hermitian(hipStream_t s, const z64* G, int m, int ldg, z64* U, int ldu, double* lam,
                   int rel, EigWork& w, DevStatus* st, int* host_sweeps, bool precheck = false);
void launch_rownorm2(hipStream_t s, const z64* B, int m, int k, int ldb, double* out);
// Sort, truncation rule, pass-2 decision.  mode 0 = truncate (cutoff, chi_max), 1 = floor only;
// force_k > 0 keeps exactly that rank (frozen-decision replay).
// extra (nullable, device): weight of directions outside sig2 that are discarded whatever the
// rule (a rank reduction's remainder), added to every tail sum and to the total.
void launch_trunc(hipStream_t s, const double* sig2, int m, double cutoff, int chi_max, int mode,
                  int force_k, int* perm, double* sig_sorted, DevStatus* st, const double* extra = nullptr);
// Write the two factors (see kernels_linalg.hip for the case table).
void launch_emit(hipStream_t s, int wide, int left_ortho, int renorm, int p, int q, int kept,
                 const z64* U, int ldu, const z64* B, int ldb, const int* perm, const double* sig,
                 z64* L, z64* R);
void launch_copy(hipStream_t s, z64* dst, const z64* src, size_t count);
void launch_fill_identity(hipStream_t s, z64* U, int m, int ld);

// ------------------------------------------------------------------ rank reduction (kernels_reduce.hip)
// Pivoted Cholesky of the Hermitian PSD G (m x m, ld ldg; destroyed: it ends as the Schur
// complement): G = L L^H + S with L (m x r, ld ldl) and tr S <= tol_rel * tr G, or r = rmax
// columns without meeting the bound (then *host_state.done == 0).  dvec (m doubles) and pv
// (m ints) are scratch; stt is a device PcState.  Returns r; host_state receives the final state
// (tres = tr S).
struct PcState {
  int32_t r, done, pad0, pad1;
  double trace, tres;
};
int pchol_reduce(hipStream_t s, z64* G, int m, int ldg, z64* L, int ldl, double tol_rel, int rmax, double* dvec,
                 int* pv, PcState* stt, PcState* host_state);
// Columns of X (m x r, ld ldx) scaled to unit 2-norm.
void launch_normalize_cols(hipStream_t s, z64* X, int m, int r, int ldx);
// X (m x r, ld r) replaced by its polar factor by `iters` Newton-Schulz steps (X nearly
// orthonormal); Xn (m x r) and S (r x r) are scratch.
void orthonormalize_cols(hipStream_t s, z64* X, z64* Xn, z64* S, int m, int r, int iters);

// ------------------------------------------------------------------ MPS kernels (kernels_mps.hip)
struct MpoCoeff {
  z64 k[kMaxD];       // c_b tau^{phase of P^b}
  z64 w[kMaxD];       // omega^j, j = 0..d-1
};
// Block-MPO site update.  kind: 0 = left end (opens the b index), 1 = interior, 2 = right end,
// 3 = local operator (l == r).  (dx, dz): exponents of P on this site.
void launch_mpo_site(hipStream_t s, int kind, int d, int chil, int chir, int dx, int dz,
                     const MpoCoeff& coeff, const z64* in, z64* out);
// Site update of the MPO sum_j coef_j (x)_i X^{x_ji} Z^{z_ji} of bond J (one term per bond
// index): kind as above; xz[2j], xz[2j+1] are the exponents of term j on this site; coef is
// used by kinds 0 and 3 only.
struct MpoTerms {
  int x[kMaxGateTerms], z[kMaxGateTerms];
  z64 coef[kMaxGateTerms];
};
void launch_mpo_sum_site(hipStream_t s, int kind, int d, int J, int chil, int chir, const MpoTerms& terms,
                         const z64* in, z64* out);
// out = Q_c Theta for the candidate c given by the host (a copy for c == 0).
void launch_rotate_copy(hipStream_t s, int d, int chil, int chir, int c, const z64* qmats, const z64* theta,
                        z64* out);
// Theta <- Q_{cstar} Theta in place (no-op when cstar == 0).  Theta (chil, d, d, chir).
void launch_apply_q(hipStream_t s, int d, int chil, int chir, const DevStatus* st, const z64* qmats,
                    z64* theta);
// Candidate scores S2_c for the candidates cand_list[0..count) (or 0..count when cand_list is
// null), in the arithmetic of `prec` (GCAMPS_SCORE_*; REPLICA takes the full set only and
// needs replica_tables).  nlimit (nullable): device count that
// overrides `count` (the list length is then only known on the device).  partial: scratch of
// count * tiles doubles for the tiled path; nbuf: scratch for the rotated matrices of a chunk
// of candidates (the tiled path processes as many candidates per launch as fit).  evs: optional
// event pairs recorded around each Gram-purity launch (count returned in *evused).
void launch_score(hipStream_t s, int prec, int d, int chil, int chir, const z64* theta,
                  const z64* q64, const c32* q32, const int* cand_list, int count,
                  const int* nlimit, double* s2, double* partial, size_t partial_cap, void* nbuf,
                  size_t nbuf_bytes, hipEvent_t* evs = nullptr, int evcap = 0, int* evused = nullptr,
                  const z64* replica_tables = nullptr);
void launch_select(hipStream_t s, int count, const double* s2, double tie_tol, DevStatus* st);

// ------------------------------------------------------------------ bond-dimension criterion (kernels_rank.hip)
constexpr int kRankMaxM = 32;        // smaller side of the two-site matrix
constexpr int kRankMaxElems = 8192;  // entries of the two-site matrix (LDS of one workgroup)
// rank_out[c] = bond dimension left by candidate c (truncation rule of the split applied to the
// singular values of reshape(Q_c Theta), one-sided Jacobi SVD per candidate).
void launch_cand_rank(hipStream_t s, int d, int chil, int chir, const z64* theta, const z64* qmats, int count,
                      double cutoff, int chi_max, int* rank_out);
// c* = 0 unless some candidate's rank is below the identity's; then the lowest index of the
// smallest rank with s2 <= min s2 (over that rank) + tie_tol.
void launch_select_rank(hipStream_t s, int count, const int* rank, const double* s2, double tie_tol,
                        DevStatus* st);
void rank_set_attributes();
void linalg_set_attributes();  // the block-Jacobi rounds' dynamic LDS limit

// ------------------------------------------------------------------ replica scoring (kernels_replica.hip)
// Full-set scores through the replica tensor of Theta (d = 2, 3): the Gram F of Theta over its
// larger bond, the pair sum A, and one D^4 dot product per candidate with its table.
constexpr int kReplicaMaxWg = 256;
constexpr int kScoreSmallM = 96;    // matrices up to this many rows are scored directly (fused kernel)  // workgroups (partial sums) of the pair sum
// complex128 elements of the tables of `count` candidates (left-cut and right-cut tables).
size_t replica_table_elems(int d, int count);
// Scratch bytes for bonds up to chi_max (F, the transposed Theta, partial sums, A).
size_t replica_scratch_bytes(int d, int chi_max);
// tables <- symmetrised V tables of the candidates qmats[0..count) (d^2 x d^2 unitaries).
void launch_replica_tables(hipStream_t s, int d, int count, const z64* qmats, z64* tables);
void launch_score_replica(hipStream_t s, int d, int chil, int chir, const z64* theta, const z64* tables,
                          int count, double* s2, void* scratch, size_t scratch_bytes);
// Low-precision window: list (ascending index) of candidates with s2lp <= min + window; the
// list length goes to st->nwindow.
void launch_window(hipStream_t s, int count, const double* s2lp, double window, int* list,
                   DevStatus* st);
// FP64 rule over the window: c* = lowest listed index with s2 <= min + tie_tol.
void launch_select_window(hipStream_t s, const int* list, const double* s2win, double tie_tol,
                          DevStatus* st);
// Weyl string applied to a dense vector of D = d^n amplitudes:
//   out(y) (+)= coeff * tau^p omega^{<z, y - x>} in(y - x)
void launch_apply_weyl_dense(hipStream_t s, int n, int d, long long D, const int* x, const int* z,
                             int p, const z64* in, z64* out, int accumulate, z64 coeff);
// psi(y) = sum_x m(x) tau^{p_x} omega^{<b_x, y - a_x>} s0(y - a_x) with per-x table
// (a_x packed as base-d index, b_x as n digits, p_x).
void launch_clifford_dense(hipStream_t s, int n, int d, long long D, const int* a_idx,
                           const int8_t* b_dig, const int* p_x, const z64* mvec, const z64* s0,
                           z64* out);
void launch_scale(hipStream_t s, z64* v, size_t count, z64 f);
void launch_norm2(hipStream_t s, const z64* v, size_t count, double* out);

// ------------------------------------------------------------------ reverse sweep (kernels_adjoint.hip)
// out[0] = 1/sqrt(sum_{j<k} sig_j^2) when renorm, else 1.
void launch_kept_norm(hipStream_t s, const double* sig, int k, int renorm, double* out);
// X (rows x cols) scaled by 1/(sig_c^2 rn^2) per column (by_cols) or per row.
void launch_inv_gram_scale(hipStream_t s, z64* X, int rows, int cols, int by_cols, const double* sig,
                           const double* rn);
// out[0] = Re sum conj(a) b.
void launch_dot_re(hipStream_t s, const z64* a, const z64* b, size_t count, double* out);
// Xbar = rn (Nbar - N dot).
void launch_renorm_bwd(hipStream_t s, const z64* Nbar, const z64* N, size_t count, const double* rn,
                       const double* dot, z64* Xbar);
// dst[a] = src[perm[a]] for rows a < keep_rows, zero rows below (m x cols).
void launch_gather_rows(hipStream_t s, const z64* src, const int* perm, int m, int cols, int keep_rows, z64* dst);
// dst[:, a] = src[:, perm[a]] (m x m).
void launch_gather_cols(hipStream_t s, const z64* src, const int* perm, int m, z64* dst);
// Kept/discarded mixing matrix of the truncated-split adjoint (sorted basis, k kept).
void launch_trunc_mix(hipStream_t s, const z64* G1, int m, int k, const double* sig, z64* Zc);
// Transpose of the MPO site map and the gradient of its coefficients (kinds 0 and 3).
void launch_mpo_site_bwd(hipStream_t s, int kind, int d, int chil, int chir, int dx, int dz, const MpoCoeff& co,
                         const z64* obar, z64* ibar);
void launch_mpo_coeff_bwd(hipStream_t s, int kind, int d, int chil, int chir, int dx, int dz, const MpoCoeff& co,
                          const z64* in, const z64* obar, z64* kbar);
// theta <- Q_c^dagger theta.
void launch_apply_qh(hipStream_t s, int d, int chil, int chir, int c, const z64* qmats, z64* theta);
}  // namespace gc
