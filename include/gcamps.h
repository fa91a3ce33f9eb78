/*
 * gcamps.h -- C ABI of the MI355X GCAMPS hot-path library (libgcamps.so).
 *
 * GCAMPS (Harper, Nakhl, Quella, Sevior, Usman; SCA/HPCAsia 2026) represents a
 * qudit state as psi = C|MPS>: C is a Clifford stored as a Z_d stabilizer
 * tableau (§2.2-§2.3) and |MPS> a matrix product state (§2.4, Eq. (MPS)).
 * Clifford gates only update the tableau (top loop of Fig. 1); a non-Clifford
 * gate is decomposed into Weyl operators, commuted through C (§2.3.1), applied
 * to the MPS and followed by disentangling (bottom loop of Fig. 1, §3).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Every function returns an int32 status: GCAMPS_OK (0) or a negative code.
 *   gcamps_last_error() gives a thread-local message for the last failure.
 * - d must be prime (the operator decomposition of §2.3.1 solves a linear
 *   system over the field Z_d); d <= 7 and n <= 128 are supported.
 * - Host arrays passed in are borrowed for the duration of the call only.
 * - Device memory: the caller allocates one device workspace of
 *   gcamps_workspace_bytes() bytes (e.g. a torch uint8 tensor) and passes it to
 *   gcamps_init; the library never frees it and the ctx must not outlive it.
 *   Pinned host staging and the per-ctx candidate tables are allocated by the
 *   library and released by gcamps_destroy / gcamps_candset_destroy.
 * - Streams: all device work of a ctx is enqueued on the HIP stream given to
 *   gcamps_init (e.g. torch.cuda.current_stream().cuda_stream).  Calls that
 *   return host values synchronise that stream.
 * - A ctx is not thread safe; distinct ctxs are independent.
 * - Site numbering starts at 0 (site 0 is the most significant digit of a
 *   computational-basis index).  Weyl phases are powers of tau = exp(i pi/d).
 * - Results are deterministic: identical inputs give bit-identical outputs.
 * - Environment: GCAMPS_AUTOTUNE=0 turns off the launch tuner, which times a
 *   few result-neutral launch parameters (candidates per thread of the scoring
 *   generator) once per shape and process; GCAMPS_TUNE_FILE=path keeps its
 *   picks in a JSON file across runs.  Neither changes any result.
 * - After GCAMPS_EDEVICE or GCAMPS_ENUMERIC the ctx is poisoned: only getters
 *   and gcamps_destroy may follow.  Other failed calls leave the state as it
 *   was.
 */
#ifndef GCAMPS_H
#define GCAMPS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  GCAMPS_OK = 0,
  GCAMPS_EINVAL = -1,       /* bad argument (site, size, null pointer, d, n) */
  GCAMPS_EUNSUPPORTED = -2, /* valid request outside what is implemented (non-prime d, ...) */
  GCAMPS_EWORKSPACE = -3,   /* workspace smaller than gcamps_workspace_bytes() */
  GCAMPS_ECAPACITY = -4,    /* a bond or candidate count would exceed configured capacity */
  GCAMPS_EDEVICE = -5,      /* HIP runtime error */
  GCAMPS_ENUMERIC = -6      /* NaN/Inf or non-convergence on the device */
};

/* Precision of disentangler candidate scoring.  The committed factorisations,
 * truncation and renormalisation are FP64 in every mode. */
enum {
  GCAMPS_SCORE_FP64 = 0, /* complex128 scoring */
  GCAMPS_SCORE_FP32 = 1, /* complex64 scoring, FP64 re-score of the near-tie window */
  GCAMPS_SCORE_BF16 = 2, /* split-BF16 scoring (each real as hi + lo BF16, FP32 accumulation, relative
                            error ~2^-16) for matrices above 96 rows, complex64 below; FP64 re-score
                            of the near-tie window */
  GCAMPS_SCORE_REPLICA = 3 /* FP64 replica-tensor scoring (d = 2, 3 only): the purity of Q_c Theta (§3)
                              rewritten as sum W(Theta) o V_c, W from the Gram of Theta over its
                              larger bond and V_c a table built once per candidate set, so a bond
                              costs one Gram product plus one d^8 dot product per candidate (exact
                              up to rounding; not a step of the paper).  Matrices of at most 96
                              rows are scored directly in FP64.  The FP64 re-score of the near-tie
                              window then decides, as in the FP32 mode. */
};

/* Disentangler choice at a bond (§3).
 * RENYI2: the candidate of smallest Renyi-2 entropy (lowest index within tie_tol).
 * BOND_DIM: the bond-dimension criterion (§4): a candidate is taken only if the bond dimension it
 *   leaves (the truncation rule of the split applied to the singular values of the rotated
 *   two-site tensor) is below the identity's; among the candidates of the smallest bond
 *   dimension the smallest Renyi-2 entropy wins (lowest index within tie_tol).  Needs
 *   GCAMPS_SCORE_FP64.  Two-site matrices with smaller side <= 32 and at most 8192 entries are
 *   ranked together by a one-sided Jacobi SVD per candidate; larger ones one candidate at a time
 *   by the split's own factorisation (Gram eigen-decomposition, relative-accuracy second pass
 *   where the rank floor decides), up to the factorisation's capacity. */
enum { GCAMPS_CRITERION_RENYI2 = 0, GCAMPS_CRITERION_BOND_DIM = 1 };

typedef struct gcamps_ctx gcamps_ctx;
typedef struct gcamps_candset gcamps_candset;

typedef struct {
  int32_t d;                /* qudit dimension, prime, 2..7 */
  int32_t n;                /* number of sites, 2..128 */
  int32_t chi_max;          /* maximal bond dimension kept by truncation */
  double cutoff;            /* discarded relative weight allowed per bond (R-TRUNC) */
  int32_t score_prec;       /* GCAMPS_SCORE_* */
  double near_tie;          /* low-precision re-score window in S2 units: >= 1e-4 with FP32 or
                               split-BF16 scoring (at least twice their measured S2 error, so the
                               FP64 choice is always inside the window), >= 1e-6 with replica
                               scoring; unused with FP64 scoring */
  double tie_tol;           /* FP64 tie tolerance of the argmin (default 1e-10) */
  int32_t max_sweeps;       /* disentangling sweeps per non-Clifford gate (default 2) */
  int32_t auto_disentangle; /* 1: gcamps_apply_phase_rotation disentangles afterwards */
  int32_t max_candidates;   /* capacity of the candidate table (>= candidate count) */
  int32_t max_gate_terms;   /* largest number of Weyl terms of a gcamps_apply_gate unitary (its MPO
                               bond, 1..81); 0 means d (diagonal phase gates only).  Bond
                               capacity is chi_max * max(d, max_gate_terms) <= 4096. */
  int32_t criterion;        /* GCAMPS_CRITERION_*: how a disentangler is chosen at a bond */
} gcamps_config;

/* A two-qudit Clifford word on the ordered pair (a, b) = (site, site + 1):
 * U = (X^w0 Z^w1 (x) X^w2 Z^w3) G_{len-1} ... G_1 G_0 with generator codes
 * 0 = F_a, 1 = F_b, 2 = P_a, 3 = P_b, 4 = SUM_{a->b}, 5 = SUM^{-1}_{a->b}
 * (F = H_d, P = S_d and SUM_d as defined in §2.3; gens[0] is applied first). */
typedef struct {
  int32_t len;
  const uint8_t* gens;
  int32_t weyl[4];
} gcamps_word;

/* Bytes of device workspace a ctx with this configuration needs.
 * Errors: EINVAL (null pointer, d/n/chi_max out of range), EUNSUPPORTED (d not prime). */
int32_t gcamps_workspace_bytes(const gcamps_config* cfg, size_t* bytes);

/* Create a state |0...0>: C = I (tableau S_k = Z_k, D_k = X_k), every MPS bond of
 * dimension 1, fidelity estimate 1 (§3).  dev_workspace: device pointer of at
 * least gcamps_workspace_bytes() bytes, 256-byte aligned; hip_stream: a
 * hipStream_t (NULL = default stream).
 * Errors: EINVAL, EUNSUPPORTED, EWORKSPACE, EDEVICE. */
int32_t gcamps_init(const gcamps_config* cfg, void* dev_workspace, size_t bytes,
                    void* hip_stream, gcamps_ctx** out);

/* Release host resources of a ctx (not the caller's workspace).  NULL is a no-op. */
int32_t gcamps_destroy(gcamps_ctx* ctx);

/* Clifford word on (site, site+1): C <- U C, a tableau update only (top loop,
 * Table 1 rules).  Errors: EINVAL (site out of [0, n-2], bad generator code). */
int32_t gcamps_apply_clifford(gcamps_ctx* ctx, int32_t site, const gcamps_word* word);

/* Several words acting on disjoint pairs, applied as one tableau launch.  The
 * pairs (sites[i], sites[i]+1) must be pairwise disjoint.  Errors: EINVAL. */
int32_t gcamps_apply_clifford_layer(gcamps_ctx* ctx, const int32_t* sites,
                                    const gcamps_word* words, int32_t count);

/* Diagonal phase gate diag(e^{i phi_0}, ..., e^{i phi_{d-1}}) on `site`
 * (bottom loop of Fig. 1, §3): U = sum_b c_b Z^b, C^dagger U C = sum_b c_b P^b
 * with P = C^dagger Z_site C from the tableau (§2.3.1); the sum is applied to the
 * MPS as a bond-d MPO on the support of P (§2.4) and compressed with FP64
 * factorisations and the truncation rule (cutoff, chi_max); the state is
 * renormalised and the fidelity estimate multiplied by (1 - discarded weight).
 * With auto_disentangle and a candidate set attached (gcamps_set_candset) the
 * disentangler runs afterwards.  phi: host array of d angles.
 * Errors: EINVAL, ECAPACITY, ENUMERIC, EDEVICE. */
int32_t gcamps_apply_phase_rotation(gcamps_ctx* ctx, int32_t site, const double* phi);

/* Compile candidate disentanglers (§3: two-qudit Cliffords Q whose application
 * to the MPS is compensated by C <- C Q^dagger) into a host object holding, per word, its
 * d^4-entry conjugation table and its d^2 x d^2 unitary.  words[0] must be the identity
 * (len 0, zero Weyl shift); count >= 1; `words` is borrowed for the call.  The set is
 * released by gcamps_candset_destroy (NULL is a no-op).
 * Errors: EINVAL (null pointer, count < 1, d not a prime in 2..7, first word not the
 * identity, generator code or Weyl exponent out of range). */
int32_t gcamps_candset_create(int32_t d, const gcamps_word* words, int32_t count,
                              gcamps_candset** out);
int32_t gcamps_candset_destroy(gcamps_candset* set);

/* Exhaustive two-qudit Clifford sets as generator words (§3, §3.1), without Weyl shifts, the
 * identity first.  Up to Weyl shifts a pair Clifford is its 4x4 symplectic matrix over Z_d.
 *   GCAMPS_WORDS_DISENTANGLERS: one word per class of Cliffords that differ only by
 *     single-qudit Cliffords applied after them, which leave the entanglement unchanged: the
 *     unique disentanglers of §3 (20 for d = 2, 90 for d = 3), each a shortest word of its class.
 *   GCAMPS_WORDS_ALL: one word per element of Sp(4, Z_d) (720 for d = 2, 51840 for d = 3).
 * Outputs (host memory): lens[i] = length of word i, gens = the words' generator codes
 * concatenated (application order, codes as in gcamps_word).  With lens == NULL only *count
 * and *total_gens are written.  The words feed gcamps_candset_create directly.
 * Errors: EINVAL (unknown kind, null count/total_gens, capacities below the set),
 * EUNSUPPORTED (d other than 2 and 3: §3.1 leaves larger d out, the group grows as d^10). */
enum { GCAMPS_WORDS_DISENTANGLERS = 0, GCAMPS_WORDS_ALL = 1 };
int32_t gcamps_clifford_words(int32_t d, int32_t kind, int32_t* lens, int32_t lens_cap, uint8_t* gens,
                              int64_t gens_cap, int32_t* count, int64_t* total_gens);

/* Apply a general non-Clifford gate U on `nsites` (1 or 2) adjacent qudits site..site+nsites-1
 * (the bottom loop of §3 for a unitary that is not diagonal or acts on two sites).  U is
 * d^k x d^k (k = nsites), row-major complex128 as interleaved (re, im), digit order with site
 * `site` most significant.  U is expanded on the Weyl basis, U = sum_{x,z} c_xz W_xz with
 * W_xz = (x)_t X^{x_t} Z^{z_t} and c_xz = Tr(W_xz^dagger U) / d^k (§2.3: the Weyl operators are
 * an orthogonal operator basis); terms with |c| <= 1e-14 max|c| are dropped.  Each kept term is
 * commuted through the Clifford (§2.3.1, as for Z_k in gcamps_apply_phase_rotation) and the sum
 * is applied to the MPS as an MPO whose bond is the number J of kept terms, then compressed
 * (§2.4) and, with auto_disentangle, disentangled (§3).  Diagonal single-site U gives the same
 * state as gcamps_apply_phase_rotation.
 * Errors: EINVAL (null pointer, site or nsites out of range, U not unitary to 1e-10),
 * ECAPACITY (J > max(d, max_gate_terms)), ENUMERIC, EDEVICE. */
int32_t gcamps_apply_gate(gcamps_ctx* ctx, int32_t site, int32_t nsites, const double* u);


/* Attach a candidate set used by auto-disentangling (uploads it to the device).
 * Errors: EINVAL (d mismatch), ECAPACITY (count > max_candidates), EDEVICE. */
int32_t gcamps_set_candset(gcamps_ctx* ctx, const gcamps_candset* set);

/* S2 of every candidate of the attached set at bond (bond, bond + 1) of the current state, the
 * disentangler's full-set score (§3; the Rényi-2 entropy of the rotated two-site tensor is how
 * this library reads the paper's entanglement measure) in the ctx's scoring mode (FP32/BF16: the low-precision first
 * pass).  Moves the orthogonality centre to `bond` (exact moves; the state is unchanged up to
 * rounding and numerically zero directions) and commits nothing.  out: host array of cap >=
 * candidate count doubles.  Errors: EINVAL (bond outside [0, n-2], no candidate set, cap too
 * small), EDEVICE. */
int32_t gcamps_score_bond(gcamps_ctx* ctx, int32_t bond, double* out, int64_t cap);
/* The factorisation every split of the bottom loop uses (§2.4: the SVD of a two-site tensor
 * reshaped across the cut, truncated by the ctx's rule: discarded weight <= cutoff, rank floor
 * 1e-13 sigma_0, at most chi_max kept, a cut inside a degenerate group moved below it), applied
 * to a caller's matrix so that it can be checked on its own.  m_host: p x q complex128,
 * row-major, interleaved (re, im), borrowed.  Requires min(p, q) and p * q within the ctx's
 * capacity (min(p, q) <= chi_max * max(d, max_gate_terms), p * q <= that times d times itself).
 * flags: 0, or GCAMPS_FACTORIZE_REDUCE for the path the truncating splits of the bottom loop
 * take: with a positive cutoff and 320 < min(p, q) <= 1024, a pivoted Cholesky factorisation of
 * the Gram first finds a basis of r columns holding all but at most
 * min(1e-14, cutoff / (2 min(p, q))) of the weight and the eigensolver runs on r x r (followed by
 * a Rayleigh-Ritz step on the full Gram); the remainder counts as discarded.
 * Outputs (host): sig_out[min(p, q)] the singular values in descending order (with
 * GCAMPS_FACTORIZE_REDUCE those of the reduced basis, zeros after them); *kept the rank
 * kept; *eps the discarded weight sum_{i >= kept} sigma_i^2 / sum_i sigma_i^2; if non-NULL,
 * l_out[p * kept] the left factor U_k (orthonormal columns, row-major complex128) and
 * r_out[kept * q] the right factor diag(s_k) V_k^dagger with s_k the kept singular values
 * scaled to unit norm (row-major complex128), so that L R = M_k / |M_k|.  The state of the ctx
 * is not changed.  Errors: EINVAL (null pointer, p or q < 1, unknown flag), ECAPACITY,
 * EUNSUPPORTED (ctx of a gradient recording), ENUMERIC, EDEVICE. */
enum { GCAMPS_FACTORIZE_REDUCE = 1 };
int32_t gcamps_factorize(gcamps_ctx* ctx, const double* m_host, int32_t p, int32_t q, int32_t flags,
                         double* sig_out, int32_t* kept, double* eps, double* l_out, double* r_out);

/* Disentangling sweeps (§3): sweep s runs over bonds 0..n-2 (s even) or n-2..0
 * (s odd).  At each bond the two-site tensor Theta is rotated by every
 * candidate Q_c and scored by the Renyi-2 entropy of its middle cut,
 * S2_c = -ln(sum |rho_c|^2 / (tr rho_c)^2), rho_c = M_c M_c^dagger; the chosen
 * c* is the lowest index with S2_c <= min S2 + tie_tol (in FP64; in FP32 mode
 * every candidate within near_tie of the FP32 minimum is re-scored in FP64
 * first).  If c* != 0: Theta <- Q Theta, C <- C Q^dagger.  Theta is then split
 * with the truncation rule.  Sweeping stops after a sweep with c* = 0
 * everywhere or after max_sweeps.  set may be NULL to use the attached set.
 * out_sweeps / out_changed_bonds may be NULL.
 * Errors: EINVAL, ECAPACITY, ENUMERIC, EDEVICE. */
int32_t gcamps_disentangle(gcamps_ctx* ctx, const gcamps_candset* set, int32_t* out_sweeps,
                           int32_t* out_changed_bonds);

/* <psi| tau^p X^x Z^z |psi> (= <MPS| C^dagger W C |MPS>, §3 observables) as
 * out[0] + i out[1].  x, z: host arrays of n exponents in [0, d).  Re<W> is the
 * expectation of the Hermitian (W + W^dagger)/2.  Errors: EINVAL, EDEVICE. */
int32_t gcamps_expectation(gcamps_ctx* ctx, const int8_t* x, const int8_t* z, int32_t p,
                           double out[2]);

/* Dense psi = C|MPS> into dev_out (d^n complex128, interleaved re/im, device
 * memory), defined up to one global phase (the tableau fixes C only up to a
 * phase).  For validation at small sizes: d^n <= 2^16.  dev_scratch: device
 * memory of at least 3 * 16 * d^n bytes, borrowed for the call; the per-index
 * Clifford table goes into the ctx's workspace (gcamps_workspace_bytes counts
 * it whenever d^n <= 2^16).  Nothing is allocated.  Synchronises the stream.
 * Errors: EINVAL (null pointer), EUNSUPPORTED (d^n > 2^16), EWORKSPACE
 * (scratch_bytes too small), ENUMERIC, EDEVICE. */
int32_t gcamps_statevector(gcamps_ctx* ctx, void* dev_out, void* dev_scratch,
                           size_t scratch_bytes);

/* gcamps_statevector without any allocation and without a caller scratch buffer, for callers
 * that cannot allocate (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  The three dense work vectors live in a static device array of the
 * library, 3 * 16 * 2^16 bytes (3 MiB), one copy per GPU held until the process ends; its
 * device address is looked up by gcamps_init on the ctx's device.  Same result as
 * gcamps_statevector, bit for bit.  Limit d^n <= 2^16.  Calls that overlap on one GPU share
 * that array and race: run them one at a time per GPU.  dev_out: d^n complex128 (device).
 * Nothing is allocated; the stream is synchronised.
 * Errors: EINVAL (null pointer), EUNSUPPORTED (d^n > 2^16), EDEVICE. */
int32_t gcamps_statevector_static(gcamps_ctx* ctx, void* dev_out);

/* One amplitude <digits|psi> of psi = C|MPS> (§3), same global-phase convention
 * as gcamps_statevector.  For validation at small sizes (d^n <= 2^16): the dense
 * state is formed in the ctx's own workspace (4 * 16 * d^n bytes plus the
 * per-index table, counted by gcamps_workspace_bytes), so nothing is allocated,
 * and the one requested entry is returned.  digits: n host values in [0, d),
 * site 0 most significant.  Synchronises the stream.
 * Errors: EINVAL (null pointer, digit out of range), EUNSUPPORTED (d^n > 2^16),
 * ENUMERIC, EDEVICE. */
int32_t gcamps_amplitude(gcamps_ctx* ctx, const int8_t* digits, double out[2]);

/* Tableau as an int32 [2n][2n+1] matrix: rows 0..n-1 = S_k = C Z_k C^dagger,
 * rows n..2n-1 = D_k = C X_k C^dagger; columns x_0..x_{n-1} | z_0..z_{n-1} | p
 * (phase in powers of tau, mod 2d). */
int32_t gcamps_get_tableau(gcamps_ctx* ctx, int32_t* out);
/* n-1 bond dimensions. */
int32_t gcamps_get_bond_dims(gcamps_ctx* ctx, int32_t* out);
/* Product of (1 - discarded weight) over every truncation so far. */
int32_t gcamps_get_fidelity(gcamps_ctx* ctx, double* f_est);
/* Disentangler choice log as int32 quadruples (gate, sweep, bond, c*).  Copies
 * min(cap, len) quadruples into out (may be NULL with cap 0) and the total
 * count into *len. */
int32_t gcamps_get_choice_log(gcamps_ctx* ctx, int32_t* out, int64_t cap, int64_t* len);
/* Site tensor `site` (chi_l, d, chi_r) as complex128 into host memory out
 * (capacity cap complex values); dims written to dims[3]. */
int32_t gcamps_get_site(gcamps_ctx* ctx, int32_t site, double* out, int64_t cap, int32_t dims[3]);
/* Statistics (16 doubles): [0] non-Clifford gates applied, [1] bonds scored,
 * [2] candidates re-scored in FP64 (FP32 mode), [3] degenerate cuts flagged,
 * [4] algorithmic flops of full-set scoring (direct: N_c (4 m^2 k + 8 d^4 chi_l chi_r) per bond;
 * replica mode: 4 (X d^2)^2 Y + 8 X (X + 1) / 2 d^8 + 2 N_c d^8 with X, Y the smaller and larger bond), [5] algorithmic flops of the Gram products of
 * the factorisations, [6] full-set scoring kernel time in ms (device events), [7] total time
 * inside gcamps_* calls in ms (host clock), [8] flops of the FP64 window re-score, [9] its
 * kernel time in ms, [10] scoring calls (bonds x passes), [11] launches of the Gram-purity MFMA
 * kernel (full-set scoring), [12] their summed kernel time in ms (device events around each
 * launch), [13] their algorithmic flops (4 m^2 k per candidate), [14] bond splits that factorised only the
 * centre tensor (identity kept), [15] algorithmic bytes read by the Gram-purity launches (each
 * rotated m x k matrix once). */
int32_t gcamps_get_stats(gcamps_ctx* ctx, double out[16]);
/* Counters for the roofline of the compression and MPO steps (§2.4, §3), accumulated since
 * gcamps_init: [0] factorisations; [1] their algorithmic flops, 4 (6 p q^2 + 20 q^3) per p x q
 * SVD with p >= q (the R-SVD operation count, complex); [2] their device time in ms (Gram
 * product to truncation rule, second pass included; the emit of the factors excluded);
 * [3] MPO site launches; [4] their algorithmic bytes (each site tensor read once, its product
 * written once, complex128); [5] their device time in ms; [6] splits of rotated two-site
 * tensors whose eigen-decomposition ran on a rank-reduced basis (pivoted Cholesky of the Gram),
 * [7] their summed basis size over their summed matrix side (0 when none).  out: host array of 8
 * doubles.  Synchronises the ctx's stream.  Errors: EINVAL, EDEVICE. */
int32_t gcamps_get_kernel_stats(gcamps_ctx* ctx, double out[8]);

/* ---------------------------------------------------------------------------
 * Batched independent circuits.
 *
 * Many circuits, each with its own configuration, are simulated concurrently
 * (the method of §2-§3 applied to each circuit; circuits never interact).
 * `lanes` host threads each own one HIP stream (default priority, created and
 * destroyed by the call) and one slice of the caller's workspace; they take
 * circuits from a shared queue ordered by estimated cost, largest first.  The
 * bonds of one circuit stay sequential; kernels of different circuits overlap on
 * the GPU.  Each circuit runs through gcamps_init and the single-state calls
 * above, so its results are bit-identical to running it alone with the same
 * configuration and candidate set.
 * ------------------------------------------------------------------------- */
enum { GCAMPS_OP_CLIFFORD_LAYER = 0, GCAMPS_OP_PHASE = 1 };

typedef struct {
  int32_t kind;             /* GCAMPS_OP_* */
  int32_t count;            /* CLIFFORD_LAYER: number of words (disjoint pairs); PHASE: unused */
  const int32_t* sites;     /* CLIFFORD_LAYER: `count` pair sites; PHASE: one site */
  const gcamps_word* words; /* CLIFFORD_LAYER: `count` words; PHASE: unused (NULL) */
  const double* phi;        /* PHASE: d angles of diag(e^{i phi_j}); CLIFFORD_LAYER: unused */
} gcamps_op;

typedef struct {
  gcamps_config cfg;     /* per circuit; cfg.d must equal the candidate set's d */
  const gcamps_op* ops;  /* applied in order, as gcamps_apply_clifford_layer /
                            gcamps_apply_phase_rotation would apply them */
  int64_t n_ops;
  /* Outputs: caller-owned host memory, each may be NULL. */
  int32_t* status;       /* GCAMPS_OK or the code of the call that failed */
  double* fidelity;      /* 1 value: the fidelity estimate after the circuit */
  int32_t* bond_dims;    /* n - 1 values */
  double* z_expect;      /* 2n values: <psi|Z_j|psi> for j = 0..n-1 as (re, im) */
  int32_t* choices;      /* choice-log quadruples (gate, sweep, bond, c*), at most choices_cap */
  int64_t choices_cap;
  int64_t* choices_len;  /* total number of quadruples */
} gcamps_batch_item;

/* Device workspace for gcamps_batch_run: min(lanes, count) slices, each the
 * largest gcamps_workspace_bytes() over the items (rounded up to 256 bytes).
 * Errors: EINVAL (null pointers, lanes outside [1, 64], malformed ops, bad config),
 * EUNSUPPORTED (non-prime d). */
int32_t gcamps_batch_workspace_bytes(const gcamps_batch_item* items, int32_t count, int32_t lanes,
                                     size_t* bytes);

/* Run `count` circuits on `lanes` concurrent lanes of the current HIP device.
 * set: candidate set attached to every circuit (may be NULL: no disentangling).
 * dev_workspace: 256-byte aligned device memory of gcamps_batch_workspace_bytes()
 * bytes, borrowed for the call.  Every item is attempted; each item's status is
 * written when non-NULL.  Returns GCAMPS_OK, or the code of the failed item with
 * the lowest index (gcamps_last_error names it).  stats (16 doubles, may be NULL):
 * [0] circuits completed, [1] non-Clifford gates applied, [2] wall time in ms,
 * [3] summed lane busy time in ms, [4] lanes used, [5] summed full-set scoring
 * kernel time in ms, [6] bonds scored, [7] Gram-purity kernel launches, [8] their
 * summed kernel time in ms, [9] their algorithmic flops (as gcamps_get_stats
 * [11]-[13], summed over circuits), [10]-[15] reserved (0).
 * Errors: EINVAL, EUNSUPPORTED, EWORKSPACE, ECAPACITY, ENUMERIC, EDEVICE. */
int32_t gcamps_batch_run(const gcamps_batch_item* items, int32_t count, const gcamps_candset* set,
                         int32_t lanes, void* dev_workspace, size_t bytes, double stats[16]);

/* ---------------------------------------------------------------------------
 * Gradient of an observable loss with respect to phase-gate angles.
 *
 * Loss: L(theta) = Re sum_j <psi|Z_j|psi> over all sites j (the observables of
 * §3: each Z_j is commuted through the final Clifford into a Weyl string and
 * evaluated on the MPS by transfer matrices).  A phase op whose op_param entry
 * is b >= 0 is diag(e^{i phi}) with phi = (0, theta[(d-1)b], ...,
 * theta[(d-1)b + d-2]); op_param -1 (or op_param NULL) keeps the op's own phi.
 * The derivative is taken with the method's discrete decisions (disentangler
 * choices and the kept rank of every factorisation) frozen at the recording
 * point theta0, which makes the truncated forward pass a smooth function of
 * theta.  It is computed in reverse mode: replay with checkpoints before every
 * gate, then gate by gate a taped replay and its reverse sweep through the MPO
 * site maps, the disentangler unitaries and the truncated factorisations.
 *
 * Workspace: one device buffer; its first gcamps_workspace_bytes(cfg) bytes
 * (rounded up to 256) hold the state, the rest is the arena for checkpoints,
 * the tape of one gate and the adjoint tensors.  ECAPACITY when the arena is
 * too small.  The gcamps_grad object owns its state and stream use; it must not
 * outlive the workspace.
 * ------------------------------------------------------------------------- */
typedef struct gcamps_grad gcamps_grad;

/* Run the circuit `ops` at theta0 (= theta) with the ordinary forward pass and
 * record the decisions; *loss (may be NULL) receives L(theta0).
 * op_param: n_ops ints (entries of Clifford ops are ignored) or NULL;
 * n_theta: multiple of d - 1 covering every parameter block used.
 * Errors: EINVAL, EUNSUPPORTED, EWORKSPACE, ECAPACITY, ENUMERIC, EDEVICE. */
int32_t gcamps_grad_record(const gcamps_config* cfg, const gcamps_op* ops, int64_t n_ops,
                           const int32_t* op_param, const double* theta, int32_t n_theta,
                           const gcamps_candset* set, void* dev_workspace, size_t bytes,
                           void* hip_stream, gcamps_grad** out, double* loss);

/* L(theta) of the frozen replay (equals the recorded loss at theta0, bit for bit).
 * Errors: EINVAL, ECAPACITY, ENUMERIC, EDEVICE. */
int32_t gcamps_grad_loss(gcamps_grad* g, const double* theta, double* loss);

/* dL/dtheta (n_theta host doubles) of the frozen replay at theta, and L(theta)
 * into *loss (may be NULL).  Errors: EINVAL, ECAPACITY, ENUMERIC, EDEVICE. */
int32_t gcamps_grad_gradient(gcamps_grad* g, const double* theta, double* loss, double* grad);

/* Statistics (8 doubles): [0] checkpointed replay and loss adjoint of the last
 * gradient in ms, [1] its reverse sweep in ms, [2] peak arena bytes, [3] taped steps,
 * [4] non-Clifford gates, [5] recording pass in ms, [6] recorded factorisations,
 * [7] recorded disentangler choices. */
int32_t gcamps_grad_stats(gcamps_grad* g, double out[8]);

/* Release the gradient object; NULL is a no-op. */
int32_t gcamps_grad_destroy(gcamps_grad* g);

/* Thread-local message for the last failed call on this thread. */
const char* gcamps_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* GCAMPS_H */
