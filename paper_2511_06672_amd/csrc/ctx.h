// Host-side state of one GCAMPS simulation (gcamps_ctx): workspace carving, the bottom
// loop of the method (commute, MPO, compression, disentangling sweeps) and, for the
// gradient, recording and frozen replay of the same steps.
#pragma once

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "kernels.h"

namespace gc {

struct Layout {
  size_t slot_elems, theta_elems, mcap, m_pad, ncand, ntp;
  int nslots;
  size_t off_slots, off_theta, off_G, off_U, off_Z, off_Utmp, off_B, off_B2, off_sig2, off_sig, off_lam,
      off_perm, off_eigG, off_eigV, off_flags, off_s2, off_s2w, off_wlist, off_partial, off_nbuf, nbuf_bytes, off_q64, off_q32,
      off_rtab, off_qinv, off_tab, off_target, off_weyl, off_err, off_status, off_luts, off_sites, off_dense,
      dense_dim, off_pcst, total;
};

Layout make_layout(const gcamps_config& c);

// ----------------------------------------------------------------- gradient support
// Bump allocator over a caller-provided device region (checkpoints, tape, adjoints).
struct Arena {
  char* base = nullptr;
  size_t cap = 0, used = 0, peak = 0;
  template <typename T>
  T* take(size_t count) {
    const size_t bytes = (count * sizeof(T) + 255) & ~size_t(255);
    GC_CHECK(used + bytes <= cap, GCAMPS_ECAPACITY,
             "gradient arena exhausted after " + std::to_string(used >> 20) + " MiB (pass a larger workspace)");
    T* p = reinterpret_cast<T*>(base + used);
    used += bytes;
    peak = std::max(peak, used);
    return p;
  }
};

// One factorisation as the reverse sweep needs it: W is the wide orientation of the split
// matrix M (W = M when p <= q, else M^H; m x kW), U (m x m) the eigenbasis of W W^H,
// B = U^H W, sig the singular values in descending order, perm their rows, k the kept rank.
struct FactRec {
  z64* U = nullptr;
  z64* B = nullptr;
  double* sig = nullptr;
  int* perm = nullptr;
  int m = 0, kW = 0, k = 0, p = 0, q = 0, wide = 0, left = 0, renorm = 0;
};

// Layout of a recorded factorisation decision (rank log entry).
constexpr int kPass2Bit = 30;
constexpr int32_t kRankMask = (1 << kPass2Bit) - 1;

enum TapeKind { TAPE_ABSORB_R = 0, TAPE_ABSORB_L = 1, TAPE_MPO = 2, TAPE_THETA = 3 };

// One step of the bottom loop, recorded for the reverse sweep.
//   ABSORB_R at i: (L, R) = split(A_i); A_i <- L; A_{i+1} <- R A_{i+1}    (x0 = old A_{i+1})
//   ABSORB_L at i: (L, R) = split(A_i); A_i <- R; A_{i-1} <- A_{i-1} L    (x0 = old A_{i-1})
//   MPO at i     : A_i <- MPO site tensor of kind mpo_kind            (x0 = old A_i, kinds 0, 3)
//   THETA at i   : (L, R) = split(Q_c A_i A_{i+1}); A_i <- L; A_{i+1} <- R (x0, x1 = old A_i, A_{i+1})
struct TapeOp {
  int kind = 0, site = 0;
  FactRec f;
  z64* x0 = nullptr;
  z64* x1 = nullptr;
  int d0[2] = {0, 0}, d1[2] = {0, 0};  // (rows, cols) of x0 and x1 as matrices
  int mpo_kind = 0, dx = 0, dz = 0, cstar = 0, chil = 0, chir = 0;
};

// Weyl string P = C^dagger W C of a gate or an observable (tau^p X^x Z^z per site) and its
// support [l, r].
struct GateRec {
  int l = 0, r = 0, p = 0, sd = 0;
  std::vector<int> x, z;
};

}  // namespace gc

using namespace gc;

struct gcamps_ctx {
  gcamps_config cfg{};
  Layout lay{};
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  int d = 0, n = 0;
  bool poisoned = false;
  // device regions
  int *tx = nullptr, *tz = nullptr, *tp = nullptr, *target = nullptr, *derr = nullptr, *dsites = nullptr;
  uint32_t* dluts = nullptr;
  DevWeyl* weyl = nullptr;
  DevStatus* st = nullptr;
  PcState* pcst = nullptr;  // rank-reduction state (device)
  void* scratch_dev = nullptr;  // device address of the library's static scratch on this ctx's GPU
  z64 *theta = nullptr, *G = nullptr, *U = nullptr, *Z = nullptr, *Utmp = nullptr, *B = nullptr, *B2 = nullptr;
  double *sig2 = nullptr, *sig = nullptr, *lam = nullptr, *s2 = nullptr, *s2w = nullptr, *partial = nullptr;
  void* nbuf = nullptr;
  int *perm = nullptr, *wlist = nullptr;
  z64* q64 = nullptr;
  c32* q32 = nullptr;
  z64* rtab = nullptr;  // replica-scoring tables of the candidate set (replica mode only)
  uint32_t* qinv = nullptr;
  EigWork eig{};
  // MPS
  std::vector<z64*> site;
  z64* Lbuf = nullptr;
  z64* Rbuf = nullptr;
  z64* spare = nullptr;
  std::vector<int> chi;  // chi[0..n], bond j between sites j-1 and j
  int centre = 0;
  // candidates
  int ncand = 0;
  uint64_t cand_uid = 0;
  // pinned staging
  char* pinned = nullptr;
  char* rb = nullptr;  // pinned read-back block (status, Cholesky state, eigensolver flags)
  size_t pinned_bytes = 0;
  hipEvent_t stage_ev = nullptr;
  bool stage_pending = false;
  hipEvent_t ev0 = nullptr, ev1 = nullptr, ev2 = nullptr, ev3 = nullptr;
  hipEvent_t evf0 = nullptr, evf1 = nullptr;  // around one factorisation (Gram to truncation rule)
  hipEvent_t evm0 = nullptr, evm1 = nullptr;  // around one gate's MPO launches
  bool mpo_pending = false;                   // evm0/evm1 recorded and not yet accumulated
  std::vector<hipEvent_t> gram_ev;  // event pairs around the Gram-purity launches of one bond
  // host state
  double f_est = 1.0;
  std::vector<int32_t> choice_log;
  int64_t gates = 0;
  double stats[16] = {0};
  // [0] factorisations, [1] their SVD flops by the R-SVD count 4 (6 p q^2 + 20 q^3) (p >= q),
  // [2] their device ms (Gram to truncation rule, second pass included), [3] MPO site launches,
  // [4] MPO bytes (each site tensor read once and its product written once), [5] MPO device ms
  double kstats[8] = {0};
  // rank reduction of the rotated-tensor splits: [0] reduced factorisations, [1] their summed
  // basis sizes r, [2] their summed sides m, [3] attempts that fell back to the full basis
  double stats_red[4] = {0};
  int last_basis = 0;  // singular values resolved by the last factorisation (m, or r when reduced)
  bool trace_fact = std::getenv("GCAMPS_TRACE_FACT") != nullptr;
  // gradient: recording and frozen replay (all null in ordinary use)
  std::vector<int32_t>* rank_rec = nullptr;          // kept rank of every factorisation
  std::vector<GateRec>* gate_rec = nullptr;          // Weyl string of every non-Clifford gate
  const std::vector<int32_t>* rank_frz = nullptr;    // forced ranks, consumed from rank_pos
  size_t rank_pos = 0;
  const std::vector<int32_t>* choice_frz = nullptr;  // forced choices, consumed from choice_pos
  size_t choice_pos = 0;
  std::vector<TapeOp>* tape = nullptr;               // reverse-sweep record of the replayed steps
  Arena* arena = nullptr;                            // storage of the tape
  FactRec last_fact;

  ~gcamps_ctx() {
    if (pinned) (void)hipHostFree(pinned);
    if (rb) (void)hipHostFree(rb);
    if (stage_ev) (void)hipEventDestroy(stage_ev);
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
    if (ev2) (void)hipEventDestroy(ev2);
    if (ev3) (void)hipEventDestroy(ev3);
    for (hipEvent_t e : {evf0, evf1, evm0, evm1})
      if (e) (void)hipEventDestroy(e);
    for (auto e : gram_ev) (void)hipEventDestroy(e);
  }

  // ---------------------------------------------------------------- staging
  char* stage_begin() {
    if (stage_pending) {
      GC_HIP(hipEventSynchronize(stage_ev));
      stage_pending = false;
    }
    return pinned;
  }
  void stage_upload(void* dst, size_t bytes) {
    GC_HIP(hipMemcpyAsync(dst, pinned, bytes, hipMemcpyHostToDevice, stream));
    GC_HIP(hipEventRecord(stage_ev, stream));
    stage_pending = true;
  }
  static_assert(sizeof(DevStatus) <= kRbPcState && kRbPcState + sizeof(PcState) <= kRbEig &&
                    kRbWeyl + sizeof(DevWeyl) <= kRbWeylErr && kRbWeylErr + sizeof(int) <= kRbBytes,
                "read-back block layout");
  void read_status(DevStatus& h) {  // through pinned memory: no staging copy
    GC_HIP(hipMemcpyAsync(rb + kRbStatus, st, sizeof(DevStatus), hipMemcpyDeviceToHost, stream));
    GC_HIP(hipStreamSynchronize(stream));
    std::memcpy(&h, rb + kRbStatus, sizeof(DevStatus));
  }

  int dim_l(int i) const { return chi[i]; }
  int dim_r(int i) const { return chi[i + 1]; }

  // ---------------------------------------------------------------- factorisation
  // Split M (p x q, row-major) into L (p x k) R (k x q).  mode 0: truncation rule with
  // renormalisation; mode 1: exact (rank floor only).  left_ortho: L has orthonormal columns
  // (else R has orthonormal rows).  Returns the status block of the final pass.
  // reduce: a truncating split of the bottom loop (mode 0 with a positive cutoff, outside
  // gradient recording and replay): the eigensolver runs on the r x r matrix of a pivoted
  // Cholesky factorisation of the Gram, which drops what the cutoff could never keep (rotated
  // two-site tensors often have rank far below m) and preconditions the Jacobi sweeps.
  DevStatus factorize(const z64* M, int p, int q, int mode, int left_ortho, z64* Lout, z64* Rout,
                      bool reduce = false) {
    const bool wide = p <= q;
    const int m = wide ? p : q, kW = wide ? q : p;
    GC_CHECK((size_t)m <= lay.mcap && (size_t)m * kW <= lay.slot_elems, GCAMPS_ECAPACITY,
             "factorisation exceeds workspace capacity");
    const z64 one = {1.0, 0.0};
    GC_HIP(hipEventRecord(evf0, stream));
    auto gram = [&]() {
      if (wide)
        launch_zgemm(stream, 0, 1, m, m, q, M, q, M, q, G, m, one, 0, 1);
      else
        launch_zgemm(stream, 1, 0, m, m, p, M, q, M, q, G, m, one, 0, 1);
    };
    gram();
    // basis: nb columns of U (ld ldu); tail: weight outside the basis, always discarded
    int nb = m, ldu = m;
    int sw_h = 0, sw_main = 0, sw_p2 = 0;  // sweeps of the eigen-decompositions (trace only)
    const double* tail = nullptr;
    const bool try_reduce = reduce && mode == 0 && cfg.cutoff > 0.0 && m > kReduceMinM && m <= kReduceMaxM && !tape &&
                            !rank_rec && !rank_frz;
    bool reduced = false;
    if (try_reduce) {
      // stop once the Schur complement's trace is below min(1e-14, cutoff / 2m) of the trace: then
      // its directions hold less than the cutoff even all together, and no eigenvalue moves by
      // more than the Gram's own rounding
      const double tol_rel = std::min(1e-14, cfg.cutoff / (2.0 * m));
      PcState* hsp = reinterpret_cast<PcState*>(rb + kRbPcState);
      const int r = pchol_reduce(stream, G, m, m, Z, m, tol_rel, m, sig, perm, pcst, hsp);
      const PcState hs = *hsp;
      if (hs.done && r >= 1) {
        // H = L^H L = Y lam Y^H with relative accuracy, so that the columns of L Y are
        // orthogonal to ~1e-14 of their norms even where lam is tiny (an absolute criterion
        // leaves them off by ~tr H / lam times that)
        launch_zgemm(stream, 1, 0, r, r, m, Z, m, Z, m, Utmp, r, one, 0, 1);
        eig_hermitian(stream, Utmp, r, r, G, r, lam, 1, eig, st, &sw_h);
        launch_zgemm(stream, 0, 0, m, r, r, Z, m, G, r, U, r, one, 0, 0);     // L Y
        launch_normalize_cols(stream, U, m, r, r);
        orthonormalize_cols(stream, U, Z, Utmp, m, r, 2);
        nb = r;
        ldu = r;
        tail = &pcst->tres;
        reduced = true;
        stats_red[0] += 1;
        stats_red[1] += r;
        stats_red[2] += m;
      } else {
        gram();  // no useful reduction: the full eigen-decomposition of the (recomputed) Gram
        stats_red[3] += 1;
      }
    }
    if (!reduced) eig_hermitian(stream, G, m, m, U, m, lam, 0, eig, st, &sw_main);
    if (wide)
      launch_zgemm(stream, 1, 0, nb, q, m, U, ldu, M, q, B, q, one, 0, 0);
    else
      launch_zgemm(stream, 1, 1, nb, p, m, U, ldu, M, q, B, p, one, 0, 0);
    if (reduced) {
      // Rayleigh-Ritz on the reduced basis: B B^H = U^H G U with the full Gram, so its
      // eigenvalues err by the square of the basis error where L L^H's err by tr S
      launch_zgemm(stream, 0, 1, nb, nb, kW, B, kW, B, kW, G, nb, one, 0, 1);
      // nearly diagonal already: the pre-check usually finds nothing to rotate, and then the
      // eigenvectors are the identity and U and B stay as they are
      eig_hermitian(stream, G, nb, nb, Z, nb, lam, 0, eig, st, &sw_main, true);
      if (sw_main != 0) {
        launch_zgemm(stream, 0, 0, m, nb, nb, U, ldu, Z, nb, Utmp, ldu, one, 0, 0);
        std::swap(U, Utmp);
        launch_zgemm(stream, 1, 0, nb, kW, nb, Z, nb, B, kW, B2, kW, one, 0, 0);
        std::swap(B, B2);
      }
    }
    // recorded decision: kept rank in the low bits, bit 30 = the accurate second pass ran
    int force_k = 0, force_pass2 = -1;
    if (rank_frz) {
      GC_CHECK(rank_pos < rank_frz->size(), GCAMPS_EINVAL, "frozen replay ran past the recorded ranks");
      const int32_t v = (*rank_frz)[rank_pos++];
      force_k = v & kRankMask;
      force_pass2 = (v >> kPass2Bit) & 1;
    }
    launch_rownorm2(stream, B, nb, kW, kW, sig2);
    launch_trunc(stream, sig2, nb, cfg.cutoff, cfg.chi_max, mode, force_k, perm, sig, st, tail);
    GC_HIP(hipEventRecord(evf1, stream));
    DevStatus h;
    read_status(h);
    GC_CHECK(nb > kSmallEig || h.converged, GCAMPS_ENUMERIC, "eigensolver did not converge");
    stats[5] += 8.0 * (double)m * m * kW * 2.0;
    const bool pass2 = force_pass2 >= 0 ? force_pass2 == 1 : h.need_pass2 != 0;
    if (pass2) {
      // accurate second pass on the nearly diagonal Gram of B (relative criterion)
      launch_zgemm(stream, 0, 1, nb, nb, kW, B, kW, B, kW, G, nb, one, 0, 1);
      eig_hermitian(stream, G, nb, nb, Z, nb, lam, 1, eig, st, &sw_p2);
      launch_zgemm(stream, 0, 0, m, nb, nb, U, ldu, Z, nb, Utmp, ldu, one, 0, 0);
      std::swap(U, Utmp);
      launch_zgemm(stream, 1, 0, nb, kW, nb, Z, nb, B, kW, B2, kW, one, 0, 0);
      std::swap(B, B2);
      launch_rownorm2(stream, B, nb, kW, kW, sig2);
      launch_trunc(stream, sig2, nb, cfg.cutoff, cfg.chi_max, mode, force_k, perm, sig, st, tail);
      GC_HIP(hipEventRecord(evf1, stream));
      read_status(h);
      GC_CHECK(nb > kSmallEig || h.converged, GCAMPS_ENUMERIC, "eigensolver did not converge (second pass)");
      stats[5] += 8.0 * (double)nb * nb * kW * 2.0;
    }
    GC_CHECK(std::isfinite(h.eps) && h.kept >= 1, GCAMPS_ENUMERIC, "factorisation produced non-finite values");
    {  // both events have completed: read_status synchronised the stream after evf1
      float fms = 0.0f;
      GC_HIP(hipEventElapsedTime(&fms, evf0, evf1));
      const double pl = std::max(p, q), ql = std::min(p, q);
      kstats[0] += 1;
      kstats[1] += 4.0 * (6.0 * pl * ql * ql + 20.0 * ql * ql * ql);
      kstats[2] += fms;
      if (trace_fact)  // GCAMPS_TRACE_FACT: one line per factorisation on stderr
        std::fprintf(stderr, "gcamps-fact m=%d k=%d mode=%d reduce=%d basis=%d kept=%d pass2=%d ms=%.3f sweeps=%d/%d/%d\n",
                     m, kW, mode, reduced ? 1 : 0, nb, h.kept, pass2 ? 1 : 0, fms, sw_h, sw_main, sw_p2);
    }
    if (rank_rec) rank_rec->push_back(h.kept | (pass2 ? (1 << kPass2Bit) : 0));
    if (tape) {
      FactRec& f = last_fact;
      f.m = m;
      f.kW = kW;
      f.k = h.kept;
      f.p = p;
      f.q = q;
      f.wide = wide ? 1 : 0;
      f.left = left_ortho;
      f.renorm = mode == 0 ? 1 : 0;
      f.U = arena->take<z64>((size_t)m * m);
      f.B = arena->take<z64>((size_t)m * kW);
      f.sig = arena->take<double>(m);
      f.perm = arena->take<int>(m);
      launch_copy(stream, f.U, U, (size_t)m * m);
      launch_copy(stream, f.B, B, (size_t)m * kW);
      GC_HIP(hipMemcpyAsync(f.sig, sig, m * sizeof(double), hipMemcpyDeviceToDevice, stream));
      GC_HIP(hipMemcpyAsync(f.perm, perm, m * sizeof(int), hipMemcpyDeviceToDevice, stream));
    }
    launch_emit(stream, wide ? 1 : 0, left_ortho, mode == 0 ? 1 : 0, p, q, h.kept, U, ldu, B, kW, perm, sig, Lout,
                Rout);
    last_basis = nb;
    return h;
  }

  // Kept rank of the split's truncation rule on M (p x q): the first pass and, where the rank
  // floor matters, the relative-accuracy second pass of factorize(), without the factors, the
  // counters or any record (the bond-dimension criterion on bonds above the batched kernel's
  // size).
  int split_rank(const z64* M, int p, int q) {
    const bool wide = p <= q;
    const int m = wide ? p : q, kW = wide ? q : p;
    GC_CHECK((size_t)m <= lay.mcap && (size_t)m * kW <= lay.slot_elems, GCAMPS_ECAPACITY,
             "factorisation exceeds workspace capacity");
    const z64 one = {1.0, 0.0};
    if (wide)
      launch_zgemm(stream, 0, 1, m, m, q, M, q, M, q, G, m, one, 0, 1);
    else
      launch_zgemm(stream, 1, 0, m, m, p, M, q, M, q, G, m, one, 0, 1);
    eig_hermitian(stream, G, m, m, U, m, lam, 0, eig, st, nullptr);
    if (wide)
      launch_zgemm(stream, 1, 0, m, q, m, U, m, M, q, B, q, one, 0, 0);
    else
      launch_zgemm(stream, 1, 1, m, p, m, U, m, M, q, B, p, one, 0, 0);
    launch_rownorm2(stream, B, m, kW, kW, sig2);
    launch_trunc(stream, sig2, m, cfg.cutoff, cfg.chi_max, 0, 0, perm, sig, st);
    DevStatus h;
    read_status(h);
    GC_CHECK(m > kSmallEig || h.converged, GCAMPS_ENUMERIC, "eigensolver did not converge");
    if (h.need_pass2) {
      launch_zgemm(stream, 0, 1, m, m, kW, B, kW, B, kW, G, m, one, 0, 1);
      eig_hermitian(stream, G, m, m, Z, m, lam, 1, eig, st, nullptr);
      launch_zgemm(stream, 1, 0, m, kW, m, Z, m, B, kW, B2, kW, one, 0, 0);
      launch_rownorm2(stream, B2, m, kW, kW, sig2);
      launch_trunc(stream, sig2, m, cfg.cutoff, cfg.chi_max, 0, 0, perm, sig, st);
      read_status(h);
      GC_CHECK(m > kSmallEig || h.converged, GCAMPS_ENUMERIC, "eigensolver did not converge (second pass)");
    }
    GC_CHECK(std::isfinite(h.eps) && h.kept >= 1, GCAMPS_ENUMERIC, "factorisation produced non-finite values");
    return h.kept;
  }

  // ---------------------------------------------------------------- centre moves (exact)
  // copy of a site tensor into the tape arena (reverse sweep input)
  z64* keep_copy(const z64* src, size_t count) {
    z64* dst = arena->take<z64>(count);
    launch_copy(stream, dst, src, count);
    return dst;
  }
  void tape_absorb(int kind, int i, const z64* nb, int rows, int cols) {
    TapeOp op;
    op.kind = kind;
    op.site = i;
    op.f = last_fact;
    op.x0 = keep_copy(nb, (size_t)rows * cols);
    op.d0[0] = rows;
    op.d0[1] = cols;
    tape->push_back(op);
  }

  void move_right(int i) {  // centre i -> i+1
    const int p = chi[i] * d, q = chi[i + 1];
    DevStatus h = factorize(site[i], p, q, 1, 1, Lbuf, Rbuf);
    const int k = h.kept;
    if (tape) tape_absorb(TAPE_ABSORB_R, i, site[i + 1], q, d * chi[i + 2]);
    std::swap(site[i], Lbuf);
    const int ncols = d * chi[i + 2];
    launch_zgemm(stream, 0, 0, k, ncols, q, Rbuf, q, site[i + 1], ncols, spare, ncols, z64{1.0, 0.0}, 0, 0);
    std::swap(site[i + 1], spare);
    chi[i + 1] = k;
    centre = i + 1;
  }
  void move_left(int i) {  // centre i -> i-1
    const int p = chi[i], q = d * chi[i + 1];
    DevStatus h = factorize(site[i], p, q, 1, 0, Lbuf, Rbuf);
    const int k = h.kept;
    if (tape) tape_absorb(TAPE_ABSORB_L, i, site[i - 1], chi[i - 1] * d, p);
    std::swap(site[i], Rbuf);
    const int nrows = chi[i - 1] * d;
    launch_zgemm(stream, 0, 0, nrows, k, p, site[i - 1], p, Lbuf, k, spare, k, z64{1.0, 0.0}, 0, 0);
    std::swap(site[i - 1], spare);
    chi[i] = k;
    centre = i - 1;
  }
  void move_centre(int target) {
    while (centre < target) move_right(centre);
    while (centre > target) move_left(centre);
  }

  // ---------------------------------------------------------------- bottom loop
  // P = C^dagger W C for a Weyl target W = tau^p X^x Z^z (x, z, p given as 2n+1 ints).
  GateRec extract_string(const int* xzp) {
    int* tg = reinterpret_cast<int*>(stage_begin());
    for (int i = 0; i < 2 * n + 1; ++i) tg[i] = xzp[i];
    stage_upload(target, (2 * n + 1) * sizeof(int));
    launch_weyl_extract(stream, n, d, tx, tz, tp, target, weyl, derr);
    GC_HIP(hipMemcpyAsync(rb + kRbWeyl, weyl, sizeof(DevWeyl), hipMemcpyDeviceToHost, stream));
    GC_HIP(hipMemcpyAsync(rb + kRbWeylErr, derr, sizeof(int), hipMemcpyDeviceToHost, stream));
    GC_HIP(hipStreamSynchronize(stream));
    DevWeyl P;
    int err = 0;
    std::memcpy(&P, rb + kRbWeyl, sizeof(DevWeyl));
    std::memcpy(&err, rb + kRbWeylErr, sizeof(int));
    GC_CHECK(err == 0, GCAMPS_ENUMERIC, "tableau decomposition failed");
    GateRec g;
    g.l = P.l;
    g.r = P.r;
    g.p = P.p;
    g.x.assign(P.x, P.x + n);
    g.z.assign(P.z, P.z + n);
    int sd = 0;
    for (int i = 0; i < n; ++i) sd += P.x[i] * P.z[i];
    g.sd = sd % d;
    return g;
  }

  // MPO coefficients K_b = c_b tau^{ph_b} of sum_b c_b P^b for diag(e^{i phi_j}) = sum_b c_b Z^b,
  // c_b = (1/d) sum_j e^{i phi_j} omega^{-bj}; P^b = tau^{ph_b} X^{bx} Z^{bz} per site with
  // ph_b = b p + 2 <x, z> b(b-1)/2 (mod 2d).
  MpoCoeff mpo_coeff(const GateRec& P, const double* phi) const {
    MpoCoeff co;
    for (int b = 0; b < d; ++b) {
      std::complex<double> cb = 0.0;
      for (int j = 0; j < d; ++j) cb += std::polar(1.0, phi[j] - 2.0 * M_PI * b * j / d);
      cb /= (double)d;
      const int ph = (b * P.p + 2 * P.sd * (b * (b - 1) / 2)) % (2 * d);
      std::complex<double> kb = cb * std::polar(1.0, M_PI * ph / d);
      co.k[b] = z64{kb.real(), kb.imag()};
      co.w[b] = z64{std::cos(2.0 * M_PI * b / d), std::sin(2.0 * M_PI * b / d)};
    }
    return co;
  }

  void phase_rotation(int s, const double* phi) {
    std::vector<int> xzp(2 * n + 1, 0);
    xzp[n + s] = 1;  // target Z_s
    GateRec P = extract_string(xzp.data());
    GC_CHECK(P.l >= 0, GCAMPS_ENUMERIC, "tableau decomposition failed");
    if (gate_rec) gate_rec->push_back(P);
    phase_apply(P, phi);
  }

  // Timing of one gate's MPO launches: events recorded around them and read once they have
  // completed (the compression that follows synchronises the stream).
  void settle_mpo() {
    if (!mpo_pending) return;
    GC_HIP(hipEventSynchronize(evm1));
    float ms = 0.0f;
    GC_HIP(hipEventElapsedTime(&ms, evm0, evm1));
    kstats[5] += ms;
    mpo_pending = false;
  }
  void mpo_begin() {
    settle_mpo();
    GC_HIP(hipEventRecord(evm0, stream));
  }
  void mpo_end() {
    GC_HIP(hipEventRecord(evm1, stream));
    mpo_pending = true;
  }
  // Algorithmic bytes of one MPO site launch of bond J on [l, r]: the site tensor read once and
  // its product (bonds multiplied by J inside the support) written once, complex128.
  void mpo_count(int i, int l, int r, int J) {
    const double in = (double)chi[i] * d * chi[i + 1];
    const double out = (double)chi[i] * (i > l ? J : 1) * d * chi[i + 1] * (i < r ? J : 1);
    kstats[3] += 1;
    kstats[4] += 16.0 * (in + out);
  }

  // Apply sum_b c_b P^b (P from the tableau) to the MPS and compress.
  void phase_apply(const GateRec& P, const double* phi) {
    const int l = P.l, r = P.r;
    const MpoCoeff co = mpo_coeff(P, phi);
    move_centre(l);
    mpo_begin();
    for (int i = l; i <= r; ++i) {
      int kind = (l == r) ? 3 : (i == l ? 0 : (i == r ? 2 : 1));
      mpo_count(i, l, r, d);
      if (tape) {
        TapeOp op;
        op.kind = TAPE_MPO;
        op.site = i;
        op.mpo_kind = kind;
        op.dx = P.x[i];
        op.dz = P.z[i];
        op.chil = chi[i];
        op.chir = chi[i + 1];
        if (kind == 0 || kind == 3) {
          op.x0 = keep_copy(site[i], (size_t)chi[i] * d * chi[i + 1]);
          op.d0[0] = chi[i] * d;
          op.d0[1] = chi[i + 1];
        }
        tape->push_back(op);
      }
      launch_mpo_site(stream, kind, d, chi[i], chi[i + 1], P.x[i], P.z[i], co, site[i], spare);
      std::swap(site[i], spare);
    }
    mpo_end();
    for (int j = l + 1; j <= r; ++j) chi[j] *= d;
    compress(l, r);
    gates += 1;
    stats[0] += 1;
  }

  // After an MPO on [l, r] (centre at l): exact moves to r, then truncating splits back to l
  // (§2.4); F_est absorbs the discarded weights.
  void compress(int l, int r) {
    if (r > l) {
      for (int i = l; i < r; ++i) move_right(i);
      for (int i = r; i > l; --i) {
        const int p = chi[i], q = d * chi[i + 1];
        DevStatus h = factorize(site[i], p, q, 0, 0, Lbuf, Rbuf, true);
        const int k = h.kept;
        if (tape) tape_absorb(TAPE_ABSORB_L, i, site[i - 1], chi[i - 1] * d, p);
        std::swap(site[i], Rbuf);
        const int nrows = chi[i - 1] * d;
        launch_zgemm(stream, 0, 0, nrows, k, p, site[i - 1], p, Lbuf, k, spare, k, z64{1.0, 0.0}, 0, 0);
        std::swap(site[i - 1], spare);
        chi[i] = k;
        centre = i - 1;
        f_est *= (1.0 - h.eps);
        stats[3] += h.flagged;
      }
    }
  }

  // General gate U on sites s..s+k-1 (k = 1, 2): Weyl expansion, each term commuted through the
  // Clifford, the sum applied as an MPO of bond J = number of terms, then compressed.
  void general_gate(int s, int k, const std::vector<z64>& U) {
    GC_CHECK(tape == nullptr && rank_rec == nullptr && rank_frz == nullptr, GCAMPS_EUNSUPPORTED,
             "general gates are not recorded for gradients");
    int D = 1;
    for (int t = 0; t < k; ++t) D *= d;
    // c_xz = Tr(W_xz^dagger U) / D with W_xz |v> = omega^{z . v} |v + x> (digits of site s first)
    struct Term {
      std::vector<int> x, z;
      std::complex<double> c;
    };
    std::vector<Term> terms;
    double cmax = 0.0;
    const int nx = D;  // exponent vectors x (and z) enumerate like basis states
    auto digits = [&](int v, std::vector<int>& out) {
      out.assign(k, 0);
      for (int t = k - 1; t >= 0; --t) {
        out[t] = v % d;
        v /= d;
      }
    };
    std::vector<int> xv, zv, sv, tv;
    for (int xi = 0; xi < nx; ++xi)
      for (int zi = 0; zi < nx; ++zi) {
        digits(xi, xv);
        digits(zi, zv);
        std::complex<double> acc = 0.0;
        for (int v = 0; v < D; ++v) {
          digits(v, sv);
          int row = 0, dot = 0;
          for (int t = 0; t < k; ++t) {
            row = row * d + (sv[t] + xv[t]) % d;
            dot += zv[t] * sv[t];
          }
          const z64 uv = U[(size_t)row * D + v];  // <v + x| U |v>
          acc += std::polar(1.0, -2.0 * M_PI * (double)(dot % d) / d) * std::complex<double>(uv.re, uv.im);
        }
        acc /= (double)D;
        cmax = std::max(cmax, std::abs(acc));
        terms.push_back({xv, zv, acc});
      }
    std::vector<Term> kept;
    for (auto& t : terms)
      if (std::abs(t.c) > 1e-14 * cmax) kept.push_back(t);
    const int J = (int)kept.size();
    GC_CHECK(J <= std::max(d, cfg.max_gate_terms), GCAMPS_ECAPACITY,
             "gate has " + std::to_string(J) + " Weyl terms; raise max_gate_terms");
    // commute every term through C: P_j = C^dagger W_j C
    std::vector<GateRec> P(J);
    int l = n, r = -1;
    for (int j = 0; j < J; ++j) {
      bool ident = true;
      for (int t = 0; t < k; ++t) ident = ident && kept[j].x[t] == 0 && kept[j].z[t] == 0;
      if (ident) {  // C^dagger I C = I: no support, no phase
        P[j].x.assign(n, 0);
        P[j].z.assign(n, 0);
        P[j].p = 0;
        continue;
      }
      std::vector<int> xzp(2 * n + 1, 0);
      for (int t = 0; t < k; ++t) {
        xzp[s + t] = kept[j].x[t];
        xzp[n + s + t] = kept[j].z[t];
      }
      P[j] = extract_string(xzp.data());
      GC_CHECK(P[j].l >= 0, GCAMPS_ENUMERIC, "tableau decomposition failed");
      l = std::min(l, P[j].l);
      r = std::max(r, P[j].r);
    }
    if (r < l) l = r = s;  // U proportional to the identity
    MpoTerms tm;
    for (int j = 0; j < J; ++j) {
      const std::complex<double> cj = kept[j].c * std::polar(1.0, M_PI * P[j].p / d);
      tm.coef[j] = z64{cj.real(), cj.imag()};
    }
    move_centre(l);
    mpo_begin();
    for (int i = l; i <= r; ++i) {
      const int kind = (l == r) ? 3 : (i == l ? 0 : (i == r ? 2 : 1));
      for (int j = 0; j < J; ++j) {
        tm.x[j] = P[j].x[i];
        tm.z[j] = P[j].z[i];
      }
      mpo_count(i, l, r, J);
      launch_mpo_sum_site(stream, kind, d, J, chi[i], chi[i + 1], tm, site[i], spare);
      std::swap(site[i], spare);
    }
    mpo_end();
    for (int j = l + 1; j <= r; ++j) chi[j] *= J;
    compress(l, r);
    gates += 1;
    stats[0] += 1;
  }

  // Full-set scores of bond (i, i+1) in the configured mode, to host memory; commits nothing.
  void score_bond(int i, double* out) {
    move_centre(i);
    const int cl = chi[i], cm = chi[i + 1], cr = chi[i + 2];
    launch_zgemm(stream, 0, 0, cl * d, d * cr, cm, site[i], cm, site[i + 1], d * cr, theta, d * cr, z64{1.0, 0.0},
                 0, 0);
    const size_t pcap = lay.ncand * lay.ntp * 2;
    launch_score(stream, cfg.score_prec, d, cl, cr, theta, q64, q32, nullptr, ncand, nullptr, s2, partial, pcap, nbuf,
                 lay.nbuf_bytes, nullptr, 0, nullptr, rtab);
    GC_HIP(hipMemcpyAsync(out, s2, (size_t)ncand * sizeof(double), hipMemcpyDeviceToHost, stream));
    GC_HIP(hipStreamSynchronize(stream));
  }

  void disentangle(int* out_sweeps, int* out_changed) {
    GC_CHECK(ncand >= 1, GCAMPS_EINVAL, "no candidate set attached");
    int sweeps = 0, changed_total = 0;
    const int prec = cfg.score_prec;
    const bool frozen = choice_frz != nullptr;
    for (int sw = 0; sw < cfg.max_sweeps; ++sw) {
      ++sweeps;
      const bool ltr = (sw % 2 == 0);
      int changed = 0;
      for (int t = 0; t < n - 1; ++t) {
        const int i = ltr ? t : n - 2 - t;
        move_centre(ltr ? i : i + 1);
        const int cl = chi[i], cm = chi[i + 1], cr = chi[i + 2];
        const int mm = std::min(cl * d, d * cr), kk = std::max(cl * d, d * cr);
        int gram_used = 0;
        bool shortcut = false;
        if (frozen) {
          // replay: the recorded choice replaces scoring and selection
          GC_CHECK(choice_pos < choice_frz->size(), GCAMPS_EINVAL, "frozen replay ran past the recorded choices");
          const int c = (*choice_frz)[choice_pos++];
          GC_CHECK(c >= 0 && c < ncand, GCAMPS_EINVAL, "recorded choice outside the candidate set");
          int* ci = reinterpret_cast<int*>(stage_begin());
          *ci = c;
          stage_upload(&st->cstar, sizeof(int));
          shortcut = (c == 0 && mm > kSmallEig);
          if (!shortcut) {
            launch_zgemm(stream, 0, 0, cl * d, d * cr, cm, site[i], cm, site[i + 1], d * cr, theta, d * cr,
                         z64{1.0, 0.0}, 0, 0);
            launch_apply_q(stream, d, cl, cr, st, q64, theta);
          }
        } else {
          launch_zgemm(stream, 0, 0, cl * d, d * cr, cm, site[i], cm, site[i + 1], d * cr, theta, d * cr,
                       z64{1.0, 0.0}, 0, 0);
          const size_t pcap = lay.ncand * lay.ntp * 2;
          const double pflops = 4.0 * mm * mm * kk + 8.0 * std::pow((double)d, 4) * cl * cr;
          GC_HIP(hipEventRecord(ev0, stream));
          launch_score(stream, prec, d, cl, cr, theta, q64, q32, nullptr, ncand, nullptr, s2, partial, pcap, nbuf,
                       lay.nbuf_bytes, gram_ev.data(), (int)gram_ev.size(), &gram_used, rtab);
          GC_HIP(hipEventRecord(ev1, stream));
          if (cfg.criterion == GCAMPS_CRITERION_BOND_DIM) {
            if (mm <= kRankMaxM && (size_t)(mm + (mm & 1)) * kk <= kRankMaxElems) {
              launch_cand_rank(stream, d, cl, cr, theta, q64, ncand, cfg.cutoff, cfg.chi_max, wlist);
            } else {
              // larger bonds: every candidate's rotated tensor through the split's own
              // factorisation (Lbuf holds Q_c Theta; the split of the bond comes later)
              std::vector<int32_t> ranks(ncand);
              for (int c = 0; c < ncand; ++c) {
                launch_rotate_copy(stream, d, cl, cr, c, q64, theta, Lbuf);
                ranks[c] = split_rank(Lbuf, cl * d, d * cr);
              }
              int32_t* hr = reinterpret_cast<int32_t*>(stage_begin());
              std::memcpy(hr, ranks.data(), (size_t)ncand * sizeof(int32_t));
              stage_upload(wlist, (size_t)ncand * sizeof(int32_t));
            }
            launch_select_rank(stream, ncand, wlist, s2, cfg.tie_tol, st);
          } else if (prec == GCAMPS_SCORE_FP64) {
            launch_select(stream, ncand, s2, cfg.tie_tol, st);
          } else {
            launch_window(stream, ncand, s2, cfg.near_tie, wlist, st);
            GC_HIP(hipEventRecord(ev2, stream));
            launch_score(stream, GCAMPS_SCORE_FP64, d, cl, cr, theta, q64, q32, wlist, ncand, &st->nwindow, s2w,
                         partial, pcap, nbuf, lay.nbuf_bytes);
            GC_HIP(hipEventRecord(ev3, stream));
            launch_select_window(stream, wlist, s2w, cfg.tie_tol, st);
          }
          if (prec == GCAMPS_SCORE_REPLICA && mm > kScoreSmallM) {
            // Gram of Theta over the larger bond (Hermitian half), pair sum, one d^8 dot per candidate
            const double X = std::min(cl, cr), Y = std::max(cl, cr), XD = X * d * d, R2 = std::pow((double)d, 8);
            stats[4] += 4.0 * XD * XD * Y + 8.0 * X * (X + 1) / 2 * R2 + 2.0 * ncand * R2;
          } else {
            stats[4] += (double)ncand * pflops;
          }
          stats[10] += 1;
          launch_apply_q(stream, d, cl, cr, st, q64, theta);
          launch_tableau_right_mult(stream, n, d, i, st, qinv, tx, tz, tp);
          // When the identity is kept, Theta = A_i A_{i+1} with the neighbour of the centre
          // orthonormal (right-orthonormal A_{i+1} when sweeping left to right, left-orthonormal
          // A_i otherwise), so Theta's Schmidt values are those of the centre tensor alone and the
          // split only needs the factorisation of that (smaller) tensor.
          if (mm > kSmallEig) {
            DevStatus pre;
            read_status(pre);
            shortcut = (pre.cstar == 0);
          }
        }
        DevStatus h;
        if (shortcut && ltr) {
          h = factorize(site[i], cl * d, cm, 0, 1, Lbuf, Rbuf, true);
          const int k = h.kept;
          if (tape) tape_absorb(TAPE_ABSORB_R, i, site[i + 1], cm, d * cr);
          launch_zgemm(stream, 0, 0, k, d * cr, cm, Rbuf, cm, site[i + 1], d * cr, spare, d * cr, z64{1.0, 0.0}, 0, 0);
          std::swap(site[i], Lbuf);
          std::swap(site[i + 1], spare);
        } else if (shortcut) {
          h = factorize(site[i + 1], cm, d * cr, 0, 0, Lbuf, Rbuf, true);
          const int k = h.kept;
          if (tape) tape_absorb(TAPE_ABSORB_L, i + 1, site[i], cl * d, cm);
          launch_zgemm(stream, 0, 0, cl * d, k, cm, site[i], cm, Lbuf, k, spare, k, z64{1.0, 0.0}, 0, 0);
          std::swap(site[i + 1], Rbuf);
          std::swap(site[i], spare);
        } else {
          TapeOp op;
          if (tape) {
            op.kind = TAPE_THETA;
            op.site = i;
            op.x0 = keep_copy(site[i], (size_t)cl * d * cm);
            op.d0[0] = cl * d;
            op.d0[1] = cm;
            op.x1 = keep_copy(site[i + 1], (size_t)cm * d * cr);
            op.d1[0] = cm;
            op.d1[1] = d * cr;
            op.chil = cl;
            op.chir = cr;
          }
          h = factorize(theta, cl * d, d * cr, 0, ltr ? 1 : 0, Lbuf, Rbuf, true);
          if (tape) {
            op.f = last_fact;
            op.cstar = h.cstar;
            tape->push_back(op);
          }
          std::swap(site[i], Lbuf);
          std::swap(site[i + 1], Rbuf);
        }
        stats[14] += shortcut ? 1 : 0;
        if (!frozen) {
          float ms = 0.f;
          GC_HIP(hipEventElapsedTime(&ms, ev0, ev1));
          stats[6] += ms;
          if (gram_used > 0) {  // Gram-purity kernel alone: algorithmic 4 m^2 k flop per candidate
            for (int e = 0; e < gram_used; ++e) {
              float gm = 0.f;
              GC_HIP(hipEventElapsedTime(&gm, gram_ev[2 * e], gram_ev[2 * e + 1]));
              stats[12] += gm;
            }
            stats[11] += gram_used;
            stats[13] += (double)ncand * 4.0 * mm * mm * kk;
            stats[15] += (double)ncand * mm * kk * (prec == GCAMPS_SCORE_FP64 ? 16.0 : 8.0);
          }
          stats[1] += 1;
          if (prec != GCAMPS_SCORE_FP64) {
            const double pflops = 4.0 * mm * mm * kk + 8.0 * std::pow((double)d, 4) * cl * cr;
            stats[2] += h.nwindow;
            stats[8] += (double)h.nwindow * pflops;
            GC_HIP(hipEventElapsedTime(&ms, ev2, ev3));
            stats[9] += ms;
          }
        }
        chi[i + 1] = h.kept;
        centre = ltr ? i + 1 : i;
        f_est *= (1.0 - h.eps);
        stats[3] += h.flagged;
        choice_log.push_back((int32_t)(gates - 1));
        choice_log.push_back(sw);
        choice_log.push_back(i);
        choice_log.push_back(h.cstar);
        if (h.cstar != 0) ++changed;
      }
      changed_total += changed;
      if (changed == 0) break;
    }
    if (out_sweeps) *out_sweeps = sweeps;
    if (out_changed) *out_changed = changed_total;
  }

  // ---------------------------------------------------------------- state save / restore
  // |0...0>: every site tensor (1, d, 1) = e_0, centre 0, fidelity estimate 1.
  void reset_mps() {
    chi.assign(n + 1, 1);
    centre = 0;
    f_est = 1.0;
    for (int i = 0; i < n; ++i) {
      GC_HIP(hipMemsetAsync(site[i], 0, d * sizeof(z64), stream));
      z64* one = reinterpret_cast<z64*>(stage_begin());
      *one = z64{1.0, 0.0};
      stage_upload(site[i], sizeof(z64));
    }
  }
  size_t mps_elems() const {
    size_t t = 0;
    for (int i = 0; i < n; ++i) t += (size_t)chi[i] * d * chi[i + 1];
    return t;
  }

};
