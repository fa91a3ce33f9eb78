// Gradient of an observable loss with respect to phase-gate angles (reverse mode).
//
// Loss: L(theta) = Re sum_j <psi|Z_j|psi> (observables of §3, each Z_j commuted through the
// final Clifford into a Weyl string and evaluated on the MPS by transfer matrices).
// Parametrised gates are diag(e^{i phi}) with phi = (0, theta[(d-1)b], ..., theta[(d-1)b+d-2])
// for parameter block b; each enters the MPS only through its MPO coefficients
// K_b = c_b tau^{ph_b}, c_b = (1/d) sum_j e^{i phi_j} omega^{-bj} (§2.3.1, §2.4).
//
// The derivative is taken with the method's discrete decisions frozen at the recording point
// (disentangler choices and the kept rank of every factorisation): the forward pass is then
// a smooth map of theta made of MPO site maps, two-qudit unitaries, matrix products and
// truncated factorisations with renormalisation.  Its reverse sweep:
//   * recording: one ordinary forward pass stores the Weyl string of every gate, the choices
//     and ranks, and the strings of the observables;
//   * replay: the same steps with the decisions forced, checkpointing the MPS before every gate;
//   * reverse: the final MPS gets dL/dA* from the transfer-matrix environments, then gate by
//     gate (last first) the gate is replayed from its checkpoint with a tape of its steps
//     (factorisations with their eigenbasis, the tensors consumed by products), and the tape
//     is run backwards.
// Adjoint of a split M = L R (FactRec orientation W, eigenbasis U, B = U^H W, sorted values
// s, kept set K, discarded set D):
//   gauge      : Nbar = (1 - L L^H) Lbar (R R^H)^{-1} R + L Rbar          (L orthonormal)
//                Nbar = Lbar R + L (L^H L)^{-1} Rbar (1 - R^H R)          (R orthonormal)
//   renormalise: Xbar = rn (Nbar - N Re<N, Nbar>)
//   truncation : Ybar = U^H Xbar_W, G1 = Ybar B^H (sorted rows),
//                Z = Ybar_K (rows of K) + Mix B with Mix[a][b] = (G1[a][b] + conj G1[b][a]) /
//                (s_kept^2 - s_discarded^2) for one index in K and one in D, Wbar = U Z.
// The kept-kept rotations of the split are a gauge and drop out; the kept/discarded terms
// carry the gap 1/(s_K^2 - s_D^2).
#include <chrono>
#include <memory>

#include "ctx.h"

using namespace gc;

struct gcamps_grad {
  gcamps_config cfg{};
  gcamps_ctx* ctx = nullptr;
  Arena arena;
  size_t persist_mark = 0;
  std::vector<GateRec> gates;              // one per non-Clifford gate
  std::vector<int> gparam;                 // parameter block (-1: fixed angles)
  std::vector<std::vector<double>> gphi;   // fixed angles
  std::vector<int32_t> ranks, choices;
  std::vector<size_t> rank_start, choice_start;
  std::vector<GateRec> obs;                // C^dagger Z_j C, j < n
  int nblocks = 0;
  bool disent = false;
  std::vector<z64*> abar;                  // adjoint of every site tensor
  z64* spare[3] = {nullptr, nullptr, nullptr};
  z64* T[12] = {};
  double* dscal = nullptr;                 // device scalars: [0] rn, [1] dot
  z64* kbar = nullptr;                     // d coefficient adjoints
  z64* dev_one = nullptr;
  double stats[8] = {0};

  ~gcamps_grad() {
    if (ctx) gcamps_destroy(ctx);
  }

  hipStream_t s() const { return ctx->stream; }

  std::vector<double> phi_of(int g, const double* theta) const {
    const int d = cfg.d;
    if (gparam[g] < 0) return gphi[g];
    std::vector<double> phi(d, 0.0);
    for (int j = 1; j < d; ++j) phi[j] = theta[(size_t)(d - 1) * gparam[g] + j - 1];
    return phi;
  }

  void start_replay() {
    ctx->reset_mps();
    ctx->choice_log.clear();
    ctx->gates = 0;
    ctx->rank_frz = &ranks;
    ctx->choice_frz = &choices;
  }
  void end_replay() {
    ctx->rank_frz = nullptr;
    ctx->choice_frz = nullptr;
    ctx->tape = nullptr;
  }

  void replay_gate(int g, const double* theta) {
    ctx->rank_pos = rank_start[g];
    ctx->choice_pos = choice_start[g];
    const std::vector<double> phi = phi_of(g, theta);
    ctx->phase_apply(gates[g], phi.data());
    if (disent) ctx->disentangle(nullptr, nullptr);
  }

  // ------------------------------------------------------------ observables and dL/dA*
  // loss = sum_j Re(tau^p <MPS|O_j|MPS>); with adj, abar[i] = dL/dA_i^* (overwritten).
  double observe(bool adj) {
    gcamps_ctx& c = *ctx;
    const int n = c.n, d = c.d;
    const size_t mark = arena.used;
    std::vector<z64*> E(n + 1), F(n + 1);
    for (int i = 0; i <= n; ++i) {
      E[i] = arena.take<z64>((size_t)c.chi[i] * c.chi[i]);
      F[i] = arena.take<z64>((size_t)c.chi[i] * c.chi[i]);
    }
    z64* res = arena.take<z64>(obs.size());
    if (adj)
      for (int i = 0; i < n; ++i)
        GC_HIP(hipMemsetAsync(abar[i], 0, (size_t)c.chi[i] * d * c.chi[i + 1] * sizeof(z64), s()));
    const z64 one = {1.0, 0.0};
    std::vector<int> shift(n);
    std::vector<z64> w((size_t)n * d);
    for (size_t j = 0; j < obs.size(); ++j) {
      const GateRec& P = obs[j];
      for (int herm = 0; herm < (adj ? 2 : 1); ++herm) {
        // site operator |t> -> w[t] |t + shift>; W^H uses the inverse shift and conjugate weights
        for (int i = 0; i < n; ++i) {
          const int x = P.x[i], z = P.z[i];
          shift[i] = herm ? (d - x) % d : x;
          for (int t = 0; t < d; ++t) {
            const int src = herm ? (t - x + d) % d : t;
            const double ang = 2.0 * M_PI * ((z * src) % d) / d;
            w[(size_t)i * d + t] = z64{std::cos(ang), herm ? -std::sin(ang) : std::sin(ang)};
          }
        }
        launch_copy(s(), E[0], dev_one, 1);
        for (int i = 0; i < n; ++i) {
          const int cl = c.chi[i], cr = c.chi[i + 1];
          for (int t = 0; t < d; ++t) {
            const z64* At = c.site[i] + (size_t)t * cr;
            const z64* As = c.site[i] + (size_t)((t + shift[i]) % d) * cr;
            launch_zgemm(s(), 0, 0, cl, cr, cl, E[i], cl, At, d * cr, T[0], cr, one, 0, 0);
            launch_zgemm(s(), 1, 0, cr, cr, cl, As, d * cr, T[0], cr, E[i + 1], cr, w[(size_t)i * d + t], t > 0, 0);
          }
        }
        if (!herm) launch_copy(s(), res + j, E[n], 1);
        if (!adj) continue;
        launch_copy(s(), F[n], dev_one, 1);
        for (int i = n - 1; i >= 0; --i) {
          const int cl = c.chi[i], cr = c.chi[i + 1];
          for (int t = 0; t < d; ++t) {
            const z64* At = c.site[i] + (size_t)t * cr;
            const z64* As = c.site[i] + (size_t)((t + shift[i]) % d) * cr;
            launch_zgemm(s(), 0, 0, cl, cr, cr, At, d * cr, F[i + 1], cr, T[0], cr, one, 0, 0);
            launch_zgemm(s(), 0, 1, cl, cl, cr, T[0], cr, As, d * cr, F[i], cl, w[(size_t)i * d + t], t > 0, 0);
          }
        }
        const std::complex<double> ph = std::polar(0.5, (herm ? -1.0 : 1.0) * M_PI * P.p / d);
        for (int i = 0; i < n; ++i) {
          const int cl = c.chi[i], cr = c.chi[i + 1];
          for (int t = 0; t < d; ++t) {
            const z64* At = c.site[i] + (size_t)t * cr;
            const int so = (t + shift[i]) % d;
            const std::complex<double> cf = ph * std::complex<double>(w[(size_t)i * d + t].re, w[(size_t)i * d + t].im);
            launch_zgemm(s(), 0, 0, cl, cr, cl, E[i], cl, At, d * cr, T[0], cr, one, 0, 0);
            launch_zgemm(s(), 0, 0, cl, cr, cr, T[0], cr, F[i + 1], cr, abar[i] + (size_t)so * cr, d * cr,
                         z64{cf.real(), cf.imag()}, 1, 0);
          }
        }
      }
    }
    std::vector<z64> h(obs.size());
    GC_HIP(hipMemcpyAsync(h.data(), res, obs.size() * sizeof(z64), hipMemcpyDeviceToHost, s()));
    GC_HIP(hipStreamSynchronize(s()));
    double loss = 0.0;
    for (size_t j = 0; j < obs.size(); ++j)
      loss += (std::complex<double>(h[j].re, h[j].im) * std::polar(1.0, M_PI * obs[j].p / d)).real();
    arena.used = mark;
    return loss;
  }

  // ------------------------------------------------------------ split adjoint
  // L (p x k), R (k x q) of the recorded split into T[0], T[1].
  void emit_factors(const FactRec& f) {
    launch_emit(s(), f.wide, f.left, f.renorm, f.p, f.q, f.k, f.U, f.m, f.B, f.kW, f.perm, f.sig, T[0], T[1]);
  }

  // Mbar (p x q) from Lbar (p x k), Rbar (k x q); L, R in T[0], T[1].  Uses T[2..11].
  void fact_bwd(const FactRec& f, const z64* Lbar, const z64* Rbar, z64* Mbar) {
    const int p = f.p, q = f.q, k = f.k, m = f.m, kW = f.kW;
    const z64 one = {1.0, 0.0}, mone = {-1.0, 0.0};
    const z64* L = T[0];
    const z64* R = T[1];
    launch_kept_norm(s(), f.sig, k, f.renorm, dscal);
    z64* Nbar = T[4];
    if (f.left) {
      launch_zgemm(s(), 1, 0, k, k, p, L, k, Lbar, k, T[2], k, one, 0, 0);        // L^H Lbar
      launch_copy(s(), T[3], Lbar, (size_t)p * k);
      launch_zgemm(s(), 0, 0, p, k, k, L, k, T[2], k, T[3], k, mone, 1, 0);       // (1 - L L^H) Lbar
      launch_inv_gram_scale(s(), T[3], p, k, 1, f.sig, dscal);                     // (R R^H)^{-1}
      launch_zgemm(s(), 0, 0, p, q, k, T[3], k, R, q, Nbar, q, one, 0, 0);
      launch_zgemm(s(), 0, 0, p, q, k, L, k, Rbar, q, Nbar, q, one, 1, 0);
    } else {
      launch_zgemm(s(), 0, 1, k, k, q, Rbar, q, R, q, T[2], k, one, 0, 0);        // Rbar R^H
      launch_copy(s(), T[3], Rbar, (size_t)k * q);
      launch_zgemm(s(), 0, 0, k, q, k, T[2], k, R, q, T[3], q, mone, 1, 0);       // Rbar (1 - R^H R)
      launch_inv_gram_scale(s(), T[3], k, q, 0, f.sig, dscal);                     // (L^H L)^{-1}
      launch_zgemm(s(), 0, 0, p, q, k, Lbar, k, R, q, Nbar, q, one, 0, 0);
      launch_zgemm(s(), 0, 0, p, q, k, L, k, T[3], q, Nbar, q, one, 1, 0);
    }
    z64* Xbar = Nbar;
    if (f.renorm) {
      launch_zgemm(s(), 0, 0, p, q, k, L, k, R, q, T[5], q, one, 0, 0);           // N = L R
      launch_dot_re(s(), T[5], Nbar, (size_t)p * q, dscal + 1);
      launch_renorm_bwd(s(), Nbar, T[5], (size_t)p * q, dscal, dscal + 1, T[6]);
      Xbar = T[6];
    }
    // Ybar = U^H Xbar_W (m x kW)
    if (f.wide)
      launch_zgemm(s(), 1, 0, m, kW, m, f.U, m, Xbar, kW, T[7], kW, one, 0, 0);
    else
      launch_zgemm(s(), 1, 1, m, kW, m, f.U, m, Xbar, m, T[7], kW, one, 0, 0);
    launch_gather_rows(s(), T[7], f.perm, m, kW, m, T[8]);                         // Ybar sorted
    launch_gather_rows(s(), f.B, f.perm, m, kW, m, T[9]);                          // B sorted
    launch_zgemm(s(), 0, 1, m, m, kW, T[8], kW, T[9], kW, T[10], m, one, 0, 0);    // G1
    launch_trunc_mix(s(), T[10], m, k, f.sig, T[11]);
    launch_gather_rows(s(), T[7], f.perm, m, kW, k, T[4]);                         // Ybar_K
    launch_zgemm(s(), 0, 0, m, kW, m, T[11], m, T[9], kW, T[4], kW, one, 1, 0);    // + Mix B
    launch_gather_cols(s(), f.U, f.perm, m, T[10]);                                // U sorted
    if (f.wide)
      launch_zgemm(s(), 0, 0, m, kW, m, T[10], m, T[4], kW, Mbar, kW, one, 0, 0);
    else
      launch_zgemm(s(), 1, 1, kW, m, m, T[4], kW, T[10], m, Mbar, m, one, 0, 0);
  }

  // ------------------------------------------------------------ one tape step backwards
  void step_back(const TapeOp& op, int g, const double* theta, double* grad) {
    gcamps_ctx& c = *ctx;
    const int d = c.d;
    const z64 one = {1.0, 0.0};
    const int i = op.site;
    switch (op.kind) {
      case TAPE_ABSORB_R: {
        const FactRec& f = op.f;
        const int k = f.k, q = f.q, cols = op.d0[1];
        emit_factors(f);
        z64* Rb = spare[2];
        launch_zgemm(s(), 0, 1, k, q, cols, abar[i + 1], cols, op.x0, cols, Rb, q, one, 0, 0);
        launch_zgemm(s(), 1, 0, q, cols, k, T[1], q, abar[i + 1], cols, spare[0], cols, one, 0, 0);
        fact_bwd(f, abar[i], Rb, spare[1]);
        std::swap(abar[i + 1], spare[0]);
        std::swap(abar[i], spare[1]);
        break;
      }
      case TAPE_ABSORB_L: {
        const FactRec& f = op.f;
        const int k = f.k, p = f.p, rows = op.d0[0];
        emit_factors(f);
        z64* Lb = spare[2];
        launch_zgemm(s(), 1, 0, p, k, rows, op.x0, p, abar[i - 1], k, Lb, k, one, 0, 0);
        launch_zgemm(s(), 0, 1, rows, p, k, abar[i - 1], k, T[0], k, spare[0], p, one, 0, 0);
        fact_bwd(f, Lb, abar[i], spare[1]);
        std::swap(abar[i - 1], spare[0]);
        std::swap(abar[i], spare[1]);
        break;
      }
      case TAPE_THETA: {
        const FactRec& f = op.f;
        emit_factors(f);
        z64* thb = spare[2];
        fact_bwd(f, abar[i], abar[i + 1], thb);
        if (op.cstar != 0) launch_apply_qh(s(), d, op.chil, op.chir, op.cstar, c.q64, thb);
        const int r0 = op.d0[0], cm = op.d0[1], c1 = op.d1[1];
        launch_zgemm(s(), 0, 1, r0, cm, c1, thb, c1, op.x1, c1, spare[0], cm, one, 0, 0);
        launch_zgemm(s(), 1, 0, cm, c1, r0, op.x0, cm, thb, c1, spare[1], c1, one, 0, 0);
        std::swap(abar[i], spare[0]);
        std::swap(abar[i + 1], spare[1]);
        break;
      }
      case TAPE_MPO: {
        const std::vector<double> phi = phi_of(g, theta);
        const MpoCoeff co = c.mpo_coeff(gates[g], phi.data());
        if ((op.mpo_kind == 0 || op.mpo_kind == 3) && gparam[g] >= 0) {
          launch_mpo_coeff_bwd(s(), op.mpo_kind, d, op.chil, op.chir, op.dx, op.dz, co, op.x0, abar[i], kbar);
          std::vector<z64> kb(d);
          GC_HIP(hipMemcpyAsync(kb.data(), kbar, d * sizeof(z64), hipMemcpyDeviceToHost, s()));
          GC_HIP(hipStreamSynchronize(s()));
          // dL/dphi_j = 2 Re sum_b conj(Kbar_b) dK_b/dphi_j,
          // dK_b/dphi_j = tau^{ph_b} (i/d) e^{i phi_j} omega^{-bj}
          const GateRec& P = gates[g];
          for (int j = 1; j < d; ++j) {
            std::complex<double> acc = 0.0;
            for (int b = 0; b < d; ++b) {
              const int ph = (b * P.p + 2 * P.sd * (b * (b - 1) / 2)) % (2 * d);
              const std::complex<double> dk = std::polar(1.0, M_PI * ph / d) * std::complex<double>(0.0, 1.0 / d) *
                                              std::polar(1.0, phi[j] - 2.0 * M_PI * b * j / d);
              acc += std::conj(std::complex<double>(kb[b].re, kb[b].im)) * dk;
            }
            grad[(size_t)(d - 1) * gparam[g] + j - 1] += 2.0 * acc.real();
          }
        }
        launch_mpo_site_bwd(s(), op.mpo_kind, d, op.chil, op.chir, op.dx, op.dz, co, abar[i], spare[0]);
        std::swap(abar[i], spare[0]);
        break;
      }
      default:
        throw Error{GCAMPS_EINVAL, "unknown tape step"};
    }
  }

  // ------------------------------------------------------------ drivers
  double loss_at(const double* theta) {
    start_replay();
    for (size_t g = 0; g < gates.size(); ++g) replay_gate((int)g, theta);
    end_replay();
    return observe(false);
  }

  double gradient_at(const double* theta, double* grad) {
    gcamps_ctx& c = *ctx;
    const int n = c.n, d = c.d;
    const size_t G = gates.size();
    for (int b = 0; b < nblocks * (d - 1); ++b) grad[b] = 0.0;
    auto t0 = std::chrono::steady_clock::now();
    const size_t mark = arena.used;
    struct Ckpt {
      z64* data;
      std::vector<int> chi;
      int centre;
    };
    std::vector<Ckpt> ck(G);
    start_replay();
    for (size_t g = 0; g < G; ++g) {
      Ckpt& k = ck[g];
      k.chi = c.chi;
      k.centre = c.centre;
      k.data = arena.take<z64>(c.mps_elems());
      size_t off = 0;
      for (int i = 0; i < n; ++i) {
        const size_t e = (size_t)c.chi[i] * d * c.chi[i + 1];
        launch_copy(s(), k.data + off, c.site[i], e);
        off += e;
      }
      replay_gate((int)g, theta);
    }
    end_replay();
    const double loss = observe(true);
    auto t1 = std::chrono::steady_clock::now();
    std::vector<TapeOp> tape;
    size_t tape_ops = 0;
    for (size_t gg = G; gg-- > 0;) {
      Ckpt& k = ck[gg];
      c.chi = k.chi;
      c.centre = k.centre;
      size_t off = 0;
      for (int i = 0; i < n; ++i) {
        const size_t e = (size_t)c.chi[i] * d * c.chi[i + 1];
        launch_copy(s(), c.site[i], k.data + off, e);
        off += e;
      }
      const size_t gmark = arena.used;
      tape.clear();
      c.rank_frz = &ranks;
      c.choice_frz = &choices;
      c.tape = &tape;
      c.arena = &arena;
      replay_gate((int)gg, theta);
      end_replay();
      tape_ops += tape.size();
      for (size_t t = tape.size(); t-- > 0;) step_back(tape[t], (int)gg, theta, grad);
      arena.used = gmark;
    }
    GC_HIP(hipStreamSynchronize(s()));
    arena.used = mark;
    auto t2 = std::chrono::steady_clock::now();
    stats[0] = std::chrono::duration<double, std::milli>(t1 - t0).count();
    stats[1] = std::chrono::duration<double, std::milli>(t2 - t1).count();
    stats[2] = (double)arena.peak;
    stats[3] = (double)tape_ops;
    return loss;
  }
};

namespace {

template <typename Fn>
int32_t grad_guard(Fn&& f) {
  try {
    f();
    return GCAMPS_OK;
  } catch (const Error& e) {
    set_error(e.msg);
    return e.code;
  } catch (const std::exception& e) {
    set_error(e.what());
    return GCAMPS_EINVAL;
  }
}

}  // namespace

extern "C" {

int32_t gcamps_grad_record(const gcamps_config* cfg, const gcamps_op* ops, int64_t n_ops, const int32_t* op_param,
                           const double* theta, int32_t n_theta, const gcamps_candset* set, void* dev_workspace,
                           size_t bytes, void* hip_stream, gcamps_grad** out, double* loss) {
  return grad_guard([&] {
    GC_CHECK(cfg && out && dev_workspace && (n_ops == 0 || ops), GCAMPS_EINVAL, "null argument");
    GC_CHECK(n_theta >= 0 && (n_theta == 0 || theta), GCAMPS_EINVAL, "null theta");
    size_t ctx_bytes = 0;
    int32_t rc = gcamps_workspace_bytes(cfg, &ctx_bytes);
    if (rc != GCAMPS_OK) throw Error{rc, gcamps_last_error()};
    ctx_bytes = (ctx_bytes + 255) & ~size_t(255);
    GC_CHECK(bytes > ctx_bytes, GCAMPS_EWORKSPACE, "workspace smaller than the state plus a gradient arena");
    const int d = cfg->d;
    GC_CHECK(n_theta % (d - 1) == 0, GCAMPS_EINVAL, "n_theta must be a multiple of d - 1");
    auto g = std::make_unique<gcamps_grad>();
    g->cfg = *cfg;
    g->nblocks = n_theta / (d - 1);
    // validate ops and parameter indices before any device work
    for (int64_t k = 0; k < n_ops; ++k) {
      const gcamps_op& op = ops[k];
      GC_CHECK(op.kind == GCAMPS_OP_CLIFFORD_LAYER || op.kind == GCAMPS_OP_PHASE, GCAMPS_EINVAL, "unknown op kind");
      if (op.kind == GCAMPS_OP_PHASE) {
        const int pb = op_param ? op_param[k] : -1;
        GC_CHECK(pb < g->nblocks, GCAMPS_EINVAL, "parameter block out of range");
        GC_CHECK(op.sites && (pb >= 0 || op.phi), GCAMPS_EINVAL, "phase op without site or angles");
      }
    }
    rc = gcamps_init(cfg, dev_workspace, ctx_bytes, hip_stream, &g->ctx);
    if (rc != GCAMPS_OK) throw Error{rc, gcamps_last_error()};
    gcamps_ctx& c = *g->ctx;
    if (set) {
      rc = gcamps_set_candset(g->ctx, set);
      if (rc != GCAMPS_OK) throw Error{rc, gcamps_last_error()};
    }
    g->disent = cfg->auto_disentangle && c.ncand > 0;
    g->arena.base = reinterpret_cast<char*>(dev_workspace) + ctx_bytes;
    g->arena.cap = bytes - ctx_bytes;
    // persistent buffers of the reverse sweep
    const size_t slot = std::max(c.lay.slot_elems, c.lay.mcap * c.lay.mcap);
    for (int i = 0; i < c.n; ++i) g->abar.push_back(g->arena.take<z64>(slot));
    for (auto& sp : g->spare) sp = g->arena.take<z64>(slot);
    for (auto& t : g->T) t = g->arena.take<z64>(slot);
    g->dscal = g->arena.take<double>(8);
    g->kbar = g->arena.take<z64>(kMaxD);
    g->dev_one = g->arena.take<z64>(1);
    const z64 one_h = {1.0, 0.0};
    GC_HIP(hipMemcpyAsync(g->dev_one, &one_h, sizeof(z64), hipMemcpyHostToDevice, c.stream));
    g->persist_mark = g->arena.used;
    // recording pass: the ordinary forward pass with decisions and strings recorded
    auto t0 = std::chrono::steady_clock::now();
    c.rank_rec = &g->ranks;
    c.gate_rec = &g->gates;
    for (int64_t k = 0; k < n_ops; ++k) {
      const gcamps_op& op = ops[k];
      if (op.kind == GCAMPS_OP_CLIFFORD_LAYER) {
        rc = gcamps_apply_clifford_layer(g->ctx, op.sites, op.words, op.count);
        if (rc != GCAMPS_OK) throw Error{rc, gcamps_last_error()};
        continue;
      }
      const int pb = op_param ? op_param[k] : -1;
      GC_CHECK(op.sites[0] >= 0 && op.sites[0] < c.n, GCAMPS_EINVAL, "site out of range");
      std::vector<double> phi(d, 0.0);
      if (pb >= 0) {
        for (int j = 1; j < d; ++j) phi[j] = theta[(size_t)(d - 1) * pb + j - 1];
      } else {
        for (int j = 0; j < d; ++j) phi[j] = op.phi[j];
      }
      g->gparam.push_back(pb);
      g->gphi.push_back(phi);
      g->rank_start.push_back(g->ranks.size());
      g->choice_start.push_back(c.choice_log.size() / 4);
      c.phase_rotation(op.sites[0], phi.data());
      if (g->disent) c.disentangle(nullptr, nullptr);
    }
    c.rank_rec = nullptr;
    c.gate_rec = nullptr;
    for (size_t e = 3; e < c.choice_log.size(); e += 4) g->choices.push_back(c.choice_log[e]);
    for (int j = 0; j < c.n; ++j) {
      std::vector<int> xzp(2 * c.n + 1, 0);
      xzp[c.n + j] = 1;
      g->obs.push_back(c.extract_string(xzp.data()));
    }
    const double L = g->observe(false);
    g->stats[5] = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (loss) *loss = L;
    *out = g.release();
  });
}

int32_t gcamps_grad_loss(gcamps_grad* g, const double* theta, double* loss) {
  return grad_guard([&] {
    GC_CHECK(g && loss && (g->nblocks == 0 || theta), GCAMPS_EINVAL, "null argument");
    *loss = g->loss_at(theta);
  });
}

int32_t gcamps_grad_gradient(gcamps_grad* g, const double* theta, double* loss, double* grad) {
  return grad_guard([&] {
    GC_CHECK(g && grad && (g->nblocks == 0 || theta), GCAMPS_EINVAL, "null argument");
    const double L = g->gradient_at(theta, grad);
    if (loss) *loss = L;
  });
}

int32_t gcamps_grad_stats(gcamps_grad* g, double out[8]) {
  return grad_guard([&] {
    GC_CHECK(g && out, GCAMPS_EINVAL, "null argument");
    for (int i = 0; i < 8; ++i) out[i] = g->stats[i];
    out[4] = (double)g->gates.size();
    out[6] = (double)g->ranks.size();
    out[7] = (double)g->choices.size();
  });
}

int32_t gcamps_grad_destroy(gcamps_grad* g) {
  delete g;
  return GCAMPS_OK;
}

}  // extern "C"
