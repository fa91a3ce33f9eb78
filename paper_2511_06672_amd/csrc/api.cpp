// Host runtime and C ABI of libgcamps: context, workspace carving, the GCAMPS bottom loop
// (commute, MPO, compression, disentangling sweeps) and the getters.
//
// Every numerical step runs in the library's HIP kernels on the ctx stream; the host keeps
// the bond dimensions (read back once per factorisation to size the next launches), the
// fidelity estimate and the choice log.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstring>
#include <atomic>
#include <memory>
#include <mutex>

#include "ctx.h"

using namespace gc;

namespace gc {
}

namespace {

thread_local std::string g_last_error;
std::atomic<uint64_t> g_uid{1};

bool is_prime(int d) {
  if (d < 2) return false;
  for (int k = 2; k * k <= d; ++k)
    if (d % k == 0) return false;
  return true;
}



void validate_config(const gcamps_config* c) {
  GC_CHECK(c != nullptr, GCAMPS_EINVAL, "config is null");
  GC_CHECK(c->d >= 2 && c->d <= kMaxD, GCAMPS_EINVAL, "d out of range [2, 7]");
  GC_CHECK(is_prime(c->d), GCAMPS_EUNSUPPORTED, "d must be prime (decomposition over the field Z_d)");
  GC_CHECK(c->n >= 2 && c->n <= kMaxN, GCAMPS_EINVAL, "n out of range [2, 128]");
  GC_CHECK(c->criterion == GCAMPS_CRITERION_RENYI2 || c->criterion == GCAMPS_CRITERION_BOND_DIM, GCAMPS_EINVAL,
           "criterion must be GCAMPS_CRITERION_RENYI2 or _BOND_DIM");
  GC_CHECK(c->criterion != GCAMPS_CRITERION_BOND_DIM || c->score_prec == GCAMPS_SCORE_FP64, GCAMPS_EINVAL,
           "the bond-dimension criterion uses FP64 scores (score_prec = GCAMPS_SCORE_FP64)");
  GC_CHECK(c->max_gate_terms >= 0 && c->max_gate_terms <= kMaxGateTerms, GCAMPS_EINVAL,
           "max_gate_terms out of range [0, 81]");
  GC_CHECK(c->chi_max >= 1 && (size_t)c->chi_max * std::max(c->d, c->max_gate_terms) <= 4096, GCAMPS_EINVAL,
           "chi_max out of range (chi_max * max(d, max_gate_terms) must not exceed 4096)");
  GC_CHECK(c->cutoff >= 0.0 && c->cutoff < 1.0, GCAMPS_EINVAL, "cutoff out of range [0, 1)");
  GC_CHECK(c->score_prec == GCAMPS_SCORE_FP64 || c->score_prec == GCAMPS_SCORE_FP32 ||
               c->score_prec == GCAMPS_SCORE_BF16 || c->score_prec == GCAMPS_SCORE_REPLICA,
           GCAMPS_EINVAL, "score_prec must be GCAMPS_SCORE_FP64, _FP32, _BF16 or _REPLICA");
  GC_CHECK(c->score_prec != GCAMPS_SCORE_REPLICA || c->d <= 3, GCAMPS_EUNSUPPORTED,
           "replica scoring is implemented for d = 2 and 3");
  GC_CHECK(c->tie_tol >= 0.0, GCAMPS_EINVAL, "tie_tol must be >= 0");
  // The FP64 re-score decides only among candidates inside the window, so the window must be
  // wider than twice the low-precision scoring error (measured up to ~2e-5 in S2 for FP32 and
  // split BF16); replica scoring is FP64 arithmetic and needs only the FP64 floor.
  GC_CHECK(c->score_prec == GCAMPS_SCORE_FP64 || c->near_tie >= 1e-6, GCAMPS_EINVAL, "near_tie must be >= 1e-6");
  GC_CHECK((c->score_prec != GCAMPS_SCORE_FP32 && c->score_prec != GCAMPS_SCORE_BF16) || c->near_tie >= kNearTieLowp,
           GCAMPS_EINVAL, "near_tie must be >= 1e-4 with FP32 or split-BF16 scoring");
  GC_CHECK(c->max_sweeps >= 0, GCAMPS_EINVAL, "max_sweeps must be >= 0");
  GC_CHECK(c->max_candidates >= 1 && c->max_candidates <= 65536, GCAMPS_EINVAL, "max_candidates out of range");
}

template <typename F>
int32_t guarded(gcamps_ctx* ctx, F&& f);

}  // namespace


namespace {

template <typename F>
int32_t guarded(gcamps_ctx* ctx, F&& f) {
  try {
    if (ctx && ctx->poisoned) throw Error{GCAMPS_EDEVICE, "context poisoned by an earlier device/numeric error"};
    auto t0 = std::chrono::steady_clock::now();
    f();
    if (ctx)
      ctx->stats[7] += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return GCAMPS_OK;
  } catch (const Error& e) {
    g_last_error = e.msg;
    if (ctx && (e.code == GCAMPS_EDEVICE || e.code == GCAMPS_ENUMERIC)) ctx->poisoned = true;
    return e.code;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return GCAMPS_EINVAL;
  }
}

}  // namespace

namespace gc {
void set_error(const std::string& msg) { g_last_error = msg; }
}  // namespace gc

namespace gc {
Layout make_layout(const gcamps_config& c) {
  Layout L{};
  const size_t d = c.d, chi = c.chi_max;
  // bond capacity: an MPO of bond J = max(d, max_gate_terms) multiplies bonds by J before compression
  const size_t chicap = chi * std::max<size_t>(d, (size_t)c.max_gate_terms);
  L.slot_elems = chicap * d * chicap;
  L.theta_elems = chi * d * d * chi;
  L.mcap = chicap;
  L.m_pad = ((chicap + 63) / 64) * 64;
  L.ncand = std::max(1, c.max_candidates);
  size_t nt = (chicap + 63) / 64;
  L.ntp = nt * (nt + 1) / 2;  // 64-wide tiles (the FP32 path uses 128-wide, fewer)
  L.nslots = c.n + 3;  // n sites + L, R, one spare
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align256(o + bytes);
    return at;
  };
  L.off_slots = take((size_t)L.nslots * L.slot_elems * sizeof(z64));
  L.off_theta = take(std::max(L.theta_elems, L.slot_elems) * sizeof(z64));
  L.off_G = take(L.mcap * L.mcap * sizeof(z64));
  L.off_U = take(L.mcap * L.mcap * sizeof(z64));
  L.off_Z = take(L.mcap * L.mcap * sizeof(z64));
  L.off_Utmp = take(L.mcap * L.mcap * sizeof(z64));
  L.off_B = take(L.slot_elems * sizeof(z64));
  L.off_B2 = take(L.slot_elems * sizeof(z64));
  L.off_sig2 = take(L.mcap * sizeof(double));
  L.off_sig = take(L.mcap * sizeof(double));
  L.off_lam = take(L.mcap * sizeof(double));
  L.off_perm = take(L.mcap * sizeof(int));
  L.off_eigG = take(3 * L.m_pad * L.m_pad * sizeof(z64));  // two matrix buffers and the accumulator
  L.off_eigV = take((L.m_pad / 64 + 1) * 64 * 64 * sizeof(z64));
  L.off_flags = take(4096);
  L.off_s2 = take(L.ncand * sizeof(double));
  L.off_s2w = take(L.ncand * sizeof(double));
  L.off_wlist = take(L.ncand * sizeof(int));
  L.off_partial = take(L.ncand * L.ntp * 2 * sizeof(double));
  // rotated candidate matrices of the tiled scorer: up to 64 candidates of m x k complex128
  L.nbuf_bytes = (size_t)std::min<size_t>(64, L.ncand) * L.theta_elems * sizeof(z64);
  // replica scoring keeps its scratch (Gram of Theta, partial sums) in the same buffer: the
  // first pass is done before the window re-score writes rotated matrices there
  const bool replica = c.score_prec == GCAMPS_SCORE_REPLICA;
  if (replica) L.nbuf_bytes = std::max(L.nbuf_bytes, replica_scratch_bytes(c.d, c.chi_max));
  L.off_nbuf = take(L.nbuf_bytes);
  L.off_rtab = take(replica ? replica_table_elems(c.d, (int)L.ncand) * sizeof(z64) : 0);
  const size_t D4 = d * d * d * d;
  L.off_q64 = take(L.ncand * D4 * sizeof(z64));
  L.off_q32 = take(L.ncand * D4 * sizeof(c32));
  L.off_qinv = take(L.ncand * D4 * sizeof(uint32_t));
  L.off_tab = take((2 * (size_t)c.n * c.n * 2 + 2 * c.n) * sizeof(int));
  L.off_target = take((2 * (size_t)c.n + 1) * sizeof(int));
  L.off_weyl = take(sizeof(DevWeyl));
  L.off_err = take(sizeof(int) * 4);
  L.off_status = take(sizeof(DevStatus));
  L.off_luts = take((size_t)c.n * D4 * sizeof(uint32_t));
  L.off_sites = take((size_t)c.n * sizeof(int));
  // dense state (validation; d^n <= kDenseMax): amplitude output and scratch (4 d^n complex128)
  // plus the per-index Clifford table (two int32 and n int8 per index)
  L.dense_dim = 1;
  for (int i = 0; i < c.n && L.dense_dim <= kDenseMax; ++i) L.dense_dim *= d;
  if (L.dense_dim > kDenseMax) L.dense_dim = 0;
  L.off_dense = take(L.dense_dim * (4 * sizeof(z64) + 2 * sizeof(int) + (size_t)c.n));
  L.off_pcst = take(sizeof(PcState));
  L.total = o;
  return L;
}
}  // namespace gc

// Scratch of gcamps_statevector_static: the three dense work vectors of the largest dense state
// (3 * 2^16 complex128, 3 MiB), one copy per GPU for the life of the process.  Host code never
// passes the array's name to a kernel: it stands for the host-side shadow, not the device copy.
// The device address of each GPU's copy is looked up once, with that GPU current, and kept.
static __device__ __align__(256) z64 scratch[3 * kDenseMax];
constexpr int kMaxDevices = 64;
static void* g_scratch_dev[kMaxDevices] = {nullptr};
static std::mutex g_scratch_mu;

// Device address of `scratch` on the current GPU (looked up at gcamps_init, once per device).
static void* scratch_address(int dev) {
  GC_CHECK(dev >= 0 && dev < kMaxDevices, GCAMPS_EDEVICE, "device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* ptr = nullptr;
    GC_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    GC_CHECK(ptr != nullptr, GCAMPS_EDEVICE, "no device address for the static scratch");
    g_scratch_dev[dev] = ptr;
  }
  return g_scratch_dev[dev];
}

// ------------------------------------------------------------------------------- C ABI
extern "C" {

const char* gcamps_last_error(void) { return g_last_error.c_str(); }

int32_t gcamps_workspace_bytes(const gcamps_config* cfg, size_t* bytes) {
  return guarded(nullptr, [&] {
    validate_config(cfg);
    GC_CHECK(bytes != nullptr, GCAMPS_EINVAL, "bytes is null");
    *bytes = make_layout(*cfg).total;
  });
}

int32_t gcamps_init(const gcamps_config* cfg, void* dev_workspace, size_t bytes, void* hip_stream,
                    gcamps_ctx** out) {
  return guarded(nullptr, [&] {
    validate_config(cfg);
    GC_CHECK(out != nullptr && dev_workspace != nullptr, GCAMPS_EINVAL, "null argument");
    GC_CHECK(((uintptr_t)dev_workspace & 255) == 0, GCAMPS_EINVAL, "workspace must be 256-byte aligned");
    Layout lay = make_layout(*cfg);
    GC_CHECK(bytes >= lay.total, GCAMPS_EWORKSPACE, "workspace smaller than gcamps_workspace_bytes()");
    static std::once_flag attrs_once;
    std::call_once(attrs_once, [] {
      rank_set_attributes();
      linalg_set_attributes();
    });
    int dev = 0;
    GC_HIP(hipGetDevice(&dev));
    void* sdev = scratch_address(dev);  // static scratch of gcamps_statevector_static on this GPU
    auto c = std::make_unique<gcamps_ctx>();
    c->scratch_dev = sdev;
    c->cfg = *cfg;
    c->lay = lay;
    c->d = cfg->d;
    c->n = cfg->n;
    c->stream = reinterpret_cast<hipStream_t>(hip_stream);
    c->ws = reinterpret_cast<char*>(dev_workspace);
    char* w = c->ws;
    const int n = cfg->n;
    for (int i = 0; i < lay.nslots; ++i) {
      z64* p = reinterpret_cast<z64*>(w + lay.off_slots) + (size_t)i * lay.slot_elems;
      if (i < n)
        c->site.push_back(p);
      else if (i == n)
        c->Lbuf = p;
      else if (i == n + 1)
        c->Rbuf = p;
      else
        c->spare = p;
    }
    c->theta = reinterpret_cast<z64*>(w + lay.off_theta);
    c->G = reinterpret_cast<z64*>(w + lay.off_G);
    c->U = reinterpret_cast<z64*>(w + lay.off_U);
    c->Z = reinterpret_cast<z64*>(w + lay.off_Z);
    c->Utmp = reinterpret_cast<z64*>(w + lay.off_Utmp);
    c->B = reinterpret_cast<z64*>(w + lay.off_B);
    c->B2 = reinterpret_cast<z64*>(w + lay.off_B2);
    c->sig2 = reinterpret_cast<double*>(w + lay.off_sig2);
    c->sig = reinterpret_cast<double*>(w + lay.off_sig);
    c->lam = reinterpret_cast<double*>(w + lay.off_lam);
    c->perm = reinterpret_cast<int*>(w + lay.off_perm);
    c->eig.G = reinterpret_cast<z64*>(w + lay.off_eigG);
    c->eig.V = reinterpret_cast<z64*>(w + lay.off_eigV);
    c->eig.flags = reinterpret_cast<int*>(w + lay.off_flags);
    c->eig.m_pad = (int)lay.m_pad;
    c->s2 = reinterpret_cast<double*>(w + lay.off_s2);
    c->s2w = reinterpret_cast<double*>(w + lay.off_s2w);
    c->wlist = reinterpret_cast<int*>(w + lay.off_wlist);
    c->partial = reinterpret_cast<double*>(w + lay.off_partial);
    c->nbuf = w + lay.off_nbuf;
    c->q64 = reinterpret_cast<z64*>(w + lay.off_q64);
    c->rtab = cfg->score_prec == GCAMPS_SCORE_REPLICA ? reinterpret_cast<z64*>(w + lay.off_rtab) : nullptr;
    c->q32 = reinterpret_cast<c32*>(w + lay.off_q32);
    c->qinv = reinterpret_cast<uint32_t*>(w + lay.off_qinv);
    int* tab = reinterpret_cast<int*>(w + lay.off_tab);
    c->tx = tab;
    c->tz = tab + 2 * (size_t)n * n;
    c->tp = tab + 4 * (size_t)n * n;
    c->target = reinterpret_cast<int*>(w + lay.off_target);
    c->weyl = reinterpret_cast<DevWeyl*>(w + lay.off_weyl);
    c->derr = reinterpret_cast<int*>(w + lay.off_err);
    c->st = reinterpret_cast<DevStatus*>(w + lay.off_status);
    c->dluts = reinterpret_cast<uint32_t*>(w + lay.off_luts);
    c->dsites = reinterpret_cast<int*>(w + lay.off_sites);
    c->pcst = reinterpret_cast<PcState*>(w + lay.off_pcst);
    c->pinned_bytes = std::max<size_t>(1 << 20, (size_t)n * 2401 * 4 + 4096);
    GC_HIP(hipHostMalloc(reinterpret_cast<void**>(&c->pinned), c->pinned_bytes, hipHostMallocDefault));
    GC_HIP(hipHostMalloc(reinterpret_cast<void**>(&c->rb), kRbBytes, hipHostMallocDefault));
    c->eig.host_rb = reinterpret_cast<double*>(c->rb + kRbEig);
    GC_HIP(hipEventCreateWithFlags(&c->stage_ev, hipEventDisableTiming));
    GC_HIP(hipEventCreate(&c->ev0));
    GC_HIP(hipEventCreate(&c->ev1));
    GC_HIP(hipEventCreate(&c->ev2));
    GC_HIP(hipEventCreate(&c->ev3));
    for (hipEvent_t* e : {&c->evf0, &c->evf1, &c->evm0, &c->evm1}) GC_HIP(hipEventCreate(e));
    c->gram_ev.resize(64);
    for (auto& e : c->gram_ev) GC_HIP(hipEventCreate(&e));
    // |0...0>: every site tensor (1, d, 1) = e_0, tableau C = I
    c->chi.assign(n + 1, 1);
    c->centre = 0;
    GC_HIP(hipMemsetAsync(c->st, 0, sizeof(DevStatus), c->stream));
    for (int i = 0; i < n; ++i) {
      GC_HIP(hipMemsetAsync(c->site[i], 0, cfg->d * sizeof(z64), c->stream));
      z64 one = {1.0, 0.0};
      GC_HIP(hipMemcpyAsync(c->site[i], &one, sizeof(z64), hipMemcpyHostToDevice, c->stream));
    }
    launch_tableau_init(c->stream, n, c->tx, c->tz, c->tp);
    GC_HIP(hipStreamSynchronize(c->stream));
    *out = c.release();
  });
}

int32_t gcamps_destroy(gcamps_ctx* ctx) {
  if (!ctx) return GCAMPS_OK;
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  delete ctx;
  return GCAMPS_OK;
}

int32_t gcamps_apply_clifford_layer(gcamps_ctx* ctx, const int32_t* sites, const gcamps_word* words,
                                    int32_t count) {
  return guarded(ctx, [&] {
    GC_CHECK(ctx && sites && words && count >= 0, GCAMPS_EINVAL, "null argument");
    if (count == 0) return;
    const int d = ctx->d, n = ctx->n, D4 = d * d * d * d;
    GC_CHECK(count <= n, GCAMPS_EINVAL, "too many words in one layer");
    std::vector<char> used(n, 0);
    std::vector<CompiledWord> cw;
    for (int w = 0; w < count; ++w) {
      GC_CHECK(sites[w] >= 0 && sites[w] <= n - 2, GCAMPS_EINVAL, "site out of range");
      GC_CHECK(!used[sites[w]] && !used[sites[w] + 1], GCAMPS_EINVAL, "layer pairs overlap");
      used[sites[w]] = used[sites[w] + 1] = 1;
      cw.push_back(compile_word(d, words[w]));
    }
    char* stg = ctx->stage_begin();
    uint32_t* lut = reinterpret_cast<uint32_t*>(stg);
    for (int w = 0; w < count; ++w) std::memcpy(lut + (size_t)w * D4, cw[w].fwd.data(), D4 * sizeof(uint32_t));
    int* st_sites = reinterpret_cast<int*>(stg + (size_t)count * D4 * sizeof(uint32_t));
    for (int w = 0; w < count; ++w) st_sites[w] = sites[w];
    // one upload: luts then sites (device regions are separate; copy twice from staging)
    GC_HIP(hipMemcpyAsync(ctx->dluts, lut, (size_t)count * D4 * sizeof(uint32_t), hipMemcpyHostToDevice,
                          ctx->stream));
    GC_HIP(hipMemcpyAsync(ctx->dsites, st_sites, count * sizeof(int), hipMemcpyHostToDevice, ctx->stream));
    GC_HIP(hipEventRecord(ctx->stage_ev, ctx->stream));
    ctx->stage_pending = true;
    launch_tableau_layer(ctx->stream, n, d, count, ctx->dsites, ctx->dluts, ctx->tx, ctx->tz, ctx->tp);
  });
}

int32_t gcamps_apply_clifford(gcamps_ctx* ctx, int32_t site, const gcamps_word* word) {
  return gcamps_apply_clifford_layer(ctx, &site, word, 1);
}

int32_t gcamps_apply_phase_rotation(gcamps_ctx* ctx, int32_t site, const double* phi) {
  return guarded(ctx, [&] {
    GC_CHECK(ctx && phi, GCAMPS_EINVAL, "null argument");
    GC_CHECK(site >= 0 && site < ctx->n, GCAMPS_EINVAL, "site out of range");
    for (int j = 0; j < ctx->d; ++j) GC_CHECK(std::isfinite(phi[j]), GCAMPS_EINVAL, "phase angle not finite");
    ctx->phase_rotation(site, phi);
    if (ctx->cfg.auto_disentangle && ctx->ncand > 0) ctx->disentangle(nullptr, nullptr);
  });
}

int32_t gcamps_clifford_words(int32_t d, int32_t kind, int32_t* lens, int32_t lens_cap, uint8_t* gens,
                              int64_t gens_cap, int32_t* count, int64_t* total_gens) {
  return guarded(nullptr, [&] {
    GC_CHECK(count && total_gens, GCAMPS_EINVAL, "null argument");
    const auto words = clifford_word_set(d, kind);
    int64_t total = 0;
    for (const auto& w : words) total += (int64_t)w.size();
    *count = (int32_t)words.size();
    *total_gens = total;
    if (!lens) return;
    GC_CHECK(lens_cap >= (int32_t)words.size() && gens_cap >= total && (total == 0 || gens), GCAMPS_EINVAL,
             "output capacity below the word set");
    int64_t o = 0;
    for (size_t i = 0; i < words.size(); ++i) {
      lens[i] = (int32_t)words[i].size();
      for (uint8_t g : words[i]) gens[o++] = g;
    }
  });
}

int32_t gcamps_apply_gate(gcamps_ctx* ctx, int32_t site, int32_t nsites, const double* u) {
  return guarded(ctx, [&] {
    GC_CHECK(ctx && u, GCAMPS_EINVAL, "null argument");
    GC_CHECK(nsites == 1 || nsites == 2, GCAMPS_EINVAL, "nsites must be 1 or 2");
    GC_CHECK(site >= 0 && site + nsites <= ctx->n, GCAMPS_EINVAL, "gate sites out of range");
    int D = 1;
    for (int t = 0; t < nsites; ++t) D *= ctx->d;
    std::vector<z64> U((size_t)D * D);
    for (size_t i = 0; i < U.size(); ++i) {
      U[i] = z64{u[2 * i], u[2 * i + 1]};
      GC_CHECK(std::isfinite(U[i].re) && std::isfinite(U[i].im), GCAMPS_EINVAL, "gate entry not finite");
    }
    for (int i = 0; i < D; ++i)  // U^dagger U = I
      for (int j = 0; j < D; ++j) {
        double re = 0.0, im = 0.0;
        for (int r = 0; r < D; ++r) {
          const z64 a = U[(size_t)r * D + i], b = U[(size_t)r * D + j];
          re += a.re * b.re + a.im * b.im;
          im += a.re * b.im - a.im * b.re;
        }
        GC_CHECK(std::fabs(re - (i == j ? 1.0 : 0.0)) < 1e-10 && std::fabs(im) < 1e-10, GCAMPS_EINVAL,
                 "gate is not unitary");
      }
    ctx->general_gate(site, nsites, U);
    if (ctx->cfg.auto_disentangle && ctx->ncand > 0) ctx->disentangle(nullptr, nullptr);
  });
}

int32_t gcamps_candset_create(int32_t d, const gcamps_word* words, int32_t count, gcamps_candset** out) {
  return guarded(nullptr, [&] {
    GC_CHECK(out && words && count >= 1, GCAMPS_EINVAL, "null argument or empty set");
    GC_CHECK(d >= 2 && d <= kMaxD && is_prime(d), GCAMPS_EINVAL, "bad d");
    GC_CHECK(words[0].len == 0 && !words[0].weyl[0] && !words[0].weyl[1] && !words[0].weyl[2] && !words[0].weyl[3],
             GCAMPS_EINVAL, "candidate 0 must be the identity");
    auto s = std::make_unique<gcamps_candset>();
    s->d = d;
    s->count = count;
    for (int i = 0; i < count; ++i) s->words.push_back(compile_word(d, words[i]));
    s->uid = g_uid.fetch_add(1);
    *out = s.release();
  });
}

int32_t gcamps_candset_destroy(gcamps_candset* set) {
  delete set;
  return GCAMPS_OK;
}

static void upload_candset(gcamps_ctx* ctx, const gcamps_candset* set) {
  GC_CHECK(set->d == ctx->d, GCAMPS_EINVAL, "candidate set built for another d");
  GC_CHECK(set->count <= ctx->cfg.max_candidates, GCAMPS_ECAPACITY, "more candidates than max_candidates");
  if (ctx->cand_uid == set->uid) return;
  const int d = ctx->d, D4 = d * d * d * d;
  std::vector<z64> q64((size_t)set->count * D4);
  std::vector<c32> q32((size_t)set->count * D4);
  std::vector<uint32_t> inv((size_t)set->count * D4);
  for (int c = 0; c < set->count; ++c)
    for (int i = 0; i < D4; ++i) {
      q64[(size_t)c * D4 + i] = set->words[c].mat[i];
      q32[(size_t)c * D4 + i] = c32{(float)set->words[c].mat[i].re, (float)set->words[c].mat[i].im};
      inv[(size_t)c * D4 + i] = set->words[c].inv[i];
    }
  GC_HIP(hipMemcpyAsync(ctx->q64, q64.data(), q64.size() * sizeof(z64), hipMemcpyHostToDevice, ctx->stream));
  GC_HIP(hipMemcpyAsync(ctx->q32, q32.data(), q32.size() * sizeof(c32), hipMemcpyHostToDevice, ctx->stream));
  GC_HIP(hipMemcpyAsync(ctx->qinv, inv.data(), inv.size() * sizeof(uint32_t), hipMemcpyHostToDevice, ctx->stream));
  if (ctx->rtab) launch_replica_tables(ctx->stream, d, set->count, ctx->q64, ctx->rtab);
  GC_HIP(hipStreamSynchronize(ctx->stream));
  ctx->ncand = set->count;
  ctx->cand_uid = set->uid;
}

int32_t gcamps_set_candset(gcamps_ctx* ctx, const gcamps_candset* set) {
  return guarded(ctx, [&] {
    GC_CHECK(ctx && set, GCAMPS_EINVAL, "null argument");
    upload_candset(ctx, set);
  });
}

int32_t gcamps_score_bond(gcamps_ctx* ctx, int32_t bond, double* out, int64_t cap) {
  return guarded(ctx, [&] {
    GC_CHECK(ctx && out, GCAMPS_EINVAL, "null argument");
    GC_CHECK(bond >= 0 && bond < ctx->n - 1, GCAMPS_EINVAL, "bond outside [0, n-2]");
    GC_CHECK(ctx->ncand >= 1, GCAMPS_EINVAL, "no candidate set attached");
    GC_CHECK(cap >= ctx->ncand, GCAMPS_EINVAL, "output capacity below the candidate count");
    ctx->score_bond(bond, out);
  });
}

int32_t gcamps_factorize(gcamps_ctx* ctx, const double* m_host, int32_t p, int32_t q, int32_t flags,
                         double* sig_out, int32_t* kept, double* eps, double* l_out, double* r_out) {
  return guarded(ctx, [&] {
    GC_CHECK(ctx && m_host && sig_out && kept && eps, GCAMPS_EINVAL, "null argument");
    GC_CHECK((flags & ~GCAMPS_FACTORIZE_REDUCE) == 0, GCAMPS_EINVAL, "unknown factorize flag");
    GC_CHECK(p >= 1 && q >= 1, GCAMPS_EINVAL, "matrix must be at least 1 x 1");
    GC_CHECK(ctx->tape == nullptr && ctx->rank_rec == nullptr && ctx->rank_frz == nullptr, GCAMPS_EUNSUPPORTED,
             "factorize is not available on a gradient recording");
    const size_t m = (size_t)std::min(p, q), pq = (size_t)p * q;
    GC_CHECK(m <= ctx->lay.mcap && pq <= ctx->lay.slot_elems, GCAMPS_ECAPACITY,
             "matrix exceeds the ctx's factorisation capacity");
    GC_HIP(hipMemcpyAsync(ctx->theta, m_host, pq * sizeof(z64), hipMemcpyHostToDevice, ctx->stream));
    const DevStatus h =
        ctx->factorize(ctx->theta, p, q, 0, 1, ctx->Lbuf, ctx->Rbuf, (flags & GCAMPS_FACTORIZE_REDUCE) != 0);
    const size_t nb = (size_t)ctx->last_basis;  // values the factorisation resolved (m, or r when reduced)
    GC_HIP(hipMemcpyAsync(sig_out, ctx->sig, nb * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    for (size_t i = nb; i < m; ++i) sig_out[i] = 0.0;
    if (l_out)
      GC_HIP(hipMemcpyAsync(l_out, ctx->Lbuf, (size_t)p * h.kept * sizeof(z64), hipMemcpyDeviceToHost, ctx->stream));
    if (r_out)
      GC_HIP(hipMemcpyAsync(r_out, ctx->Rbuf, (size_t)h.kept * q * sizeof(z64), hipMemcpyDeviceToHost, ctx->stream));
    GC_HIP(hipStreamSynchronize(ctx->stream));
    *kept = h.kept;
    *eps = h.eps;
  });
}

int32_t gcamps_disentangle(gcamps_ctx* ctx, const gcamps_candset* set, int32_t* out_sweeps,
                           int32_t* out_changed_bonds) {
  return guarded(ctx, [&] {
    GC_CHECK(ctx, GCAMPS_EINVAL, "null argument");
    if (set) upload_candset(ctx, set);
    int sw = 0, ch = 0;
    ctx->disentangle(&sw, &ch);
    if (out_sweeps) *out_sweeps = sw;
    if (out_changed_bonds) *out_changed_bonds = ch;
  });
}

int32_t gcamps_expectation(gcamps_ctx* ctx, const int8_t* x, const int8_t* z, int32_t p, double out[2]) {
  return guarded(ctx, [&] {
    GC_CHECK(ctx && x && z && out, GCAMPS_EINVAL, "null argument");
    const int n = ctx->n, d = ctx->d;
    int* tg = reinterpret_cast<int*>(ctx->stage_begin());
    for (int i = 0; i < n; ++i) {
      GC_CHECK(x[i] >= 0 && x[i] < d && z[i] >= 0 && z[i] < d, GCAMPS_EINVAL, "exponent out of range");
      tg[i] = x[i];
      tg[n + i] = z[i];
    }
    tg[2 * n] = ((p % (2 * d)) + 2 * d) % (2 * d);
    ctx->stage_upload(ctx->target, (2 * n + 1) * sizeof(int));
    launch_weyl_extract(ctx->stream, n, d, ctx->tx, ctx->tz, ctx->tp, ctx->target, ctx->weyl, ctx->derr);
    DevWeyl P;
    GC_HIP(hipMemcpyAsync(&P, ctx->weyl, sizeof(DevWeyl), hipMemcpyDeviceToHost, ctx->stream));
    GC_HIP(hipStreamSynchronize(ctx->stream));
    // transfer matrices, E_0 = [[1]]; buffers: Utmp (E), Z (E'), G (tmp)
    z64* E = ctx->Utmp;
    z64* En = ctx->Z;
    z64* tmp = ctx->B2;
    z64 one = {1.0, 0.0};
    GC_HIP(hipMemcpyAsync(E, &one, sizeof(z64), hipMemcpyHostToDevice, ctx->stream));
    for (int i = 0; i < n; ++i) {
      const int cl = ctx->chi[i], cr = ctx->chi[i + 1];
      const z64* A = ctx->site[i];
      for (int t = 0; t < d; ++t) {
        launch_zgemm(ctx->stream, 0, 0, cl, cr, cl, E, cl, A + (size_t)t * cr, d * cr, tmp, cr, one, 0, 0);
        const int s = (t + P.x[i]) % d;
        const double ang = 2.0 * M_PI * ((P.z[i] * t) % d) / d;
        z64 w = {std::cos(ang), std::sin(ang)};
        launch_zgemm(ctx->stream, 1, 0, cr, cr, cl, A + (size_t)s * cr, d * cr, tmp, cr, En, cr, w, t > 0 ? 1 : 0, 0);
      }
      std::swap(E, En);
    }
    z64 e;
    GC_HIP(hipMemcpyAsync(&e, E, sizeof(z64), hipMemcpyDeviceToHost, ctx->stream));
    GC_HIP(hipStreamSynchronize(ctx->stream));
    std::complex<double> val = std::complex<double>(e.re, e.im) * std::polar(1.0, M_PI * P.p / d);
    out[0] = val.real();
    out[1] = val.imag();
  });
}

static long long dense_dim(gcamps_ctx* ctx) {
  GC_CHECK(ctx->lay.dense_dim > 0, GCAMPS_EUNSUPPORTED, "dense state limited to d^n <= 2^16");
  return (long long)ctx->lay.dense_dim;
}

// Dense psi = C|MPS> into out (D complex128); scratch holds 3 D complex128.  The per-index
// Clifford table lives in the ctx's dense region after its 4 D complex128, so nothing is
// allocated here.
static void statevector_impl(gcamps_ctx* ctx, z64* out, z64* scratch) {
  const int n = ctx->n, d = ctx->d;
  const long long D = dense_dim(ctx);
  hipStream_t s = ctx->stream;
  z64* mv = scratch;
  z64* va = scratch + D;
  z64* vb = scratch + 2 * D;
  // dense MPS vector: v (R x chi_i) * A_i (chi_i x d chi_{i+1})
  launch_copy(s, va, ctx->site[0], (size_t)d * ctx->chi[1]);
  long long R = d;
  for (int i = 1; i < n; ++i) {
    const int cl = ctx->chi[i], cr = ctx->chi[i + 1];
    GC_CHECK(R * d * cr <= D, GCAMPS_ECAPACITY, "bond dimensions exceed the dense bound");
    z64* dst = (i == n - 1) ? mv : vb;
    launch_zgemm(s, 0, 0, (int)R, d * cr, cl, va, cl, ctx->site[i], d * cr, dst, d * cr, z64{1.0, 0.0}, 0, 0);
    R *= d;
    if (i != n - 1) std::swap(va, vb);
  }
  // tableau rows to host
  std::vector<int> hx(2 * n * n), hz(2 * n * n), hp(2 * n);
  GC_HIP(hipMemcpyAsync(hx.data(), ctx->tx, hx.size() * sizeof(int), hipMemcpyDeviceToHost, s));
  GC_HIP(hipMemcpyAsync(hz.data(), ctx->tz, hz.size() * sizeof(int), hipMemcpyDeviceToHost, s));
  GC_HIP(hipMemcpyAsync(hp.data(), ctx->tp, hp.size() * sizeof(int), hipMemcpyDeviceToHost, s));
  GC_HIP(hipStreamSynchronize(s));
  // |s0> = C|0>: projector prod_k (1/d) sum_j S_k^j applied to a fixed generic vector
  std::vector<z64> start(D);
  for (long long y = 0; y < D; ++y) start[y] = z64{std::cos(0.731 * y + 0.2), std::sin(1.37 * y + 0.5) + 0.3};
  GC_HIP(hipMemcpy(va, start.data(), D * sizeof(z64), hipMemcpyHostToDevice));
  // all exponent rows of S_k^j (k < n, j < d) uploaded once: [k][j][x | z]
  std::vector<int> pows((size_t)n * d * 2 * n);
  std::vector<int> pph((size_t)n * d);
  for (int k = 0; k < n; ++k) {
    int xzsum = 0;
    for (int i = 0; i < n; ++i) xzsum += hx[k * n + i] * hz[k * n + i];
    for (int j = 0; j < d; ++j) {
      int* row = &pows[((size_t)k * d + j) * 2 * n];
      for (int i = 0; i < n; ++i) {
        row[i] = (j * hx[k * n + i]) % d;
        row[n + i] = (j * hz[k * n + i]) % d;
      }
      pph[(size_t)k * d + j] = (j * hp[k] + 2 * (xzsum % d) * (j * (j - 1) / 2)) % (2 * d);
    }
  }
  int* dxz = reinterpret_cast<int*>(ctx->B2);
  GC_HIP(hipMemcpy(dxz, pows.data(), pows.size() * sizeof(int), hipMemcpyHostToDevice));
  for (int k = 0; k < n; ++k) {
    for (int j = 0; j < d; ++j) {
      const int* row = dxz + ((size_t)k * d + j) * 2 * n;
      launch_apply_weyl_dense(s, n, d, D, row, row + n, pph[(size_t)k * d + j], va, vb, j > 0 ? 1 : 0,
                              z64{1.0 / d, 0.0});
    }
    std::swap(va, vb);
  }
  double nrm = 0.0;
  double* dn = reinterpret_cast<double*>(dxz + pows.size() + 64);
  launch_norm2(s, va, D, dn);
  GC_HIP(hipMemcpyAsync(&nrm, dn, sizeof(double), hipMemcpyDeviceToHost, s));
  GC_HIP(hipStreamSynchronize(s));
  GC_CHECK(nrm > 1e-20, GCAMPS_ENUMERIC, "stabilizer projection vanished");
  launch_scale(s, va, D, z64{1.0 / std::sqrt(nrm), 0.0});
  // per-x table of C X^x C^dagger = prod_k D_k^{x_k} = tau^{p_x} X^{a_x} Z^{b_x}
  std::vector<int> aidx(D), px(D);
  std::vector<int8_t> bd((size_t)D * n);
  std::vector<int> ax(n), bz(n);
  for (long long x = 0; x < D; ++x) {
    std::fill(ax.begin(), ax.end(), 0);
    std::fill(bz.begin(), bz.end(), 0);
    int p = 0;
    long long rem = x;
    std::vector<int> dig(n);
    for (int i = n - 1; i >= 0; --i) {
      dig[i] = (int)(rem % d);
      rem /= d;
    }
    for (int k = 0; k < n; ++k) {
      int e = dig[k];
      if (!e) continue;
      const int* rx = &hx[(n + k) * n];
      const int* rz = &hz[(n + k) * n];
      int xz = 0;
      for (int i = 0; i < n; ++i) xz += rx[i] * rz[i];
      int pw = (e * hp[n + k] + 2 * (xz % d) * (e * (e - 1) / 2)) % (2 * d);
      int cross = 0;
      for (int i = 0; i < n; ++i) cross += bz[i] * ((e * rx[i]) % d);
      p = (p + pw + 2 * (cross % d)) % (2 * d);
      for (int i = 0; i < n; ++i) {
        ax[i] = (ax[i] + e * rx[i]) % d;
        bz[i] = (bz[i] + e * rz[i]) % d;
      }
    }
    long long packed = 0;
    for (int i = 0; i < n; ++i) packed = packed * d + ax[i];
    aidx[x] = (int)packed;
    px[x] = p;
    for (int i = 0; i < n; ++i) bd[(size_t)x * n + i] = (int8_t)bz[i];
  }
  char* tbl = ctx->ws + ctx->lay.off_dense + (size_t)4 * D * sizeof(z64);
  int* d_aidx = reinterpret_cast<int*>(tbl);
  int* d_px = d_aidx + D;
  int8_t* d_bd = reinterpret_cast<int8_t*>(d_px + D);
  GC_HIP(hipMemcpy(d_aidx, aidx.data(), D * sizeof(int), hipMemcpyHostToDevice));
  GC_HIP(hipMemcpy(d_px, px.data(), D * sizeof(int), hipMemcpyHostToDevice));
  GC_HIP(hipMemcpy(d_bd, bd.data(), (size_t)D * n, hipMemcpyHostToDevice));
  launch_clifford_dense(s, n, d, D, d_aidx, d_bd, d_px, mv, va, out);
  GC_HIP(hipStreamSynchronize(s));
}

int32_t gcamps_statevector(gcamps_ctx* ctx, void* dev_out, void* dev_scratch, size_t scratch_bytes) {
  return guarded(ctx, [&] {
    GC_CHECK(ctx && dev_out && dev_scratch, GCAMPS_EINVAL, "null argument");
    const long long D = dense_dim(ctx);
    GC_CHECK(scratch_bytes >= (size_t)3 * D * sizeof(z64), GCAMPS_EWORKSPACE, "scratch smaller than 3*16*d^n bytes");
    statevector_impl(ctx, reinterpret_cast<z64*>(dev_out), reinterpret_cast<z64*>(dev_scratch));
  });
}

int32_t gcamps_statevector_static(gcamps_ctx* ctx, void* dev_out) {
  return guarded(ctx, [&] {
    GC_CHECK(ctx && dev_out, GCAMPS_EINVAL, "null argument");
    const long long D = dense_dim(ctx);
    GC_CHECK((size_t)D <= kDenseMax, GCAMPS_EUNSUPPORTED, "dense state above the static scratch (d^n <= 2^16)");
    GC_CHECK(ctx->scratch_dev != nullptr, GCAMPS_EDEVICE, "static scratch not resolved for this ctx's device");
    // every work vector is written before it is read (no part must start at zero)
    statevector_impl(ctx, reinterpret_cast<z64*>(dev_out), reinterpret_cast<z64*>(ctx->scratch_dev));
  });
}

int32_t gcamps_amplitude(gcamps_ctx* ctx, const int8_t* digits, double out[2]) {
  return guarded(ctx, [&] {
    GC_CHECK(ctx && digits && out, GCAMPS_EINVAL, "null argument");
    const long long D = dense_dim(ctx);
    long long y = 0;
    for (int i = 0; i < ctx->n; ++i) {
      GC_CHECK(digits[i] >= 0 && digits[i] < ctx->d, GCAMPS_EINVAL, "digit out of range");
      y = y * ctx->d + digits[i];
    }
    // the whole dense state is built in the ctx's dense region (validation-sized)
    z64* buf = reinterpret_cast<z64*>(ctx->ws + ctx->lay.off_dense);
    statevector_impl(ctx, buf, buf + D);
    z64 v;
    GC_HIP(hipMemcpy(&v, buf + y, sizeof(z64), hipMemcpyDeviceToHost));
    out[0] = v.re;
    out[1] = v.im;
  });
}

int32_t gcamps_get_tableau(gcamps_ctx* ctx, int32_t* out) {
  return guarded(nullptr, [&] {
    GC_CHECK(ctx && out, GCAMPS_EINVAL, "null argument");
    const int n = ctx->n;
    std::vector<int> hx(2 * n * n), hz(2 * n * n), hp(2 * n);
    GC_HIP(hipMemcpyAsync(hx.data(), ctx->tx, hx.size() * sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    GC_HIP(hipMemcpyAsync(hz.data(), ctx->tz, hz.size() * sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    GC_HIP(hipMemcpyAsync(hp.data(), ctx->tp, hp.size() * sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    GC_HIP(hipStreamSynchronize(ctx->stream));
    for (int r = 0; r < 2 * n; ++r) {
      for (int i = 0; i < n; ++i) {
        out[r * (2 * n + 1) + i] = hx[r * n + i];
        out[r * (2 * n + 1) + n + i] = hz[r * n + i];
      }
      out[r * (2 * n + 1) + 2 * n] = hp[r];
    }
  });
}

int32_t gcamps_get_bond_dims(gcamps_ctx* ctx, int32_t* out) {
  return guarded(nullptr, [&] {
    GC_CHECK(ctx && out, GCAMPS_EINVAL, "null argument");
    for (int i = 0; i < ctx->n - 1; ++i) out[i] = ctx->chi[i + 1];
  });
}

int32_t gcamps_get_fidelity(gcamps_ctx* ctx, double* f_est) {
  return guarded(nullptr, [&] {
    GC_CHECK(ctx && f_est, GCAMPS_EINVAL, "null argument");
    *f_est = ctx->f_est;
  });
}

int32_t gcamps_get_choice_log(gcamps_ctx* ctx, int32_t* out, int64_t cap, int64_t* len) {
  return guarded(nullptr, [&] {
    GC_CHECK(ctx && len, GCAMPS_EINVAL, "null argument");
    const int64_t total = (int64_t)ctx->choice_log.size() / 4;
    *len = total;
    if (out && cap > 0)
      std::memcpy(out, ctx->choice_log.data(), (size_t)std::min(cap, total) * 4 * sizeof(int32_t));
  });
}

int32_t gcamps_get_site(gcamps_ctx* ctx, int32_t site, double* out, int64_t cap, int32_t dims[3]) {
  return guarded(nullptr, [&] {
    GC_CHECK(ctx && dims, GCAMPS_EINVAL, "null argument");
    GC_CHECK(site >= 0 && site < ctx->n, GCAMPS_EINVAL, "site out of range");
    dims[0] = ctx->chi[site];
    dims[1] = ctx->d;
    dims[2] = ctx->chi[site + 1];
    const int64_t cnt = (int64_t)dims[0] * dims[1] * dims[2];
    if (out) {
      GC_CHECK(cap >= cnt, GCAMPS_EINVAL, "output capacity too small");
      GC_HIP(hipMemcpyAsync(out, ctx->site[site], cnt * sizeof(z64), hipMemcpyDeviceToHost, ctx->stream));
      GC_HIP(hipStreamSynchronize(ctx->stream));
    }
  });
}

int32_t gcamps_get_kernel_stats(gcamps_ctx* ctx, double out[8]) {
  return guarded(ctx, [&] {
    GC_CHECK(ctx && out, GCAMPS_EINVAL, "null argument");
    ctx->settle_mpo();
    for (int i = 0; i < 6; ++i) out[i] = ctx->kstats[i];
    out[6] = ctx->stats_red[0];
    out[7] = ctx->stats_red[2] > 0 ? ctx->stats_red[1] / ctx->stats_red[2] : 0.0;
  });
}

int32_t gcamps_get_stats(gcamps_ctx* ctx, double out[16]) {
  return guarded(nullptr, [&] {
    GC_CHECK(ctx && out, GCAMPS_EINVAL, "null argument");
    for (int i = 0; i < 16; ++i) out[i] = ctx->stats[i];
  });
}

}  // extern "C"
