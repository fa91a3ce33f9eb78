// Batched independent circuits: a lane pool over HIP streams.
//
// Each lane is a host thread that owns one HIP stream and one slice of the caller's
// workspace.  Lanes take circuits from a shared queue ordered by estimated cost (largest
// first) and run each one through the single-state C ABI, so a circuit in a batch executes
// exactly the kernel sequence it would execute alone.  The bottom loop of one circuit is a
// chain of dependent factorisations; the parallelism here is across circuits, whose
// latency-bound kernels (eigensolver rounds, small splits) overlap on the GPU.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "internal.h"

using namespace gc;

namespace {

inline size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

constexpr int kMaxLanes = 64;

size_t lane_bytes(const gcamps_batch_item* items, int32_t count) {
  size_t per = 0;
  for (int i = 0; i < count; ++i) {
    size_t b = 0;
    const int32_t rc = gcamps_workspace_bytes(&items[i].cfg, &b);
    if (rc != GCAMPS_OK)
      throw Error{rc, "item " + std::to_string(i) + ": " + std::string(gcamps_last_error())};
    per = std::max(per, align256(b));
  }
  return per;
}

void validate_items(const gcamps_batch_item* items, int32_t count, int32_t lanes) {
  GC_CHECK(items != nullptr && count >= 1, GCAMPS_EINVAL, "batch: null items or empty batch");
  GC_CHECK(lanes >= 1 && lanes <= kMaxLanes, GCAMPS_EINVAL, "batch: lanes out of range [1, 64]");
  for (int i = 0; i < count; ++i) {
    const gcamps_batch_item& it = items[i];
    GC_CHECK(it.n_ops >= 0 && (it.n_ops == 0 || it.ops != nullptr), GCAMPS_EINVAL,
             "batch: item " + std::to_string(i) + " has null ops");
    for (int64_t k = 0; k < it.n_ops; ++k) {
      const gcamps_op& op = it.ops[k];
      GC_CHECK(op.kind == GCAMPS_OP_CLIFFORD_LAYER || op.kind == GCAMPS_OP_PHASE, GCAMPS_EINVAL,
               "batch: item " + std::to_string(i) + " op " + std::to_string(k) + " has an unknown kind");
      if (op.kind == GCAMPS_OP_CLIFFORD_LAYER)
        GC_CHECK(op.count >= 0 && (op.count == 0 || (op.sites && op.words)), GCAMPS_EINVAL,
                 "batch: item " + std::to_string(i) + " op " + std::to_string(k) + " is missing sites/words");
      else
        GC_CHECK(op.sites && op.phi, GCAMPS_EINVAL,
                 "batch: item " + std::to_string(i) + " op " + std::to_string(k) + " is missing site/phi");
    }
  }
}

// Relative cost used to order the queue: phase gates times chain length.
double item_cost(const gcamps_batch_item& it) {
  int64_t phases = 0;
  for (int64_t k = 0; k < it.n_ops; ++k) phases += it.ops[k].kind == GCAMPS_OP_PHASE;
  return (double)(phases + 1) * it.cfg.n * it.cfg.chi_max;
}

struct LaneResult {
  double busy_ms = 0.0, score_ms = 0.0, bonds = 0.0, gates = 0.0, gram_n = 0.0, gram_ms = 0.0, gram_flops = 0.0;
  int done = 0;
};

// Run one circuit on a lane; returns the status and writes the item's outputs.
int32_t run_item(const gcamps_batch_item& it, const gcamps_candset* set, void* ws, size_t ws_bytes,
                 hipStream_t stream, LaneResult& lr, std::string& err) {
  gcamps_ctx* ctx = nullptr;
  int32_t rc = gcamps_init(&it.cfg, ws, ws_bytes, stream, &ctx);
  auto fail = [&](int32_t code) {
    err = gcamps_last_error();
    if (ctx) gcamps_destroy(ctx);
    return code;
  };
  if (rc != GCAMPS_OK) return fail(rc);
  if (set && (rc = gcamps_set_candset(ctx, set)) != GCAMPS_OK) return fail(rc);
  for (int64_t k = 0; k < it.n_ops; ++k) {
    const gcamps_op& op = it.ops[k];
    if (op.kind == GCAMPS_OP_CLIFFORD_LAYER)
      rc = gcamps_apply_clifford_layer(ctx, op.sites, op.words, op.count);
    else
      rc = gcamps_apply_phase_rotation(ctx, op.sites[0], op.phi);
    if (rc != GCAMPS_OK) return fail(rc);
  }
  const int n = it.cfg.n;
  if (it.z_expect) {
    std::vector<int8_t> x(n, 0), z(n, 0);
    for (int j = 0; j < n; ++j) {
      z[j] = 1;
      if ((rc = gcamps_expectation(ctx, x.data(), z.data(), 0, it.z_expect + 2 * j)) != GCAMPS_OK) return fail(rc);
      z[j] = 0;
    }
  }
  if (it.fidelity && (rc = gcamps_get_fidelity(ctx, it.fidelity)) != GCAMPS_OK) return fail(rc);
  if (it.bond_dims && (rc = gcamps_get_bond_dims(ctx, it.bond_dims)) != GCAMPS_OK) return fail(rc);
  if (it.choices_len || it.choices) {
    int64_t len = 0;
    rc = gcamps_get_choice_log(ctx, it.choices, it.choices ? it.choices_cap : 0, &len);
    if (rc != GCAMPS_OK) return fail(rc);
    if (it.choices_len) *it.choices_len = len;
  }
  double st[16];
  if ((rc = gcamps_get_stats(ctx, st)) != GCAMPS_OK) return fail(rc);
  lr.busy_ms += st[7];
  lr.score_ms += st[6];
  lr.bonds += st[1];
  lr.gates += st[0];
  lr.gram_n += st[11];
  lr.gram_ms += st[12];
  lr.gram_flops += st[13];
  lr.done += 1;
  gcamps_destroy(ctx);
  return GCAMPS_OK;
}

}  // namespace

extern "C" {

int32_t gcamps_batch_workspace_bytes(const gcamps_batch_item* items, int32_t count, int32_t lanes,
                                     size_t* bytes) {
  try {
    GC_CHECK(bytes != nullptr, GCAMPS_EINVAL, "batch: bytes is null");
    validate_items(items, count, lanes);
    *bytes = lane_bytes(items, count) * (size_t)std::min(lanes, count);
    return GCAMPS_OK;
  } catch (const Error& e) {
    set_error(e.msg);
    return e.code;
  }
}

int32_t gcamps_batch_run(const gcamps_batch_item* items, int32_t count, const gcamps_candset* set,
                         int32_t lanes, void* dev_workspace, size_t bytes, double stats[16]) {
  try {
    validate_items(items, count, lanes);
    GC_CHECK(dev_workspace != nullptr, GCAMPS_EINVAL, "batch: null workspace");
    GC_CHECK(((uintptr_t)dev_workspace & 255) == 0, GCAMPS_EINVAL, "batch: workspace must be 256-byte aligned");
    const int nl = std::min(lanes, count);
    const size_t per = lane_bytes(items, count);
    GC_CHECK(bytes >= per * (size_t)nl, GCAMPS_EWORKSPACE, "batch: workspace smaller than gcamps_batch_workspace_bytes()");
    if (set)
      for (int i = 0; i < count; ++i)
        GC_CHECK(items[i].cfg.d == set->d, GCAMPS_EINVAL, "batch: item d differs from the candidate set's d");
    int device = 0;
    GC_HIP(hipGetDevice(&device));

    // queue: largest estimated cost first (stable, so equal costs keep input order)
    std::vector<int> order(count);
    for (int i = 0; i < count; ++i) order[i] = i;
    std::vector<double> cost(count);
    for (int i = 0; i < count; ++i) cost[i] = item_cost(items[i]);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });

    std::vector<hipStream_t> streams(nl, nullptr);
    for (int l = 0; l < nl; ++l) GC_HIP(hipStreamCreateWithFlags(&streams[l], hipStreamNonBlocking));
    struct StreamGuard {
      std::vector<hipStream_t>& s;
      ~StreamGuard() {
        for (auto x : s)
          if (x) (void)hipStreamDestroy(x);
      }
    } guard{streams};

    std::atomic<int> next{0};
    std::vector<LaneResult> lres(nl);
    std::mutex err_mu;
    int32_t first_rc = GCAMPS_OK;
    int first_item = -1;
    std::string first_msg;
    const auto t0 = std::chrono::steady_clock::now();
    auto lane_fn = [&](int l) {
      if (hipSetDevice(device) != hipSuccess) {
        std::lock_guard<std::mutex> lk(err_mu);
        if (first_rc == GCAMPS_OK) {
          first_rc = GCAMPS_EDEVICE;
          first_msg = "batch: hipSetDevice failed in a lane";
        }
        return;
      }
      char* ws = reinterpret_cast<char*>(dev_workspace) + (size_t)l * per;
      for (;;) {
        const int q = next.fetch_add(1);
        if (q >= count) break;
        const int idx = order[q];
        const gcamps_batch_item& it = items[idx];
        std::string msg;
        const int32_t rc = run_item(it, set, ws, per, streams[l], lres[l], msg);
        if (it.status) *it.status = rc;
        if (rc != GCAMPS_OK) {
          std::lock_guard<std::mutex> lk(err_mu);
          if (first_rc == GCAMPS_OK || idx < first_item) {
            first_rc = rc;
            first_item = idx;
            first_msg = "batch item " + std::to_string(idx) + ": " + msg;
          }
        }
      }
    };
    std::vector<std::thread> pool;
    for (int l = 1; l < nl; ++l) pool.emplace_back(lane_fn, l);
    lane_fn(0);
    for (auto& t : pool) t.join();
    const double wall = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (stats) {
      for (int i = 0; i < 16; ++i) stats[i] = 0.0;
      for (const auto& r : lres) {
        stats[0] += r.done;
        stats[1] += r.gates;
        stats[3] += r.busy_ms;
        stats[5] += r.score_ms;
        stats[6] += r.bonds;
        stats[7] += r.gram_n;
        stats[8] += r.gram_ms;
        stats[9] += r.gram_flops;
      }
      stats[2] = wall;
      stats[4] = nl;
    }
    if (first_rc != GCAMPS_OK) {
      set_error(first_msg);
      return first_rc;
    }
    return GCAMPS_OK;
  } catch (const Error& e) {
    set_error(e.msg);
    return e.code;
  }
}

}  // extern "C"
