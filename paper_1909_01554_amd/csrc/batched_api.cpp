// Batched products: plan construction (device-resident problem table sorted by
// decreasing k) and launches of the persistent kernel.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/bmm.h"
#include "bmm_internal.h"

using namespace bmm;

namespace {

#define bfail bmm::set_error

struct Plan {
  BatchedDesc* descs = nullptr;  // device
  BatchedSeg* segs = nullptr;    // device: every queue's segments, queue after queue
  unsigned int* counters = nullptr;
  BatchedQueues queues{};
  int64_t count = 0;
  int grid = 0;
  int device = 0;
  int leaf = BMM_LEAF_MFMA_I8;  // BMM_LEAF_MFMA_I8 or BMM_LEAF_MFMA_F4
  int tile = 2;                 // 1: 128 x 64 per wave, 2: 64 x 64, 3: 64 x 128
  // Marks the end of the last launch enqueued outside stream capture; the next launch
  // (on any stream) waits for it, so launches that share the queue counters never overlap.
  hipEvent_t done = nullptr;
};

bool capturing(hipStream_t s) {
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  return hipStreamIsCapturing(s, &st) == hipSuccess && st != hipStreamCaptureStatusNone;
}

// Launch a plan's kernels (counter reset + persistent kernel) on s.  Outside stream
// capture the launch is ordered after the plan's previous one by its event.
int plan_enqueue(Plan* P, hipStream_t s) {
  if (P->count == 0) return BMM_OK;
  const bool cap = capturing(s);
  if (!cap) {
    if (!P->done && hipEventCreateWithFlags(&P->done, hipEventDisableTiming) != hipSuccess)
      return bfail(BMM_E_DEVICE, "plan event: %s", hipGetErrorString(hipGetLastError()));
    if (hipStreamWaitEvent(s, P->done, 0) != hipSuccess)
      return bfail(BMM_E_DEVICE, "plan order: %s", hipGetErrorString(hipGetLastError()));
  }
  hipError_t e = launch_batched_persistent(
      P->descs, P->segs, P->queues, P->counters, P->grid, P->tile,
      P->leaf == BMM_LEAF_MFMA_F4 ? 1 : 0, s);
  if (e != hipSuccess) return bfail(BMM_E_DEVICE, "batched launch: %s", hipGetErrorString(e));
  if (!cap && hipEventRecord(P->done, s) != hipSuccess)
    return bfail(BMM_E_DEVICE, "plan event: %s", hipGetErrorString(hipGetLastError()));
  return BMM_OK;
}

void plan_free(Plan* P) {
  if (P->descs || P->counters || P->done) {
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(P->device);
    if (P->done) {
      (void)hipEventSynchronize(P->done);
      (void)hipEventDestroy(P->done);
    } else {
      (void)hipDeviceSynchronize();
    }
    (void)hipFree(P->descs);
    (void)hipFree(P->segs);
    (void)hipFree(P->counters);
    (void)hipSetDevice(cur);
  }
  P->descs = nullptr;
  P->segs = nullptr;
  P->counters = nullptr;
  P->done = nullptr;
}

int validate_problem(const bmm_problem& p, int64_t i) {
  if (p.semiring != BMM_GF2 && p.semiring != BMM_BOOLEAN)
    return bfail(BMM_E_INVAL, "problem %ld: bad semiring", (long)i);
  if (p.m < 0 || p.k < 0 || p.n < 0) return bfail(BMM_E_INVAL, "problem %ld: negative size", (long)i);
  if (p.m == 0 || p.n == 0) return BMM_OK;
  const int64_t kw = (p.k + 63) / 64, nw = (p.n + 63) / 64;
  if (!p.C || p.ldc < nw) return bfail(BMM_E_INVAL, "problem %ld: bad C or ldc", (long)i);
  if (p.k > 0) {
    if (!p.A || !p.B) return bfail(BMM_E_INVAL, "problem %ld: null A or B", (long)i);
    if (p.lda < kw) return bfail(BMM_E_INVAL, "problem %ld: lda too small", (long)i);
    if (p.b_transposed ? p.ldb < kw : p.ldb < nw)
      return bfail(BMM_E_INVAL, "problem %ld: ldb too small", (long)i);
  }
  if (((uintptr_t)p.A | (uintptr_t)p.B | (uintptr_t)p.C) & 7)
    return bfail(BMM_E_INVAL, "problem %ld: pointers must be 8-byte aligned", (long)i);
  return BMM_OK;
}

// wg_per_cu > 0 fixes the persistent grid (workgroups per CU); 0 takes the record.
int build_plan(const bmm_problem* problems, int64_t count, const bmm_options* opt,
               int wg_per_cu, Plan* out) {
  if (count < 0 || (count > 0 && !problems)) return bfail(BMM_E_INVAL, "bad problem list");
  std::vector<int64_t> order;
  double ops = 0;
  int64_t kmax = 0;
  for (int64_t i = 0; i < count; ++i) {
    int rc = validate_problem(problems[i], i);
    if (rc != BMM_OK) return rc;
    if (!problems[i].b_transposed)
      return bfail(BMM_E_INVAL, "problem %ld: plans need B passed transposed", (long)i);
    if (problems[i].m > 0 && problems[i].n > 0) order.push_back(i);
    ops += 2.0 * problems[i].m * problems[i].k * problems[i].n;
    kmax = std::max(kmax, problems[i].k);
  }
  // leaf kind and tile: explicit options, else the autotuner's record for plans of this
  // count and total work, else int8 with 64 x 64 tiles
  int leaf = opt ? opt->leaf : BMM_LEAF_AUTO;
  int tile = opt ? opt->tile : 0;
  int tl = 0, tt = 0, tw = 0;
  if (batched_tuned(count, ops, &tl, &tt, &tw)) {
    if (leaf == BMM_LEAF_AUTO) leaf = tl;
    if (tile <= 0) tile = tt;
    if (wg_per_cu <= 0) wg_per_cu = tw;
  }
  if (wg_per_cu <= 0) wg_per_cu = 4;
  if (leaf == BMM_LEAF_AUTO) leaf = BMM_LEAF_MFMA_I8;
  if (tile <= 0) tile = 2;
  if (leaf != BMM_LEAF_MFMA_I8 && leaf != BMM_LEAF_MFMA_F4)
    return bfail(BMM_E_UNSUPPORTED, "batched plans run the int8 or fp4 matrix-core leaf");
  if (tile < 1 || tile > 4) return bfail(BMM_E_INVAL, "batched tile must be 1, 2, 3 or 4");
  if (leaf == BMM_LEAF_MFMA_F4 && kmax >= ((int64_t)1 << 24))
    return bfail(BMM_E_UNSUPPORTED, "the fp4 leaf counts exactly only for k < 2^24");
  if (kmax >= ((int64_t)1 << 31))
    return bfail(BMM_E_UNSUPPORTED, "the int8 leaf counts exactly only for k < 2^31");
  // longest k first, so the queues drain with short items at the end
  std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) {
    return problems[a].k > problems[b].k;
  });
  const int TR = batched_tile_rows(tile), TC = batched_tile_cols(tile);
  std::vector<BatchedDesc> host;
  std::vector<BatchedSeg> qsegs[kXcds];
  uint64_t qitems[kXcds] = {};
  int rot = 0;
  for (int64_t i : order) {
    const bmm_problem& p = problems[i];
    BatchedDesc d;
    d.A = p.A;
    d.BT = p.B;
    d.C = p.C;
    d.lda = p.lda;
    d.ldbt = p.ldb;
    d.ldc = p.ldc;
    d.m = p.m;
    d.k = p.k;
    d.n = p.n;
    d.semiring = p.semiring;
    d.aligned = ((((uintptr_t)p.A | (uintptr_t)p.B) & 15) == 0 && ((p.lda | p.ldb) & 1) == 0) ? 1 : 0;
    // wave tiles cover whole 64-bit words of C, so padding bits are written (as zero)
    const int64_t tiles_m = (p.m + TR - 1) / TR;
    const int64_t tiles_n = (((p.n + 63) / 64) * 64 + TC - 1) / TC;
    const int64_t items_m = (tiles_m + 1) / 2, items_n = (tiles_n + 1) / 2;
    if (tiles_m >= ((int64_t)1 << 31) || tiles_n >= ((int64_t)1 << 31))
      return bfail(BMM_E_UNSUPPORTED, "problem %ld: too many tiles", (long)i);
    d.tiles_m = (int32_t)tiles_m;
    d.tiles_n = (int32_t)tiles_n;
    d.items_m = (int32_t)items_m;
    d.items_n = (int32_t)items_n;
    const uint32_t pi = (uint32_t)host.size();
    host.push_back(d);
    // the problem's items, in banded order, split into contiguous ranges over the
    // queues; the odd items left over rotate from problem to problem
    const uint64_t items = (uint64_t)items_m * (uint64_t)items_n;
    if (items >= ((uint64_t)1 << 32))  // segments hold a problem's item index in 32 bits
      return bfail(BMM_E_UNSUPPORTED, "problem %ld: too many work items", (long)i);
    const uint64_t base = items / kXcds, rem = items % kXcds;
    uint64_t lo = 0;
    for (int xi = 0; xi < kXcds; ++xi) {
      const uint64_t sz = base + ((uint64_t)xi < rem ? 1 : 0);
      if (sz == 0) continue;
      const int x = (rot + xi) % kXcds;
      qsegs[x].push_back(BatchedSeg{(uint32_t)qitems[x], pi, (uint32_t)lo, 0u});
      qitems[x] += sz;
      lo += sz;
    }
    rot = (int)((rot + rem) % kXcds);
  }
  Plan P;
  P.leaf = leaf;
  P.tile = tile;
  P.count = (int64_t)host.size();
  std::vector<BatchedSeg> segs;
  for (int x = 0; x < kXcds; ++x) {
    if (qitems[x] >= ((uint64_t)1 << 32) - ((uint64_t)1 << 20))
      return bfail(BMM_E_UNSUPPORTED, "batched plans hold fewer than 2^32 items per queue");
    P.queues.seg_off[x] = (uint32_t)segs.size();
    P.queues.seg_count[x] = (uint32_t)qsegs[x].size();
    P.queues.items[x] = (uint32_t)qitems[x];
    segs.insert(segs.end(), qsegs[x].begin(), qsegs[x].end());
  }
  if (hipGetDevice(&P.device) != hipSuccess) return bfail(BMM_E_DEVICE, "hipGetDevice");
  int cus = 256;
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, P.device);
  P.grid = std::max(kXcds, cus * wg_per_cu);
  if (P.count > 0) {
    const size_t cbytes = sizeof(unsigned int) * kXcds * kBatchedCounterStride;
    if (bmm::dev_malloc((void**)&P.descs, sizeof(BatchedDesc) * host.size()) != hipSuccess ||
        bmm::dev_malloc((void**)&P.segs, sizeof(BatchedSeg) * segs.size()) != hipSuccess ||
        bmm::dev_malloc((void**)&P.counters, cbytes) != hipSuccess) {
      (void)hipGetLastError();
      (void)hipFree(P.descs);
      (void)hipFree(P.segs);
      return bfail(BMM_E_NOMEM, "plan allocation");
    }
    if (hipMemcpy(P.descs, host.data(), sizeof(BatchedDesc) * host.size(),
                  hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(P.segs, segs.data(), sizeof(BatchedSeg) * segs.size(),
                  hipMemcpyHostToDevice) != hipSuccess) {
      (void)hipFree(P.descs);
      (void)hipFree(P.segs);
      (void)hipFree(P.counters);
      return bfail(BMM_E_DEVICE, "plan upload: %s", hipGetErrorString(hipGetLastError()));
    }
  }
  *out = P;
  return BMM_OK;
}

#define BMM_BTRY(expr)              \
  do {                              \
    int _rc = (expr);               \
    if (_rc != BMM_OK) return _rc;  \
  } while (0)

// Library-owned plans of bmm_batched, keyed by the problem table (pointers, sizes,
// pitches, semirings), the leaf and tile options and the device.  An entry owns the
// device problem table, a staging buffer for right operands not given transposed,
// and a HIP graph of its launch sequence (the transposes into staging, the counter
// reset and the persistent kernel), captured on its first call and replayed on the
// caller's stream by later calls.  Launches of one entry are ordered by its event.
struct BatchedEntry {
  std::vector<bmm_problem> key;
  int leaf = 0, tile = 0, device = 0;
  uint64_t tune_gen = 0;  // the batched tuning records the plan was built from
  Plan plan;
  std::vector<bmm_problem> staged;  // the problems as the plan sees them (B^T everywhere)
  uint64_t* stage = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipEvent_t done = nullptr;
  uint64_t used = 0;

  static bool same(const bmm_problem& a, const bmm_problem& b) {
    return a.semiring == b.semiring && a.m == b.m && a.k == b.k && a.n == b.n && a.A == b.A &&
           a.B == b.B && a.C == b.C && a.lda == b.lda && a.ldb == b.ldb && a.ldc == b.ldc &&
           (a.b_transposed != 0) == (b.b_transposed != 0);
  }
  bool matches(const bmm_problem* p, int64_t count, int lf, int tl, int dev) const {
    if (dev != device || lf != leaf || tl != tile || (int64_t)key.size() != count ||
        tune_gen != batched_tune_generation())
      return false;
    for (int64_t i = 0; i < count; ++i)
      if (!same(key[(size_t)i], p[i])) return false;
    return true;
  }

  // The transposes of untransposed right operands, then the plan's kernels.
  int enqueue(hipStream_t s) {
    for (size_t i = 0; i < key.size(); ++i) {
      const bmm_problem& p = key[i];
      if (p.b_transposed || p.m == 0 || p.n == 0 || p.k == 0) continue;
      const bmm_problem& q = staged[i];
      hipError_t e = launch_transpose(p.B, p.ldb, 0, const_cast<uint64_t*>(q.B), q.ldb, 0, p.k,
                                      p.n, 1, s);
      if (e != hipSuccess) return bfail(BMM_E_DEVICE, "transpose: %s", hipGetErrorString(e));
    }
    if (plan.count == 0) return BMM_OK;
    hipError_t e = launch_batched_persistent(plan.descs, plan.segs, plan.queues, plan.counters,
                                             plan.grid, plan.tile,
                                             plan.leaf == BMM_LEAF_MFMA_F4 ? 1 : 0, s);
    if (e != hipSuccess) return bfail(BMM_E_DEVICE, "batched launch: %s", hipGetErrorString(e));
    return BMM_OK;
  }

  int build(const bmm_problem* p, int64_t count, const bmm_options* opt, int lf, int tl,
            int dev) {
    key.assign(p, p + count);
    tune_gen = batched_tune_generation();
    leaf = lf;
    tile = tl;
    device = dev;
    staged = key;
    size_t need = 0;
    for (const auto& q : key)
      if (!q.b_transposed && q.m > 0 && q.n > 0 && q.k > 0)
        need += (size_t)q.n * ((q.k + 63) / 64) * 8;
    if (need && bmm::dev_malloc((void**)&stage, need) != hipSuccess) {
      (void)hipGetLastError();
      stage = nullptr;
      return bfail(BMM_E_NOMEM, "batched staging of %zu bytes", need);
    }
    size_t off = 0;
    for (auto& q : staged) {
      if (!q.b_transposed && q.m > 0 && q.n > 0 && q.k > 0) {
        const int64_t kw = (q.k + 63) / 64;
        q.B = stage + off / 8;
        q.ldb = kw;
        off += (size_t)q.n * kw * 8;
      }
      q.b_transposed = 1;
    }
    BMM_BTRY(build_plan(staged.data(), count, opt, 0, &plan));
    if (hipEventCreateWithFlags(&done, hipEventDisableTiming) != hipSuccess)
      return bfail(BMM_E_DEVICE, "batched event: %s", hipGetErrorString(hipGetLastError()));
    // capture the sequence once; if this runtime cannot, launches enqueue it directly
    hipStream_t cs = nullptr;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) == hipSuccess) {
      bool ok = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess;
      const int rc = ok ? enqueue(cs) : BMM_OK;
      hipGraph_t g = nullptr;
      if (ok) ok = hipStreamEndCapture(cs, &g) == hipSuccess && rc == BMM_OK && g;
      if (ok && hipGraphInstantiate(&exec, g, nullptr, nullptr, 0) == hipSuccess) {
        graph = g;
      } else {
        exec = nullptr;
        if (g) (void)hipGraphDestroy(g);
      }
      (void)hipGetLastError();
      (void)hipStreamDestroy(cs);
    }
    return BMM_OK;
  }

  int launch(hipStream_t s, bool cap) {
    if (cap) return enqueue(s);  // inside the caller's capture: the kernels themselves
    if (hipStreamWaitEvent(s, done, 0) != hipSuccess)
      return bfail(BMM_E_DEVICE, "batched order: %s", hipGetErrorString(hipGetLastError()));
    if (exec) {
      if (hipGraphLaunch(exec, s) != hipSuccess)
        return bfail(BMM_E_DEVICE, "batched graph launch: %s",
                     hipGetErrorString(hipGetLastError()));
    } else {
      BMM_BTRY(enqueue(s));
    }
    if (hipEventRecord(done, s) != hipSuccess)
      return bfail(BMM_E_DEVICE, "batched event: %s", hipGetErrorString(hipGetLastError()));
    return BMM_OK;
  }

  ~BatchedEntry() {
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(device);
    if (done) (void)hipEventSynchronize(done);
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (done) (void)hipEventDestroy(done);
    plan_free(&plan);
    (void)hipFree(stage);
    (void)hipSetDevice(cur);
  }
};

constexpr size_t kBatchedCacheEntries = 8;
std::mutex g_batched_mu;
std::vector<std::unique_ptr<BatchedEntry>> g_entries;
uint64_t g_batched_clock = 0;

}  // namespace

extern "C" {

int bmm_batched_plan_create(const bmm_problem* problems, int64_t count,
                            const bmm_options* opt, void** plan_out) {
  if (!plan_out) return bfail(BMM_E_INVAL, "null plan_out");
  Plan* P = new Plan();
  int rc = build_plan(problems, count, opt, 0, P);
  if (rc != BMM_OK) {
    delete P;
    return rc;
  }
  *plan_out = P;
  return BMM_OK;
}

int bmm_batched_plan_launch(void* plan, void* hip_stream) {
  if (!plan) return bfail(BMM_E_INVAL, "null plan");
  return plan_enqueue(static_cast<Plan*>(plan), (hipStream_t)hip_stream);
}

void bmm_batched_plan_destroy(void* plan) {
  if (!plan) return;
  Plan* P = static_cast<Plan*>(plan);
  plan_free(P);
  delete P;
}

int bmm_autotune_batched(const bmm_problem* problems, int64_t count, int* leaf_out,
                         int* tile_out, double* seconds_out) {
  if (count <= 0 || !problems) return bfail(BMM_E_INVAL, "bad problem list");
  double ops = 0;
  for (int64_t i = 0; i < count; ++i) ops += 2.0 * problems[i].m * problems[i].k * problems[i].n;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return bfail(BMM_E_DEVICE, "event create");
  double best = 1e30;
  int best_leaf = BMM_LEAF_MFMA_I8, best_tile = 2, best_wpc = 4, rc = BMM_OK;
  for (int leaf : {BMM_LEAF_MFMA_I8, BMM_LEAF_MFMA_F4}) {
    for (int tile : {1, 2, 3, 4}) {
      for (int wpc : {2, 4}) {
        bmm_options o;
        bmm_options_init(&o);
        o.leaf = leaf;
        o.tile = tile;
        Plan* plan = new Plan();
        rc = build_plan(problems, count, &o, wpc, plan);
        if (rc == BMM_E_UNSUPPORTED) {  // e.g. fp4 with k >= 2^24: not a candidate
          delete plan;
          rc = BMM_OK;
          continue;
        }
        if (rc != BMM_OK) {
          delete plan;
          break;
        }
        rc = bmm_batched_plan_launch(plan, nullptr);  // warm-up
        if (rc == BMM_OK) {
          (void)hipEventRecord(e0, nullptr);
          rc = bmm_batched_plan_launch(plan, nullptr);
          (void)hipEventRecord(e1, nullptr);
        }
        float ms = 0.f;
        if (rc == BMM_OK && (hipEventSynchronize(e1) != hipSuccess ||
                             hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
          rc = bfail(BMM_E_DEVICE, "autotune timing: %s", hipGetErrorString(hipGetLastError()));
        bmm_batched_plan_destroy(plan);
        if (rc != BMM_OK) break;
        if (ms * 1e-3 < best) {
          best = ms * 1e-3;
          best_leaf = leaf;
          best_tile = tile;
          best_wpc = wpc;
        }
      }
      if (rc != BMM_OK) break;
    }
    if (rc != BMM_OK) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != BMM_OK) return rc;
  batched_tune_set(count, ops, best_leaf, best_tile, best_wpc);
  if (leaf_out) *leaf_out = best_leaf;
  if (tile_out) *tile_out = best_tile;
  if (seconds_out) *seconds_out = best;
  return BMM_OK;
}

int bmm_batched(const bmm_problem* problems, int64_t count, const bmm_options* opt,
                void* hip_stream) {
  if (count < 0 || (count > 0 && !problems)) return bfail(BMM_E_INVAL, "bad problem list");
  if (count == 0) return BMM_OK;
  for (int64_t i = 0; i < count; ++i) {
    int rc = validate_problem(problems[i], i);
    if (rc != BMM_OK) return rc;
  }
  hipStream_t s = (hipStream_t)hip_stream;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return bfail(BMM_E_DEVICE, "hipGetDevice");
  const int leaf = opt ? opt->leaf : BMM_LEAF_AUTO, tile = opt ? opt->tile : 0;
  std::lock_guard<std::mutex> lock(g_batched_mu);
  BatchedEntry* E = nullptr;
  const uint64_t gen = batched_tune_generation();
  g_entries.erase(std::remove_if(g_entries.begin(), g_entries.end(),
                                 [gen](const auto& e) { return e->tune_gen != gen; }),
                  g_entries.end());
  for (auto& e : g_entries)
    if (e->matches(problems, count, leaf, tile, dev)) E = e.get();
  const bool cap = capturing(s);
  if (!E) {
    if (cap)
      return bfail(BMM_E_UNSUPPORTED, "the first bmm_batched call with a problem table "
                   "builds its plan (allocation, upload) and must run outside stream capture");
    auto fresh = std::make_unique<BatchedEntry>();
    BMM_BTRY(fresh->build(problems, count, opt, leaf, tile, dev));
    if (g_entries.size() >= kBatchedCacheEntries) {
      // least recently used first
      auto lru = std::min_element(g_entries.begin(), g_entries.end(),
                                  [](const auto& a, const auto& b) { return a->used < b->used; });
      g_entries.erase(lru);
    }
    g_entries.push_back(std::move(fresh));
    E = g_entries.back().get();
  }
  E->used = ++g_batched_clock;
  return E->launch(s, cap);
}

}  // extern "C"

namespace bmm {
void batched_cache_clear() {
  std::lock_guard<std::mutex> lock(g_batched_mu);
  g_entries.clear();
}
}  // namespace bmm
