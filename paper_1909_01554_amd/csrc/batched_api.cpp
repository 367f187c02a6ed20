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

#define BMM_BTRY(expr)              \
  do {                              \
    int _rc = (expr);               \
    if (_rc != BMM_OK) return _rc;  \
  } while (0)

// One persistent group of a plan: a device problem table, its per-XCD queues and their
// counters, for problems that share a matrix-core leaf kind and tile.
struct Plan {
  BatchedDesc* descs = nullptr;  // device
  BatchedSeg* segs = nullptr;    // device: every queue's segments, queue after queue
  unsigned int* counters = nullptr;
  BatchedQueues queues{};
  int64_t count = 0;
  int grid = 0;
  int device = 0;
  int leaf = BMM_LEAF_MFMA_I8;  // BMM_LEAF_MFMA_I8 or BMM_LEAF_MFMA_F4
  int tile = 4;                 // 1: 128 x 64 per wave, 2: 64 x 64, 3: 64 x 128,
                                // 4: 128 x 64 with LDS-shared operand rows
};

bool capturing(hipStream_t s) {
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  return hipStreamIsCapturing(s, &st) == hipSuccess && st != hipStreamCaptureStatusNone;
}

// Free a group's device memory; the caller has made sure no launch of it still runs.
void plan_free(Plan* P) {
  (void)hipFree(P->descs);
  (void)hipFree(P->segs);
  (void)hipFree(P->counters);
  P->descs = nullptr;
  P->segs = nullptr;
  P->counters = nullptr;
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

// One persistent group: the problems `idx` of the table (validated, B^T given), all
// with the same matrix-core leaf kind and tile, on a grid of wg_per_cu workgroups per CU.
int build_plan(const bmm_problem* problems, const std::vector<int64_t>& idx, int leaf,
               int tile, int wg_per_cu, Plan* out) {
  std::vector<int64_t> order;
  int64_t kmax = 0;
  for (int64_t i : idx) {
    if (problems[i].m > 0 && problems[i].n > 0) order.push_back(i);
    kmax = std::max(kmax, problems[i].k);
  }
  if (leaf != BMM_LEAF_MFMA_I8 && leaf != BMM_LEAF_MFMA_F4)
    return bfail(BMM_E_UNSUPPORTED, "persistent groups run the int8 or fp4 matrix-core leaf");
  if (tile < 1 || tile > 4) return bfail(BMM_E_INVAL, "batched tile must be 1, 2, 3 or 4");
  if (leaf == BMM_LEAF_MFMA_F4 && kmax >= ((int64_t)1 << 24))
    return bfail(BMM_E_UNSUPPORTED, "the fp4 leaf counts exactly only for k < 2^24");
  if (kmax >= ((int64_t)1 << 31))
    return bfail(BMM_E_UNSUPPORTED, "the int8 leaf counts exactly only for k < 2^31");
  if (wg_per_cu <= 0) wg_per_cu = 4;
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

// Size class of a problem for per-class leaf choices (k < 1024, < 4096, else).
int k_class(int64_t k) { return k < 1024 ? 0 : (k < 4096 ? 1 : 2); }
constexpr int kKClasses = 3;

// A batched plan: the problems grouped by the leaf kind and tile chosen for each, one
// persistent launch per matrix-core group and one VALU leaf launch per VALU problem,
// enqueued in that order.  `done` orders launches of one plan (see plan_enqueue).
struct PlanSet {
  std::vector<Plan> groups;
  std::vector<std::pair<int, LeafBatch>> valu;  // (semiring, product)
  int device = 0;
  hipEvent_t done = nullptr;
};

// Choices per problem: opt's leaf and tile where given; else the autotuner's per-class
// record for plans of this count and total work, else its plan-wide record, else int8
// with the LDS-shared 128 x 64 item (tile 4).  force_* (>= 0) override everything.
int build_set(const bmm_problem* problems, int64_t count, const bmm_options* opt,
              int force_leaf, int force_tile, int force_wpc, PlanSet* out) {
  if (count < 0 || (count > 0 && !problems)) return bfail(BMM_E_INVAL, "bad problem list");
  double ops = 0;
  for (int64_t i = 0; i < count; ++i) {
    int rc = validate_problem(problems[i], i);
    if (rc != BMM_OK) return rc;
    if (!problems[i].b_transposed)
      return bfail(BMM_E_INVAL, "problem %ld: plans need B passed transposed", (long)i);
    ops += 2.0 * problems[i].m * problems[i].k * problems[i].n;
  }
  const int oleaf = opt ? opt->leaf : BMM_LEAF_AUTO;
  const int otile = opt ? opt->tile : 0;
  if (oleaf < BMM_LEAF_AUTO || oleaf > BMM_LEAF_MFMA_F4)
    return bfail(BMM_E_INVAL, "unknown leaf %d", oleaf);
  int pl = 0, pt = 0, pw = 0;
  const bool plan_rec = batched_tuned(count, ops, &pl, &pt, &pw);
  int wpc = force_wpc > 0 ? force_wpc : (plan_rec ? pw : 4);
  // (leaf, tile) -> problem indices, in table order
  std::vector<std::pair<std::pair<int, int>, std::vector<int64_t>>> groups;
  PlanSet S;
  for (int64_t i = 0; i < count; ++i) {
    const bmm_problem& p = problems[i];
    int leaf = oleaf, tile = otile, cl = 0, ct = 0;
    const bool class_rec = batched_class_tuned(count, ops, k_class(p.k), &cl, &ct);
    if (leaf == BMM_LEAF_AUTO) leaf = class_rec ? cl : (plan_rec ? pl : BMM_LEAF_MFMA_I8);
    if (tile <= 0) tile = class_rec && cl == leaf ? ct : (plan_rec && pl == leaf ? pt : 4);
    if (force_leaf > 0) leaf = force_leaf;
    if (force_tile > 0) tile = force_tile;
    if (leaf == BMM_LEAF_VALU) {
      if (p.m > 0 && p.n > 0)
        S.valu.push_back({p.semiring, LeafBatch{p.A, p.lda, 0, p.B, p.ldb, 0, p.C, p.ldc, 0,
                                                p.m, p.k, p.n, 1, 0}});
      continue;
    }
    auto it = std::find_if(groups.begin(), groups.end(),
                           [&](const auto& g) { return g.first == std::make_pair(leaf, tile); });
    if (it == groups.end()) {
      groups.push_back({{leaf, tile}, {}});
      it = groups.end() - 1;
    }
    it->second.push_back(i);
  }
  if (hipGetDevice(&S.device) != hipSuccess) return bfail(BMM_E_DEVICE, "hipGetDevice");
  for (auto& g : groups) {
    S.groups.emplace_back();
    int rc = build_plan(problems, g.second, g.first.first, g.first.second, wpc, &S.groups.back());
    if (rc != BMM_OK) {
      S.groups.pop_back();
      for (Plan& P : S.groups) plan_free(&P);
      return rc;
    }
  }
  *out = std::move(S);
  return BMM_OK;
}

// The set's kernels on s: VALU products (k = 0: C zeroed), then every persistent group.
int set_kernels(const PlanSet* S, hipStream_t s) {
  for (const auto& [sr, lb] : S->valu) {
    hipError_t e = lb.k == 0 ? launch_zero(lb.C, lb.ldc, lb.m, (lb.n + 63) / 64, s)
                             : launch_leaf_valu(sr, lb, 0, s);
    if (e != hipSuccess) return bfail(BMM_E_DEVICE, "batched VALU leaf: %s", hipGetErrorString(e));
  }
  for (const Plan& P : S->groups) {
    if (P.count == 0) continue;
    hipError_t e = launch_batched_persistent(P.descs, P.segs, P.queues, P.counters, P.grid,
                                             P.tile, P.leaf == BMM_LEAF_MFMA_F4 ? 1 : 0, s);
    if (e != hipSuccess) return bfail(BMM_E_DEVICE, "batched launch: %s", hipGetErrorString(e));
  }
  return BMM_OK;
}

// Launch a set on s.  Outside stream capture the launch is ordered after the set's
// previous one by its event (launches share the groups' queue counters).
int set_enqueue(PlanSet* S, hipStream_t s) {
  const bool cap = capturing(s);
  if (!cap) {
    if (!S->done && hipEventCreateWithFlags(&S->done, hipEventDisableTiming) != hipSuccess)
      return bfail(BMM_E_DEVICE, "plan event: %s", hipGetErrorString(hipGetLastError()));
    if (hipStreamWaitEvent(s, S->done, 0) != hipSuccess)
      return bfail(BMM_E_DEVICE, "plan order: %s", hipGetErrorString(hipGetLastError()));
  }
  BMM_BTRY(set_kernels(S, s));
  if (!cap && hipEventRecord(S->done, s) != hipSuccess)
    return bfail(BMM_E_DEVICE, "plan event: %s", hipGetErrorString(hipGetLastError()));
  return BMM_OK;
}

// Free a set once its launches have finished: the last one ordered by its event, or,
// if it was only ever launched inside stream capture, whatever the device still runs.
void set_free(PlanSet* S) {
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(S->device);
  if (S->done) {
    (void)hipEventSynchronize(S->done);
    (void)hipEventDestroy(S->done);
    S->done = nullptr;
  } else if (!S->groups.empty()) {
    (void)hipDeviceSynchronize();
  }
  for (Plan& P : S->groups) plan_free(&P);
  (void)hipSetDevice(cur);
  S->groups.clear();
  S->valu.clear();
}

// Library-owned plans of bmm_batched, keyed by the problem table (pointers, sizes,
// pitches, semirings), the leaf and tile options and the device.  An entry owns the
// device problem table, a staging buffer for right operands not given transposed,
// and a HIP graph of its launch sequence (the transposes into staging, then the plan's
// kernels: VALU products, and per persistent group the counter reset and the persistent
// kernel), captured on its first call and replayed on the caller's stream by later
// calls.  Launches of one entry are ordered by its event.
struct BatchedEntry {
  std::vector<bmm_problem> key;
  int leaf = 0, tile = 0, device = 0;
  uint64_t tune_gen = 0;  // the batched tuning records the plan was built from
  PlanSet plan;
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
    return set_kernels(&plan, s);
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
    BMM_BTRY(build_set(staged.data(), count, opt, 0, 0, 0, &plan));
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
    for (Plan& P : plan.groups) plan_free(&P);  // the entry's event covered its launches
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
  PlanSet* S = new PlanSet();
  int rc = build_set(problems, count, opt, 0, 0, 0, S);
  if (rc != BMM_OK) {
    delete S;
    return rc;
  }
  *plan_out = S;
  return BMM_OK;
}

int bmm_batched_plan_launch(void* plan, void* hip_stream) {
  if (!plan) return bfail(BMM_E_INVAL, "null plan");
  return set_enqueue(static_cast<PlanSet*>(plan), (hipStream_t)hip_stream);
}

void bmm_batched_plan_destroy(void* plan) {
  if (!plan) return;
  PlanSet* S = static_cast<PlanSet*>(plan);
  set_free(S);
  delete S;
}

}  // extern "C"

namespace {

// Seconds of one launch of the set built with these forced choices (after a warm-up),
// or a negative value when the choice does not apply (e.g. fp4 with k >= 2^24).
int time_set(const bmm_problem* problems, int64_t count, int leaf, int tile, int wpc,
             hipEvent_t e0, hipEvent_t e1, double* secs) {
  *secs = -1.0;
  PlanSet S;
  int rc = build_set(problems, count, nullptr, leaf, tile, wpc, &S);
  if (rc == BMM_E_UNSUPPORTED) return BMM_OK;
  BMM_BTRY(rc);
  rc = set_enqueue(&S, nullptr);  // warm-up
  if (rc == BMM_OK) {
    (void)hipEventRecord(e0, nullptr);
    rc = set_enqueue(&S, nullptr);
    (void)hipEventRecord(e1, nullptr);
  }
  float ms = 0.f;
  if (rc == BMM_OK && (hipEventSynchronize(e1) != hipSuccess ||
                       hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
    rc = bfail(BMM_E_DEVICE, "autotune timing: %s", hipGetErrorString(hipGetLastError()));
  set_free(&S);
  if (rc == BMM_OK) *secs = ms * 1e-3;
  return rc;
}

}  // namespace

extern "C" {

int bmm_autotune_batched(const bmm_problem* problems, int64_t count, int* leaf_out,
                         int* tile_out, double* seconds_out) {
  if (count <= 0 || !problems) return bfail(BMM_E_INVAL, "bad problem list");
  double ops = 0;
  for (int64_t i = 0; i < count; ++i) ops += 2.0 * problems[i].m * problems[i].k * problems[i].n;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return bfail(BMM_E_DEVICE, "event create");
  // 1. one leaf kind and tile for the whole plan, and the persistent grid
  double best = 1e30;
  int best_leaf = BMM_LEAF_MFMA_I8, best_tile = 4, best_wpc = 4, rc = BMM_OK;
  for (int leaf : {BMM_LEAF_MFMA_I8, BMM_LEAF_MFMA_F4})
    for (int tile : {1, 2, 3, 4})
      for (int wpc : {2, 4}) {
        double t = 0;
        if (rc == BMM_OK) rc = time_set(problems, count, leaf, tile, wpc, e0, e1, &t);
        if (rc == BMM_OK && t >= 0 && t < best) {
          best = t;
          best_leaf = leaf;
          best_tile = tile;
          best_wpc = wpc;
        }
      }
  // 2. per size class of k: every leaf kind (VALU included) and tile on that class's
  // problems alone, then the mix of the classes' choices against the single choice
  std::vector<std::pair<int, int>> cls(kKClasses, {0, 0});
  double mixed = -1.0;
  if (rc == BMM_OK) {
    std::vector<std::vector<bmm_problem>> members(kKClasses);
    for (int64_t i = 0; i < count; ++i) members[k_class(problems[i].k)].push_back(problems[i]);
    for (int c = 0; c < kKClasses && rc == BMM_OK; ++c) {
      if (members[c].empty()) continue;
      double cbest = 1e30;
      cls[c] = {best_leaf, best_tile};
      std::vector<std::pair<int, int>> cands = {{BMM_LEAF_VALU, 1}};
      for (int leaf : {BMM_LEAF_MFMA_I8, BMM_LEAF_MFMA_F4})
        for (int tile : {1, 2, 3, 4}) cands.push_back({leaf, tile});
      for (auto [leaf, tile] : cands) {
        double t = 0;
        rc = time_set(members[c].data(), (int64_t)members[c].size(), leaf, tile, best_wpc, e0,
                      e1, &t);
        if (rc != BMM_OK) break;
        if (t >= 0 && t < cbest) {
          cbest = t;
          cls[c] = {leaf, tile};
        }
      }
    }
    if (rc == BMM_OK) {
      // the mix: record the class choices, time the plan they give
      for (int c = 0; c < kKClasses; ++c)
        if (cls[c].first) batched_class_set(count, ops, c, cls[c].first, cls[c].second);
      batched_tune_set(count, ops, best_leaf, best_tile, best_wpc);
      PlanSet S;
      rc = build_set(problems, count, nullptr, 0, 0, best_wpc, &S);
      if (rc == BMM_OK) {
        rc = set_enqueue(&S, nullptr);
        if (rc == BMM_OK) {
          (void)hipEventRecord(e0, nullptr);
          rc = set_enqueue(&S, nullptr);
          (void)hipEventRecord(e1, nullptr);
        }
        float ms = 0.f;
        if (rc == BMM_OK && (hipEventSynchronize(e1) != hipSuccess ||
                             hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
          rc = bfail(BMM_E_DEVICE, "autotune timing: %s", hipGetErrorString(hipGetLastError()));
        set_free(&S);
        mixed = ms * 1e-3;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != BMM_OK) return rc;
  // keep the per-class choices only where the mix beats the single choice
  if (!(mixed > 0 && mixed < best)) {
    batched_class_clear(count, ops);
  } else {
    best = mixed;
  }
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
