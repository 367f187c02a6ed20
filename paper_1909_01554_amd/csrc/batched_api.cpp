// Batched products: plan construction (device-resident problem table sorted by
// decreasing k) and launches of the persistent kernel.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
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
};

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
  if (tile < 1 || tile > 3) return bfail(BMM_E_INVAL, "batched tile must be 1, 2 or 3");
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
    if (hipMalloc((void**)&P.descs, sizeof(BatchedDesc) * host.size()) != hipSuccess ||
        hipMalloc((void**)&P.segs, sizeof(BatchedSeg) * segs.size()) != hipSuccess ||
        hipMalloc((void**)&P.counters, cbytes) != hipSuccess) {
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
  Plan* P = static_cast<Plan*>(plan);
  if (P->count == 0) return BMM_OK;
  hipError_t e = launch_batched_persistent(
      P->descs, P->segs, P->queues, P->counters, P->grid, P->tile,
      P->leaf == BMM_LEAF_MFMA_F4 ? 1 : 0, (hipStream_t)hip_stream);
  if (e != hipSuccess) return bfail(BMM_E_DEVICE, "batched launch: %s", hipGetErrorString(e));
  return BMM_OK;
}

void bmm_batched_plan_destroy(void* plan) {
  if (!plan) return;
  Plan* P = static_cast<Plan*>(plan);
  if (P->descs || P->counters) {
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(P->device);
    (void)hipDeviceSynchronize();
    (void)hipFree(P->descs);
    (void)hipFree(P->segs);
    (void)hipFree(P->counters);
    (void)hipSetDevice(cur);
  }
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
    for (int tile : {1, 2, 3}) {
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
  hipStream_t s = (hipStream_t)hip_stream;
  // Stage non-transposed right operands into one scratch allocation.
  std::vector<bmm_problem> probs(problems, problems + count);
  size_t need = 0;
  for (int64_t i = 0; i < count; ++i) {
    int rc = validate_problem(probs[i], i);
    if (rc != BMM_OK) return rc;
    if (!probs[i].b_transposed && probs[i].m > 0 && probs[i].n > 0 && probs[i].k > 0)
      need += (size_t)probs[i].n * ((probs[i].k + 63) / 64) * 8;
  }
  uint64_t* stage = nullptr;
  if (need) {
    if (hipMalloc((void**)&stage, need) != hipSuccess) {
      (void)hipGetLastError();
      return bfail(BMM_E_NOMEM, "batched staging of %zu bytes", need);
    }
    size_t off = 0;
    for (int64_t i = 0; i < count; ++i) {
      bmm_problem& p = probs[i];
      if (p.b_transposed || p.m == 0 || p.n == 0 || p.k == 0) {
        p.b_transposed = 1;
        if (p.k == 0) p.ldb = std::max<int64_t>(p.ldb, 0);
        continue;
      }
      const int64_t kw = (p.k + 63) / 64;
      uint64_t* bt = stage + off / 8;
      hipError_t e = launch_transpose(p.B, p.ldb, 0, bt, kw, 0, p.k, p.n, 1, s);
      if (e != hipSuccess) {
        (void)hipFree(stage);
        return bfail(BMM_E_DEVICE, "transpose: %s", hipGetErrorString(e));
      }
      p.B = bt;
      p.ldb = kw;
      p.b_transposed = 1;
      off += (size_t)p.n * kw * 8;
    }
  } else {
    for (auto& p : probs) p.b_transposed = 1;
  }
  void* plan = nullptr;
  int rc = bmm_batched_plan_create(probs.data(), count, opt, &plan);
  if (rc == BMM_OK) rc = bmm_batched_plan_launch(plan, hip_stream);
  if (rc == BMM_OK && hipStreamSynchronize(s) != hipSuccess)
    rc = bfail(BMM_E_DEVICE, "batched sync: %s", hipGetErrorString(hipGetLastError()));
  bmm_batched_plan_destroy(plan);
  if (stage) {
    (void)hipStreamSynchronize(s);
    (void)hipFree(stage);
  }
  return rc;
}

}  // extern "C"
