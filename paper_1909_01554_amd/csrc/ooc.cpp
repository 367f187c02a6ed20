// Out-of-core product on one GPU (sections 3.3, 3.16 and 3.18 of the paper,
// re-planned for a single device with large HBM).
//
// A, B and C live in page-locked host memory.  C is cut into b x b blocks;
// for each block (I, K) the pipeline streams the pairs (A_IJ, B_JK) through two
// HBM slots: a copy stream uploads the next pair while the compute stream
// transposes B_JK and accumulates A_IJ * B_JK into the HBM copy of C_IK (the
// leaf's accumulate mode), and a third stream downloads finished C blocks
// while the next block is computed.  Events order the streams; the host only
// enqueues.  Each C block has one owner (the pipeline slot computing it), so no
// locks are needed, like the paper's disjoint output segments.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <vector>

#include "../../include/bmm.h"
#include "bmm_internal.h"

using namespace bmm;

namespace {

#define ofail bmm::set_error

int hip_ok(hipError_t e, const char* what) {
  if (e == hipSuccess) return BMM_OK;
  return ofail(BMM_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define OOC_TRY(expr)                \
  do {                               \
    int _rc = (expr);                \
    if (_rc != BMM_OK) return _rc;   \
  } while (0)

bool is_pinned(const void* p) {
  hipPointerAttribute_t attr;
  if (hipPointerGetAttributes(&attr, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return attr.type == hipMemoryTypeHost;
}

struct Resources {
  hipStream_t copy = nullptr, comp = nullptr, down = nullptr;
  hipEvent_t loaded[2] = {nullptr, nullptr}, used[2] = {nullptr, nullptr};
  hipEvent_t cdone[2] = {nullptr, nullptr}, cfree[2] = {nullptr, nullptr};
  uint64_t *a[2] = {nullptr, nullptr}, *b[2] = {nullptr, nullptr}, *c[2] = {nullptr, nullptr};
  uint64_t* bt = nullptr;
  void* ws = nullptr;  // alternative-basis workspace (GF(2) block products)

  ~Resources() {
    if (copy) (void)hipStreamSynchronize(copy);
    if (comp) (void)hipStreamSynchronize(comp);
    if (down) (void)hipStreamSynchronize(down);
    for (int i = 0; i < 2; ++i) {
      if (loaded[i]) (void)hipEventDestroy(loaded[i]);
      if (used[i]) (void)hipEventDestroy(used[i]);
      if (cdone[i]) (void)hipEventDestroy(cdone[i]);
      if (cfree[i]) (void)hipEventDestroy(cfree[i]);
      (void)hipFree(a[i]);
      (void)hipFree(b[i]);
      (void)hipFree(c[i]);
    }
    (void)hipFree(bt);
    (void)hipFree(ws);
    if (copy) (void)hipStreamDestroy(copy);
    if (comp) (void)hipStreamDestroy(comp);
    if (down) (void)hipStreamDestroy(down);
  }
};

}  // namespace

extern "C" int bmm_ooc(int semiring, const uint64_t* A, int64_t lda, const uint64_t* B,
                       int64_t ldb, uint64_t* C, int64_t ldc, int64_t m, int64_t k, int64_t n,
                       int64_t block, const bmm_options* opt, double* seconds_out) {
  bmm_options o;
  bmm_options_init(&o);
  if (opt) o = *opt;
  if (semiring != BMM_GF2 && semiring != BMM_BOOLEAN) return ofail(BMM_E_INVAL, "bad semiring");
  if (m < 0 || k < 0 || n < 0) return ofail(BMM_E_INVAL, "negative size");
  if (m == 0 || n == 0) return BMM_OK;
  const int64_t kw = (k + 63) / 64, nw = (n + 63) / 64;
  if (!A || !B || !C) return ofail(BMM_E_INVAL, "null host pointer");
  if (lda < kw || ldb < nw || ldc < nw) return ofail(BMM_E_INVAL, "pitch too small");
  if (!is_pinned(A) || !is_pinned(B) || !is_pinned(C))
    return ofail(BMM_E_INVAL, "host operands must be page-locked (hipHostMalloc)");
  if (block <= 0) block = o.block;
  if (block <= 0) block = (int64_t)1 << 17;
  if (block % 64) return ofail(BMM_E_INVAL, "block must be a multiple of 64 bits");
  const int64_t bm = std::min(block, m), bk = std::min(block, std::max<int64_t>(k, 64)),
                bn = std::min(block, (n + 63) / 64 * 64);
  const int64_t bkw = (bk + 63) / 64, bnw = bn / 64;

  int leaf = o.leaf == BMM_LEAF_AUTO ? BMM_LEAF_MFMA_I8 : o.leaf;
  if (leaf < BMM_LEAF_VALU || leaf > BMM_LEAF_MFMA_F4) return ofail(BMM_E_INVAL, "unknown leaf");
  if (leaf == BMM_LEAF_MFMA_F4 && std::min(block, k) >= ((int64_t)1 << 24))
    return ofail(BMM_E_UNSUPPORTED, "the fp4 leaf counts exactly only for k < 2^24");
  int tile = o.tile > 0 ? o.tile : 1;

  const auto t0 = std::chrono::steady_clock::now();
  Resources R;
  OOC_TRY(hip_ok(hipStreamCreateWithFlags(&R.copy, hipStreamNonBlocking), "stream"));
  OOC_TRY(hip_ok(hipStreamCreateWithFlags(&R.comp, hipStreamNonBlocking), "stream"));
  OOC_TRY(hip_ok(hipStreamCreateWithFlags(&R.down, hipStreamNonBlocking), "stream"));
  for (int i = 0; i < 2; ++i) {
    OOC_TRY(hip_ok(hipEventCreateWithFlags(&R.loaded[i], hipEventDisableTiming), "event"));
    OOC_TRY(hip_ok(hipEventCreateWithFlags(&R.used[i], hipEventDisableTiming), "event"));
    OOC_TRY(hip_ok(hipEventCreateWithFlags(&R.cdone[i], hipEventDisableTiming), "event"));
    OOC_TRY(hip_ok(hipEventCreateWithFlags(&R.cfree[i], hipEventDisableTiming), "event"));
    if (hipMalloc((void**)&R.a[i], (size_t)bm * bkw * 8) != hipSuccess ||
        hipMalloc((void**)&R.b[i], (size_t)bk * bnw * 8) != hipSuccess ||
        hipMalloc((void**)&R.c[i], (size_t)bm * bnw * 8) != hipSuccess) {
      (void)hipGetLastError();
      return ofail(BMM_E_NOMEM, "out-of-core HBM buffers for block %ld", (long)block);
    }
  }
  if (hipMalloc((void**)&R.bt, (size_t)bn * bkw * 8) != hipSuccess) {
    (void)hipGetLastError();
    return ofail(BMM_E_NOMEM, "out-of-core transpose buffer");
  }

  // GF(2): the alternative-basis recursion on each block product whose shape admits
  // it; the workspace is sized for the full block (smaller edge blocks need less).
  const bool cubic_only = o.depth_serial == 0 && o.depth_parallel == 0;
  size_t ws_bytes = 0;
  if (semiring == BMM_GF2 && !cubic_only) {
    int d = 0;
    bmm_options po = o;
    po.depth_serial = po.depth_parallel = -1;
    if (strassen_alt_plan(bm, bk, bn, -1, po, &ws_bytes, &d) != BMM_OK || d == 0) {
      ws_bytes = 0;
    } else if (hipMalloc(&R.ws, ws_bytes) != hipSuccess) {
      (void)hipGetLastError();
      return ofail(BMM_E_NOMEM, "out-of-core Strassen workspace (%zu bytes)", ws_bytes);
    }
  }
  // Depth of the recursion for a block product of this shape (0: cubic leaf).
  auto block_depth = [&](int64_t r, int64_t kk, int64_t c) -> int {
    if (!R.ws) return 0;
    size_t need = 0;
    int d = 0;
    bmm_options po = o;
    po.depth_serial = po.depth_parallel = -1;
    if (strassen_alt_plan(r, kk, c, -1, po, &need, &d) != BMM_OK) return 0;
    return need <= ws_bytes ? d : 0;
  };

  const int64_t nI = (m + bm - 1) / bm, nJ = (k + bk - 1) / bk, nK = (n + bn - 1) / bn;
  int64_t step = 0;    // index of the (A, B) pair being staged
  int64_t cblock = 0;  // index of the C block being computed
  for (int64_t I = 0; I < nI; ++I) {
    const int64_t rows = std::min(bm, m - I * bm);
    for (int64_t K = 0; K < nK; ++K) {
      const int64_t cols = std::min(bn, n - K * bn);
      const int64_t cwords = (cols + 63) / 64;
      const int cs = (int)(cblock & 1);
      // the C slot must have been downloaded before it is reused
      if (cblock >= 2) OOC_TRY(hip_ok(hipStreamWaitEvent(R.comp, R.cfree[cs], 0), "wait"));
      if (nJ == 0 || k == 0)
        OOC_TRY(hip_ok(launch_zero(R.c[cs], bnw, rows, cwords, R.comp), "zero"));
      int cdepth = -1;  // depth of this C block's products (all J share it), -1: unset
      for (int64_t J = 0; J < nJ; ++J) {
        const int64_t depth = std::min(bk, k - J * bk);
        const int64_t dwords = (depth + 63) / 64;
        const int s = (int)(step & 1);
        // upload the pair into slot s once its previous user has finished
        if (step >= 2) OOC_TRY(hip_ok(hipStreamWaitEvent(R.copy, R.used[s], 0), "wait"));
        OOC_TRY(hip_ok(hipMemcpy2DAsync(R.a[s], bkw * 8, A + I * bm * lda + J * (bk / 64),
                                        lda * 8, dwords * 8, rows, hipMemcpyHostToDevice,
                                        R.copy),
                       "H2D A"));
        OOC_TRY(hip_ok(hipMemcpy2DAsync(R.b[s], bnw * 8, B + J * bk * ldb + K * (bn / 64),
                                        ldb * 8, cwords * 8, depth, hipMemcpyHostToDevice,
                                        R.copy),
                       "H2D B"));
        OOC_TRY(hip_ok(hipEventRecord(R.loaded[s], R.copy), "record"));
        OOC_TRY(hip_ok(hipStreamWaitEvent(R.comp, R.loaded[s], 0), "wait"));
        OOC_TRY(hip_ok(launch_transpose(R.b[s], bnw, 0, R.bt, bkw, 0, depth, cols, 1, R.comp),
                       "transpose"));
        int d = block_depth(rows, depth, cols);
        if (cdepth < 0) cdepth = d;
        if (d != cdepth) d = 0;  // a ragged k block: cubic, in the basis the C block is in
        if (d > 0) {
          // A_IJ and B_JK^T change basis in their HBM slots; the product accumulates
          // into the alternative-basis C block
          OOC_TRY(hip_ok(launch_basis(R.a[s], bkw, 0, rows, dwords, 1, d, 0, R.comp, o.scheme, 0),
                         "basis A"));
          OOC_TRY(hip_ok(launch_basis(R.bt, bkw, 0, cols, dwords, 1, d, 0, R.comp, o.scheme, 1),
                         "basis B"));
          bmm_options po = o;
          po.depth_serial = po.depth_parallel = -1;
          po.leaf = leaf;
          po.tile = o.tile;
          OOC_TRY(strassen_alt(R.a[s], bkw, R.bt, bkw, R.c[cs], bnw, rows, depth, cols, d, R.ws,
                               ws_bytes, po, J > 0 ? 1 : 0, R.comp));
        } else {
          if (cdepth > 0) {
            // the C block is held in the alternative basis: change it to the standard
            // basis, accumulate this product, and change it back
            OOC_TRY(hip_ok(launch_basis(R.c[cs], bnw, 0, rows, cwords, 1, cdepth, 1, R.comp,
                                        o.scheme, 0),
                           "basis C"));
          }
          LeafBatch p{R.a[s], bkw, 0, R.bt, bkw, 0, R.c[cs], bnw, 0, rows, depth, cols, 1,
                      J > 0 ? 1 : 0};
          hipError_t e = leaf == BMM_LEAF_VALU ? launch_leaf_valu(semiring, p, tile - 1, R.comp)
                         : leaf == BMM_LEAF_MFMA_F4
                             ? launch_leaf_mfma_f4(semiring, p, tile - 1, R.comp)
                             : launch_leaf_mfma(semiring, p, tile - 1, R.comp);
          OOC_TRY(hip_ok(e, "leaf"));
          if (cdepth > 0)
            OOC_TRY(hip_ok(to_alt_basis(R.c[cs], bnw, rows, cwords, cdepth, o.scheme, R.comp),
                           "basis C"));
        }
        OOC_TRY(hip_ok(hipEventRecord(R.used[s], R.comp), "record"));
        ++step;
      }
      if (cdepth > 0)
        OOC_TRY(hip_ok(launch_basis(R.c[cs], bnw, 0, rows, cwords, 1, cdepth, 1, R.comp,
                                    o.scheme, 0),
                       "basis C"));
      OOC_TRY(hip_ok(hipEventRecord(R.cdone[cs], R.comp), "record"));
      OOC_TRY(hip_ok(hipStreamWaitEvent(R.down, R.cdone[cs], 0), "wait"));
      OOC_TRY(hip_ok(hipMemcpy2DAsync(C + I * bm * ldc + K * (bn / 64), ldc * 8, R.c[cs],
                                      bnw * 8, cwords * 8, rows, hipMemcpyDeviceToHost,
                                      R.down),
                     "D2H C"));
      OOC_TRY(hip_ok(hipEventRecord(R.cfree[cs], R.down), "record"));
      ++cblock;
    }
  }
  OOC_TRY(hip_ok(hipStreamSynchronize(R.comp), "sync"));
  OOC_TRY(hip_ok(hipStreamSynchronize(R.down), "sync"));
  const auto t1 = std::chrono::steady_clock::now();
  if (seconds_out) *seconds_out = std::chrono::duration<double>(t1 - t0).count();
  return BMM_OK;
}
