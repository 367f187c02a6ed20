// Out-of-core product on one GPU (sections 3.3, 3.16 and 3.18 of the paper,
// re-planned for a single device with large HBM).
//
// GF(2) with square operands of 2^dh blocks per side runs dh host levels of the
// recursion (sections 3.7 and 3.12, Algorithm 3): for each of the 7^dh
// sub-instances the GPU forms its two operands from uploaded standard-basis
// blocks (the weights of alpha.phi and beta.phi, e.g. 14 blocks of A per level
// for the self-inverse design), changes them to the device levels' basis,
// runs the recursion's core, and XORs the product into its gamma targets in an
// HBM copy of C-hat; one inverse basis change over all dh + d levels finishes
// C before a single download.  This does (7/8)^dh of the block-order work.
// Other shapes, and GF(2) with BMM_FLAG_OOC_BLOCK_ORDER, use the block order:
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
#include "scheme.h"

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

// Host <-> device copy times, per direction: HIP events on the copy's own stream
// bracket every transfer, so each rate is bytes over the copies' own durations (the
// PCIe link's rate while it moves data), not over the product's wall time.
struct CopyLog {
  struct Xfer {
    hipEvent_t e0, e1;
    double bytes;
    int d2h;
  };
  std::vector<Xfer> xs;
  int begin(hipStream_t s) {
    Xfer x{nullptr, nullptr, 0.0, 0};
    if (hipEventCreate(&x.e0) != hipSuccess || hipEventCreate(&x.e1) != hipSuccess) {
      if (x.e0) (void)hipEventDestroy(x.e0);
      return ofail(BMM_E_DEVICE, "copy timing event");
    }
    xs.push_back(x);
    return hip_ok(hipEventRecord(x.e0, s), "record");
  }
  int end(hipStream_t s, double bytes, int d2h) {
    xs.back().bytes = bytes;
    xs.back().d2h = d2h;
    return hip_ok(hipEventRecord(xs.back().e1, s), "record");
  }
  // after every copy has finished
  void totals(double* h2d_b, double* h2d_s, double* d2h_b, double* d2h_s) const {
    *h2d_b = *h2d_s = *d2h_b = *d2h_s = 0.0;
    for (const Xfer& x : xs) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, x.e0, x.e1) != hipSuccess) {
        (void)hipGetLastError();
        continue;
      }
      (x.d2h ? *d2h_b : *h2d_b) += x.bytes;
      (x.d2h ? *d2h_s : *h2d_s) += ms * 1e-3;
    }
  }
  ~CopyLog() {
    for (const Xfer& x : xs) {
      (void)hipEventDestroy(x.e0);
      if (x.e1) (void)hipEventDestroy(x.e1);
    }
  }
};

// Per-direction transfer totals of the calling thread's last bmm_ooc call.
thread_local double g_xfer[4] = {0.0, 0.0, 0.0, 0.0};

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

// Coefficient masks of one host level of a scheme: a[h] and b[h] over the
// standard quadrants (bit q, order 00 01 10 11) of A and B for operand h, and
// g[q] over the seven products for result quadrant q, from the scheme's own
// programs run on masks.
struct LevelMasks {
  uint32_t a[7], b[7], g[4];
};

template <int SCH>
LevelMasks level_masks() {
  LevelMasks L;
  uint64_t o[7];
  uint64_t x00 = 1, x01 = 2, x10 = 4, x11 = 8;
  scheme::fwd<SCH>(x00, x01, x10, x11);
  scheme::alpha<SCH>(x00, x01, x10, x11, o);
  for (int h = 0; h < 7; ++h) L.a[h] = (uint32_t)o[h];
  uint64_t y00 = 1, y01 = 2, y10 = 4, y11 = 8;
  scheme::fwd<SCH>(y00, y01, y10, y11);
  scheme::beta<SCH>(y00, y01, y10, y11, o);
  for (int h = 0; h < 7; ++h) L.b[h] = (uint32_t)o[h];
  uint64_t q[7];
  for (int h = 0; h < 7; ++h) q[h] = 1ull << h;
  uint64_t c[4];
  scheme::compress_one<SCH>(q, c[0], c[1], c[2], c[3]);
  for (int i = 0; i < 4; ++i) L.g[i] = (uint32_t)c[i];
  return L;
}

LevelMasks masks_of(int sch) {
  if (sch == BMM_SCHEME_CHAINING) return level_masks<BMM_SCHEME_CHAINING>();
  if (sch == BMM_SCHEME_WINOGRAD) return level_masks<BMM_SCHEME_WINOGRAD>();
  return level_masks<BMM_SCHEME_SELF_INVERSE>();
}

// Quadrant of block (r, c) of a 2^dh x 2^dh grid at host level l (0 = top).
inline int quad_at(int64_t r, int64_t c, int dh, int l) {
  const int sh = dh - 1 - l;
  return (int)(((r >> sh) & 1) << 1 | ((c >> sh) & 1));
}

// Digit of sub-instance h at host level l (base 7, top level most significant).
inline int digit_at(int64_t h, int dh, int l) {
  for (int i = dh - 1; i > l; --i) h /= 7;
  return (int)(h % 7);
}

struct HostRes {
  hipStream_t copy = nullptr, comb = nullptr, comp = nullptr;
  hipEvent_t loaded[2] = {}, freed[2] = {}, ready[2] = {}, done[2] = {};
  uint64_t *stage[2] = {}, *T[2] = {}, *ST[2] = {}, *btmp = nullptr, *Q = nullptr,
           *Chat = nullptr;
  void* ws = nullptr;

  ~HostRes() {
    for (hipStream_t st : {copy, comb, comp})
      if (st) (void)hipStreamSynchronize(st);
    for (int i = 0; i < 2; ++i) {
      for (hipEvent_t e : {loaded[i], freed[i], ready[i], done[i]})
        if (e) (void)hipEventDestroy(e);
      (void)hipFree(stage[i]);
      (void)hipFree(T[i]);
      (void)hipFree(ST[i]);
    }
    (void)hipFree(btmp);
    (void)hipFree(Q);
    (void)hipFree(Chat);
    (void)hipFree(ws);
    for (hipStream_t st : {copy, comb, comp})
      if (st) (void)hipStreamDestroy(st);
  }
};

// The host-level recursion; returns 1 (nothing done) when the shape or the free
// HBM does not admit it, else a bmm status.
int ooc_host_levels(const uint64_t* A, int64_t lda, const uint64_t* B, int64_t ldb,
                    uint64_t* C, int64_t ldc, int64_t n, int64_t b, const bmm_options& o,
                    int leaf, CopyLog& log) {
  if (n % b || n / b < 2 || b % 64) return 1;
  int dh = 0;
  while (((int64_t)b << dh) < n) ++dh;
  if (((int64_t)b << dh) != n) return 1;  // n / b must be a power of two
  bmm_options po = o;
  po.depth_serial = po.depth_parallel = -1;
  po.leaf = leaf;
  po.flags = 0;
  size_t ws_bytes = 0;
  int d = 0;
  if (strassen_alt_plan(b, b, b, -1, po, &ws_bytes, &d) != BMM_OK) return 1;
  const int64_t bw = b / 64, nw = n / 64;
  const size_t blk = (size_t)b * bw * 8;
  const size_t need = 8 * blk + (size_t)n * nw * 8 + ws_bytes;
  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
    (void)hipGetLastError();
    return 1;
  }
  if (need + ((size_t)1 << 30) > free_b) return 1;

  const LevelMasks L = masks_of(o.scheme);
  const int64_t g = (int64_t)1 << dh;  // blocks per side
  int64_t H = 1;
  for (int l = 0; l < dh; ++l) H *= 7;
  auto coef = [&](const uint32_t* m, int64_t h, int64_t r, int64_t c) {
    for (int l = 0; l < dh; ++l)
      if (!((m[digit_at(h, dh, l)] >> quad_at(r, c, dh, l)) & 1)) return false;
    return true;
  };
  auto coef_c = [&](int64_t h, int64_t r, int64_t c) {
    for (int l = 0; l < dh; ++l)
      if (!((L.g[quad_at(r, c, dh, l)] >> digit_at(h, dh, l)) & 1)) return false;
    return true;
  };

  HostRes R;
  for (hipStream_t* st : {&R.copy, &R.comb, &R.comp})
    OOC_TRY(hip_ok(hipStreamCreateWithFlags(st, hipStreamNonBlocking), "stream"));
  for (int i = 0; i < 2; ++i) {
    for (hipEvent_t* e : {&R.loaded[i], &R.freed[i], &R.ready[i], &R.done[i]})
      OOC_TRY(hip_ok(hipEventCreateWithFlags(e, hipEventDisableTiming), "event"));
    if (bmm::dev_malloc((void**)&R.stage[i], blk) != hipSuccess ||
        bmm::dev_malloc((void**)&R.T[i], blk) != hipSuccess ||
        bmm::dev_malloc((void**)&R.ST[i], blk) != hipSuccess) {
      (void)hipGetLastError();
      return ofail(BMM_E_NOMEM, "out-of-core host-level buffers");
    }
  }
  if (bmm::dev_malloc((void**)&R.btmp, blk) != hipSuccess || bmm::dev_malloc((void**)&R.Q, blk) != hipSuccess ||
      bmm::dev_malloc((void**)&R.Chat, (size_t)n * nw * 8) != hipSuccess ||
      (ws_bytes && bmm::dev_malloc(&R.ws, ws_bytes) != hipSuccess)) {
    (void)hipGetLastError();
    return ofail(BMM_E_NOMEM, "out-of-core host-level buffers");
  }
  OOC_TRY(hip_ok(launch_zero(R.Chat, nw, n, nw, R.comp), "zero C"));

  int64_t up = 0;  // blocks uploaded so far (staging slot up % 2)
  for (int64_t h = 0; h < H; ++h) {
    const int t = (int)(h & 1);
    if (h >= 2) OOC_TRY(hip_ok(hipStreamWaitEvent(R.comb, R.done[t], 0), "wait"));
    for (int side = 0; side < 2; ++side) {
      bool first = true;
      for (int64_t r = 0; r < g; ++r)
        for (int64_t c = 0; c < g; ++c) {
          if (!coef(side == 0 ? L.a : L.b, h, r, c)) continue;
          const int s = (int)(up & 1);
          if (up >= 2) OOC_TRY(hip_ok(hipStreamWaitEvent(R.copy, R.freed[s], 0), "wait"));
          const uint64_t* src = side == 0 ? A + r * b * lda + c * bw : B + r * b * ldb + c * bw;
          const int64_t ld = side == 0 ? lda : ldb;
          OOC_TRY(log.begin(R.copy));
          OOC_TRY(hip_ok(hipMemcpy2DAsync(R.stage[s], bw * 8, src, ld * 8, bw * 8, b,
                                          hipMemcpyHostToDevice, R.copy),
                         "H2D block"));
          OOC_TRY(log.end(R.copy, (double)blk, 0));
          OOC_TRY(hip_ok(hipEventRecord(R.loaded[s], R.copy), "record"));
          OOC_TRY(hip_ok(hipStreamWaitEvent(R.comb, R.loaded[s], 0), "wait"));
          const uint64_t* add = R.stage[s];
          uint64_t* acc = side == 0 ? R.T[t] : R.ST[t];
          if (side == 1) {  // B block (J, K) -> its transpose, stored as block (K, J) of B^T
            OOC_TRY(hip_ok(launch_transpose(R.stage[s], bw, 0, R.btmp, bw, 0, b, b, 1, R.comb),
                           "transpose"));
            add = R.btmp;
          }
          OOC_TRY(hip_ok(first ? launch_copy(add, bw, acc, bw, b, bw, R.comb)
                               : launch_xor(add, bw, acc, bw, b, bw, R.comb),
                         "combine"));
          OOC_TRY(hip_ok(hipEventRecord(R.freed[s], R.comb), "record"));
          first = false;
          ++up;
        }
      if (first) OOC_TRY(hip_ok(launch_zero(side == 0 ? R.T[t] : R.ST[t], bw, b, bw, R.comb),
                                "zero"));
    }
    OOC_TRY(hip_ok(launch_basis(R.T[t], bw, 0, b, bw, 1, d, 0, R.comb, o.scheme, 0), "basis"));
    OOC_TRY(hip_ok(launch_basis(R.ST[t], bw, 0, b, bw, 1, d, 0, R.comb, o.scheme, 1), "basis"));
    OOC_TRY(hip_ok(hipEventRecord(R.ready[t], R.comb), "record"));
    OOC_TRY(hip_ok(hipStreamWaitEvent(R.comp, R.ready[t], 0), "wait"));
    OOC_TRY(strassen_alt(R.T[t], bw, R.ST[t], bw, R.Q, bw, b, b, b, d, R.ws, ws_bytes, po, 0,
                         R.comp));
    OOC_TRY(hip_ok(hipEventRecord(R.done[t], R.comp), "record"));
    for (int64_t r = 0; r < g; ++r)
      for (int64_t c = 0; c < g; ++c)
        if (coef_c(h, r, c))
          OOC_TRY(hip_ok(launch_xor(R.Q, bw, R.Chat + r * b * nw + c * bw, nw, b, bw, R.comp),
                         "accumulate"));
  }
  OOC_TRY(hip_ok(launch_basis(R.Chat, nw, 0, n, nw, 1, dh + d, 1, R.comp, o.scheme, 0),
                 "basis C"));
  OOC_TRY(log.begin(R.comp));
  OOC_TRY(hip_ok(hipMemcpy2DAsync(C, ldc * 8, R.Chat, nw * 8, nw * 8, n, hipMemcpyDeviceToHost,
                                  R.comp),
                 "D2H C"));
  OOC_TRY(log.end(R.comp, (double)n * nw * 8, 1));
  OOC_TRY(hip_ok(hipStreamSynchronize(R.comp), "sync"));
  OOC_TRY(hip_ok(hipStreamSynchronize(R.copy), "sync"));
  return BMM_OK;
}

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
  // the cubic block products take the tile any product of their shape would take
  int tile = o.tile;
  {
    bmm_options q = o;
    q.leaf = leaf;
    int lf = leaf;
    choose_leaf(semiring, bm, bk, bn, 1, q, &lf, &tile);
  }

  const auto t0 = std::chrono::steady_clock::now();
  for (double& x : g_xfer) x = 0.0;
  CopyLog log;
  if (semiring == BMM_GF2 && !(o.flags & BMM_FLAG_OOC_BLOCK_ORDER) &&
      !(o.depth_serial == 0 && o.depth_parallel == 0) && m == k && k == n) {
    const int rc = ooc_host_levels(A, lda, B, ldb, C, ldc, n, block, o, leaf, log);
    if (rc != 1) {
      if (rc == BMM_OK) {
        if (seconds_out)
          *seconds_out =
              std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        log.totals(&g_xfer[0], &g_xfer[1], &g_xfer[2], &g_xfer[3]);
      }
      return rc;
    }
  }
  Resources R;
  OOC_TRY(hip_ok(hipStreamCreateWithFlags(&R.copy, hipStreamNonBlocking), "stream"));
  OOC_TRY(hip_ok(hipStreamCreateWithFlags(&R.comp, hipStreamNonBlocking), "stream"));
  OOC_TRY(hip_ok(hipStreamCreateWithFlags(&R.down, hipStreamNonBlocking), "stream"));
  for (int i = 0; i < 2; ++i) {
    OOC_TRY(hip_ok(hipEventCreateWithFlags(&R.loaded[i], hipEventDisableTiming), "event"));
    OOC_TRY(hip_ok(hipEventCreateWithFlags(&R.used[i], hipEventDisableTiming), "event"));
    OOC_TRY(hip_ok(hipEventCreateWithFlags(&R.cdone[i], hipEventDisableTiming), "event"));
    OOC_TRY(hip_ok(hipEventCreateWithFlags(&R.cfree[i], hipEventDisableTiming), "event"));
    if (bmm::dev_malloc((void**)&R.a[i], (size_t)bm * bkw * 8) != hipSuccess ||
        bmm::dev_malloc((void**)&R.b[i], (size_t)bk * bnw * 8) != hipSuccess ||
        bmm::dev_malloc((void**)&R.c[i], (size_t)bm * bnw * 8) != hipSuccess) {
      (void)hipGetLastError();
      return ofail(BMM_E_NOMEM, "out-of-core HBM buffers for block %ld", (long)block);
    }
  }
  if (bmm::dev_malloc((void**)&R.bt, (size_t)bn * bkw * 8) != hipSuccess) {
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
    } else if (bmm::dev_malloc(&R.ws, ws_bytes) != hipSuccess) {
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
        OOC_TRY(log.begin(R.copy));
        OOC_TRY(hip_ok(hipMemcpy2DAsync(R.a[s], bkw * 8, A + I * bm * lda + J * (bk / 64),
                                        lda * 8, dwords * 8, rows, hipMemcpyHostToDevice,
                                        R.copy),
                       "H2D A"));
        OOC_TRY(hip_ok(hipMemcpy2DAsync(R.b[s], bnw * 8, B + J * bk * ldb + K * (bn / 64),
                                        ldb * 8, cwords * 8, depth, hipMemcpyHostToDevice,
                                        R.copy),
                       "H2D B"));
        OOC_TRY(log.end(R.copy, (double)(rows * dwords + depth * cwords) * 8, 0));
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
      OOC_TRY(log.begin(R.down));
      OOC_TRY(hip_ok(hipMemcpy2DAsync(C + I * bm * ldc + K * (bn / 64), ldc * 8, R.c[cs],
                                      bnw * 8, cwords * 8, rows, hipMemcpyDeviceToHost,
                                      R.down),
                     "D2H C"));
      OOC_TRY(log.end(R.down, (double)rows * cwords * 8, 1));
      OOC_TRY(hip_ok(hipEventRecord(R.cfree[cs], R.down), "record"));
      ++cblock;
    }
  }
  OOC_TRY(hip_ok(hipStreamSynchronize(R.comp), "sync"));
  OOC_TRY(hip_ok(hipStreamSynchronize(R.down), "sync"));
  OOC_TRY(hip_ok(hipStreamSynchronize(R.copy), "sync"));
  const auto t1 = std::chrono::steady_clock::now();
  if (seconds_out) *seconds_out = std::chrono::duration<double>(t1 - t0).count();
  log.totals(&g_xfer[0], &g_xfer[1], &g_xfer[2], &g_xfer[3]);
  return BMM_OK;
}

extern "C" int bmm_ooc_last_transfers(double* h2d_bytes, double* h2d_seconds,
                                      double* d2h_bytes, double* d2h_seconds) {
  if (h2d_bytes) *h2d_bytes = g_xfer[0];
  if (h2d_seconds) *h2d_seconds = g_xfer[1];
  if (d2h_bytes) *d2h_bytes = g_xfer[2];
  if (d2h_seconds) *d2h_seconds = g_xfer[3];
  return BMM_OK;
}
