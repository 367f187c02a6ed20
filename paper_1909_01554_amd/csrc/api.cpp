// C-ABI entry points: argument checks, plans and launch sequences.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/bmm.h"
#include "bmm_internal.h"

using namespace bmm;

namespace {

thread_local std::string g_last_error;

}  // namespace

namespace bmm {

// Allocation-failure hook for tests: while positive, every library device allocation
// fails as if the device were out of memory, and the count drops by one.
std::atomic<int64_t> g_fail_allocs{0};

hipError_t dev_malloc(void** p, size_t bytes) {
  int64_t left = g_fail_allocs.load();
  while (left > 0) {
    if (g_fail_allocs.compare_exchange_weak(left, left - 1)) {
      *p = nullptr;
      return hipErrorOutOfMemory;
    }
  }
  return hipMalloc(p, bytes);
}

int set_error(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}
}  // namespace bmm

namespace {

#define fail bmm::set_error

int check_hip(hipError_t e, const char* what) {
  if (e == hipSuccess) return BMM_OK;
  if (e == kGridTooLarge)
    return fail(BMM_E_UNSUPPORTED, "%s: the launch would need 2^32 or more work-items "
                "(split the product into smaller blocks)", what);
  return fail(BMM_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define BMM_TRY(expr)                 \
  do {                                \
    int _rc = (expr);                 \
    if (_rc != BMM_OK) return _rc;    \
  } while (0)

#define HIP_TRY(expr, what) BMM_TRY(check_hip((expr), (what)))

inline int64_t words_of(int64_t bits) { return (bits + 63) / 64; }

struct Extent {
  uintptr_t lo, hi;
};

Extent extent(const void* p, int64_t rows, int64_t ld, int64_t row_words) {
  const uintptr_t lo = reinterpret_cast<uintptr_t>(p);
  if (rows <= 0 || row_words <= 0) return {lo, lo};
  return {lo, lo + (uintptr_t)(((rows - 1) * ld + row_words) * 8)};
}

bool overlaps(Extent a, Extent b) { return a.lo < b.hi && b.lo < a.hi; }

bmm_options defaults() {
  bmm_options o;
  bmm_options_init(&o);
  return o;
}

// ---- library-owned scratch (per device), used for B^T in the cubic calls ----
std::mutex g_mu;
std::map<int, std::pair<void*, size_t>> g_scratch;

int scratch(size_t bytes, void** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
  std::lock_guard<std::mutex> lock(g_mu);
  auto& slot = g_scratch[dev];
  if (slot.second < bytes) {
    if (slot.first) {
      // earlier work may still read the old buffer
      HIP_TRY(hipDeviceSynchronize(), "hipDeviceSynchronize");
      HIP_TRY(hipFree(slot.first), "hipFree");
      slot = {nullptr, 0};
    }
    size_t want = std::max(bytes, (size_t)1 << 20);
    void* p = nullptr;
    if (dev_malloc(&p, want) != hipSuccess || !p) {
      (void)hipGetLastError();
      return fail(BMM_E_NOMEM, "scratch allocation of %zu bytes failed", want);
    }
    slot = {p, want};
  }
  *out = slot.first;
  return BMM_OK;
}

// ---- autotune table ----
// Keyed by semiring, leaf shape and batch bucket (1, 2, 4, ..., 64 = "64 or more").
struct TuneKey {
  int semiring;
  int64_t m, k, n, batch;
  bool operator<(const TuneKey& o) const {
    return std::tie(semiring, m, k, n, batch) < std::tie(o.semiring, o.m, o.k, o.n, o.batch);
  }
};
// Per key: the fastest leaf kind and the fastest tile of every leaf kind (0 = unknown).
struct TuneVal {
  int best_leaf = 0;
  int tile[4] = {0, 0, 0, 0};
};
std::map<TuneKey, TuneVal> g_tune;
// Strassen (depth, serial depth, shifted leaf level) per shape, from bmm_autotune_strassen.
std::map<std::tuple<int64_t, int64_t, int64_t>, std::tuple<int, int, int>> g_depth;
// Cubic k-panel schedule per (semiring, m, k, n): panel length in bits, from
// bmm_autotune_k_panel.
std::map<std::tuple<int, int64_t, int64_t, int64_t>, int64_t> g_kpanel;
// Batched plans: (problem count, floor(log2(total ops))) -> (leaf, tile, workgroups per CU).
std::map<std::pair<int64_t, int>, std::tuple<int, int, int>> g_batched;
// Per size class of k within such plans: (count, floor(log2(total ops)), class) ->
// (leaf, tile), where the autotuner found a mix of choices faster than one choice.
std::map<std::tuple<int64_t, int, int>, std::pair<int, int>> g_bclass;
// Bumped whenever g_batched or g_bclass changes, so cached batched plans built from older
// records are rebuilt.
std::atomic<uint64_t> g_batched_gen{0};

int ops_bucket(double ops) {
  int b = 0;
  while (ops >= 2.0 && b < 200) {
    ops *= 0.5;
    ++b;
  }
  return b;
}

int64_t batch_bucket(int64_t b) {
  int64_t q = 1;
  while (q < b && q < 64) q <<= 1;
  return q;
}

void pick_leaf(int semiring, int64_t m, int64_t k, int64_t n, int64_t batch,
               const bmm_options& o, int* leaf, int* tile) {
  *leaf = o.leaf;
  *tile = o.tile;
  if (*leaf == BMM_LEAF_AUTO || *tile <= 0) {
    std::lock_guard<std::mutex> lock(g_mu);
    auto it = g_tune.find({semiring, m, k, n, batch_bucket(batch)});
    if (it != g_tune.end()) {
      if (*leaf == BMM_LEAF_AUTO && it->second.best_leaf > 0) *leaf = it->second.best_leaf;
      if (*tile <= 0 && *leaf >= 1 && *leaf <= 3) *tile = it->second.tile[*leaf];
    }
  }
  if (*leaf == BMM_LEAF_AUTO) *leaf = BMM_LEAF_MFMA_I8;
  if (*tile <= 0) {
    // default MFMA tile for shapes the table lacks, from the gfx950 timings: when 128 x 64
    // wave tiles give fewer than 16 waves per CU over the whole launch, 64 x 64 tiles fill
    // the chip better; long k runs int8 on 64 x 128 wave tiles in the chunked loop (tile 7)
    // and fp4 LDS-staged (tile 5); everything else 128 x 64 per wave
    const int64_t waves = batch * ((m + 127) / 128) * ((n + 63) / 64);
    if (*leaf != BMM_LEAF_VALU && waves < 4096) *tile = 2;
    else if (*leaf == BMM_LEAF_MFMA_I8 && k >= 8192) *tile = 7;
    else if (*leaf == BMM_LEAF_MFMA_F4 && k >= 4096) *tile = 5;
    else *tile = 1;
  }
}

int run_leaf(int semiring, int leaf, int tile, const LeafBatch& p, hipStream_t s) {
  hipError_t e;
  if (leaf == BMM_LEAF_VALU) {
    e = launch_leaf_valu(semiring, p, tile - 1, s);
  } else if (leaf == BMM_LEAF_MFMA_I8) {
    if (p.k >= ((int64_t)1 << 31))
      return fail(BMM_E_UNSUPPORTED, "the int8 leaf counts exactly only for k < 2^31");
    e = launch_leaf_mfma(semiring, p, tile - 1, s);
  } else if (leaf == BMM_LEAF_MFMA_F4) {
    if (p.k >= ((int64_t)1 << 24))
      return fail(BMM_E_UNSUPPORTED, "the fp4 leaf counts exactly only for k < 2^24");
    e = launch_leaf_mfma_f4(semiring, p, tile - 1, s);
  } else {
    return fail(BMM_E_INVAL, "unknown leaf %d", leaf);
  }
  return check_hip(e, "leaf launch");
}

int validate_product(const uint64_t* A, int64_t lda, const uint64_t* B, int64_t ldb,
                     const uint64_t* C, int64_t ldc, int64_t m, int64_t k, int64_t n,
                     bool b_t) {
  if (m < 0 || k < 0 || n < 0) return fail(BMM_E_INVAL, "negative size (m=%ld k=%ld n=%ld)", (long)m, (long)k, (long)n);
  if (m == 0 || n == 0) return BMM_OK;
  const int64_t kw = words_of(k), nw = words_of(n);
  if (!C) return fail(BMM_E_INVAL, "C is null");
  if (ldc < nw) return fail(BMM_E_INVAL, "ldc=%ld < %ld words", (long)ldc, (long)nw);
  if ((reinterpret_cast<uintptr_t>(C) & 7) != 0) return fail(BMM_E_INVAL, "C not 8-byte aligned");
  if (k == 0) return BMM_OK;
  if (!A || !B) return fail(BMM_E_INVAL, "A or B is null");
  if (((reinterpret_cast<uintptr_t>(A) | reinterpret_cast<uintptr_t>(B)) & 7) != 0)
    return fail(BMM_E_INVAL, "A or B not 8-byte aligned");
  if (lda < kw) return fail(BMM_E_INVAL, "lda=%ld < %ld words", (long)lda, (long)kw);
  if (b_t ? ldb < kw : ldb < nw) return fail(BMM_E_INVAL, "ldb=%ld too small", (long)ldb);
  const Extent ec = extent(C, m, ldc, nw);
  if (overlaps(ec, extent(A, m, lda, kw))) return fail(BMM_E_INVAL, "C overlaps A");
  if (overlaps(ec, b_t ? extent(B, n, ldb, kw) : extent(B, k, ldb, nw)))
    return fail(BMM_E_INVAL, "C overlaps B");
  return BMM_OK;
}

}  // namespace

namespace bmm {

// Panel length (bits) of a cubic product's k: the options' own (rounded up to whole
// words; negative = one panel), else the k-panel table's record, else one panel.
int64_t k_panel_bits(int semiring, int64_t m, int64_t k, int64_t n, const bmm_options& o) {
  int64_t bits = 0;
  if (o.k_panel > 0) {
    bits = (o.k_panel + 63) / 64 * 64;
  } else if (o.k_panel == 0) {
    std::lock_guard<std::mutex> lock(g_mu);
    auto it = g_kpanel.find({semiring, m, k, n});
    if (it != g_kpanel.end()) bits = it->second;
  }
  return bits > 0 && bits < k ? bits : std::max<int64_t>(k, 1);
}

int cubic_product(int semiring, const uint64_t* A, int64_t lda, const uint64_t* B, int64_t ldb,
                  uint64_t* C, int64_t ldc, int64_t m, int64_t k, int64_t n,
                  const bmm_options* opt, void* stream, const BtScratch* caller_bt) {
  const bmm_options o = opt ? *opt : defaults();
  const bool b_t = (o.flags & BMM_FLAG_B_TRANSPOSED) != 0;
  BMM_TRY(validate_product(A, lda, B, ldb, C, ldc, m, k, n, b_t));
  if (m == 0 || n == 0) return BMM_OK;
  const bool acc = (o.flags & BMM_FLAG_ACCUMULATE) != 0;
  hipStream_t s = (hipStream_t)stream;
  if (k == 0) {
    if (!acc) HIP_TRY(launch_zero(C, ldc, m, words_of(n), s), "zero");
    return BMM_OK;
  }
  int leaf, tile;
  pick_leaf(semiring, m, k, n, 1, o, &leaf, &tile);
  // The VALU leaf's outer-product form (tile 2) reads B row-major; every other leaf reads
  // B^T. Whichever form the leaf needs and the caller did not pass is staged in scratch.
  const bool outer = leaf == BMM_LEAF_VALU && tile == 2;
  const int64_t kw = words_of(k), nw = words_of(n);
  const bool stage = outer ? b_t : !b_t;
  const size_t stage_bytes = outer ? (size_t)k * nw * 8 : (size_t)n * kw * 8;
  if (caller_bt && stage && stage_bytes > caller_bt->bytes)
    return fail(BMM_E_UNSUPPORTED,
                "staging B for this leaf needs %zu bytes of scratch and this entry point has "
                "%zu: pass B in the form the leaf reads (B^T for the MFMA leaves and VALU tile "
                "1, B for VALU tile 2) or call bmm_gf2 / bmm_boolean",
                stage_bytes, caller_bt->bytes);
  const uint64_t* Bl = B;  // B^T, or B for the outer-product form
  int64_t ldl = ldb;
  if (stage) {
    void* buf = nullptr;
    if (caller_bt) BMM_TRY(caller_bt->get(&buf));
    else BMM_TRY(scratch(stage_bytes, &buf));
    if (outer)  // B^T (n x k) -> B (k x n)
      HIP_TRY(launch_transpose(B, ldb, 0, (uint64_t*)buf, nw, 0, n, k, 1, s), "transpose");
    else        // B (k x n) -> B^T (n x k)
      HIP_TRY(launch_transpose(B, ldb, 0, (uint64_t*)buf, kw, 0, k, n, 1, s), "transpose");
    Bl = (const uint64_t*)buf;
    ldl = outer ? nw : kw;
  }
  // k in panels: C = sum over panels of A[:, panel] B[panel, :], each panel's product
  // added into C (XOR or OR) after the first; the leaf and tile are the full shape's
  const int64_t panel = k_panel_bits(semiring, m, k, n, o);
  for (int64_t p0 = 0; p0 < k; p0 += panel) {
    const int64_t kp = std::min(panel, k - p0);
    const int pacc = (acc || p0 > 0) ? 1 : 0;
    if (outer) {
      HIP_TRY(launch_leaf_valu_outer(semiring, A + p0 / 64, lda, Bl + p0 * ldl, ldl, C, ldc, m,
                                     kp, n, pacc, s),
              "leaf launch");
    } else {
      LeafBatch p{A + p0 / 64, lda, 0, Bl + p0 / 64, ldl, 0, C, ldc, 0, m, kp, n, 1, pacc};
      BMM_TRY(run_leaf(semiring, leaf, tile, p, s));
    }
  }
  return BMM_OK;
}

}  // namespace bmm

namespace {

// Host-resident operands (BMM_FLAG_HOST_OPERANDS) go through the out-of-core
// pipeline, synchronously: earlier work on the caller's stream finishes first (it may
// produce A or B), and C is complete on return.  cubic = 1 keeps the cubic method
// for GF(2) (block order, no recursion levels).
int host_product(int semiring, const uint64_t* A, int64_t lda, const uint64_t* B,
                 int64_t ldb, uint64_t* C, int64_t ldc, int64_t m, int64_t k, int64_t n,
                 bmm_options o, void* stream, bool cubic) {
  if (o.flags & (BMM_FLAG_ACCUMULATE | BMM_FLAG_B_TRANSPOSED | BMM_FLAG_ALT_BASIS_IO))
    return fail(BMM_E_UNSUPPORTED, "host operands: accumulation, B passed transposed and "
                "alternative-basis input are not supported out of core");
  if (cubic) {
    o.flags |= BMM_FLAG_OOC_BLOCK_ORDER;
    o.depth_serial = o.depth_parallel = 0;
  }
  HIP_TRY(hipStreamSynchronize((hipStream_t)stream), "hipStreamSynchronize");
  return bmm_ooc(semiring, A, lda, B, ldb, C, ldc, m, k, n, o.block, &o, nullptr);
}

int cubic(int semiring, const uint64_t* A, int64_t lda, const uint64_t* B, int64_t ldb,
          uint64_t* C, int64_t ldc, int64_t m, int64_t k, int64_t n, const bmm_options* opt,
          void* stream) {
  const bmm_options o = opt ? *opt : defaults();
  if (o.flags & BMM_FLAG_HOST_OPERANDS)
    return host_product(semiring, A, lda, B, ldb, C, ldc, m, k, n, o, stream, true);
  return cubic_product(semiring, A, lda, B, ldb, C, ldc, m, k, n, opt, stream, nullptr);
}

// ---- Strassen plan ----
struct Level {
  size_t T, S, Q;  // byte offsets in the workspace
};

struct StrassenPlan {
  int depth = 0, ds = 0, dp = 0;
  int shift = 0;  // 0: plain leaf; 1, 2: last parallel level inside the int8 leaf
                  // (2: with 8-byte operand loads)
  bool lean = false;  // depth-first levels hold one child at a time
  int scheme = BMM_SCHEME_SELF_INVERSE;
  int64_t m = 0, kw = 0, n = 0, nw = 0;
  size_t ahat = 0, bhat = 0;
  std::vector<Level> serial;         // levels 1..ds (index l-1)
  std::vector<int> psteps;           // parallel step sizes (1 or 2 levels)
  std::vector<Level> par;            // buffers after each parallel step
  size_t bytes = 0;
};

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

// Whether (depth, ds) is the depth tuner's record for this shape (its shift choice
// belongs to that split only).
bool depth_is_tuned(int64_t m, int64_t k, int64_t n, int depth, int ds) {
  std::lock_guard<std::mutex> lock(g_mu);
  auto it = g_depth.find({m, k, n});
  return it != g_depth.end() && std::get<0>(it->second) == depth &&
         std::get<1>(it->second) == ds;
}

// Which operands the product stages in its workspace: a copy of A unless A is
// read where it lies (already in the alternative basis, or changed in place and
// restored); B^T unless B is passed transposed and read where it lies.
struct Staging {
  bool a, b;
};
Staging staging_of(const bmm_options& o) {
  const bool alt = (o.flags & BMM_FLAG_ALT_BASIS_IO) != 0;
  const bool inplace = (o.flags & BMM_FLAG_INPLACE_BASIS) != 0;
  const bool b_t = (o.flags & BMM_FLAG_B_TRANSPOSED) != 0;
  return Staging{!alt && !inplace, !b_t || (!alt && !inplace)};
}

// stage_a / stage_b: plan room for a copy of A / for B^T (see Staging).
int make_plan(int64_t m, int64_t k, int64_t n, int depth, const bmm_options& o, bool stage_a,
              StrassenPlan* plan, bool stage_b = true) {
  if (m < 0 || k < 0 || n < 0) return fail(BMM_E_INVAL, "negative size");
  if (depth < -1 || depth > 12) return fail(BMM_E_INVAL, "depth %d out of range", depth);
  if (o.scheme < BMM_SCHEME_SELF_INVERSE || o.scheme > BMM_SCHEME_WINOGRAD)
    return fail(BMM_E_INVAL, "unknown scheme %d", o.scheme);
  StrassenPlan P;
  P.scheme = o.scheme;
  P.m = m;
  P.kw = words_of(k);
  P.n = n;
  P.nw = words_of(n);
  int tuned_ds = -1, tuned_shift = 0;
  if (depth == -1) {
    std::lock_guard<std::mutex> lock(g_mu);
    auto it = g_depth.find({m, k, n});
    if (it != g_depth.end()) std::tie(depth, tuned_ds, tuned_shift) = it->second;
  }
  if (depth == -1) {
    // largest depth keeping every leaf dimension >= 2048 bits (at most 8 levels): the
    // depth tuner's optimum at n = 2^18 on gfx950 has 2048-bit leaves
    depth = 0;
    while (depth < 8) {
      const int d = depth + 1;
      const int64_t u = (int64_t)1 << d;
      if (m % u || k % (64 * u) || n % (64 * u)) break;
      if (m / u < 2048 || k / u < 2048 || n / u < 2048) break;
      depth = d;
    }
  }
  const int64_t u = (int64_t)1 << depth;
  if (m % u || k % (64 * u) || n % (64 * u))
    return fail(BMM_E_UNSUPPORTED,
                "Strassen depth %d needs m %% 2^d == 0 and k, n %% (64 * 2^d) == 0", depth);
  P.depth = depth;
  int dp = o.depth_parallel, ds = o.depth_serial;
  if (dp < 0 && ds < 0 && tuned_ds >= 0 && tuned_ds <= depth) {
    ds = tuned_ds;
    dp = depth - ds;
  } else if (dp < 0 && ds < 0) {
    dp = std::min(depth, 4);
    ds = depth - dp;
  } else if (dp < 0) {
    ds = std::min(ds, depth);
    dp = depth - ds;
  } else if (ds < 0) {
    dp = std::min(dp, depth);
    ds = depth - dp;
  }
  if (ds + dp != depth || ds < 0 || dp < 0)
    return fail(BMM_E_INVAL, "depth_serial %d + depth_parallel %d != depth %d", ds, dp, depth);
  P.ds = ds;
  P.dp = dp;
  // the shifted leaf level: the option, else the tuned choice for this shape (with the
  // tuned depth split only), else off; it needs a parallel level, the int8 leaf and a
  // leaf shape the kernel covers, else the plain leaf runs
  if (o.shift < -1 || o.shift > 2) return fail(BMM_E_INVAL, "shift %d out of range", o.shift);
  int sh = o.shift >= 0 ? o.shift : (depth_is_tuned(m, k, n, depth, ds) ? tuned_shift : 0);
  if (sh > 0) {
    const int64_t u = (int64_t)1 << depth;
    int lf = 0, tl = 0;
    int64_t leaves = 1;
    for (int i = 0; i < dp; ++i) leaves *= 7;
    pick_leaf(BMM_GF2, m / u, k / u, n / u, leaves, o, &lf, &tl);
    if (dp < 1 || lf != BMM_LEAF_MFMA_I8 || !leaf_shift_supported(o.scheme, m / u, k / u, n / u))
      sh = 0;
  }
  P.shift = sh;
  size_t off = 0;
  if (stage_a) {
    P.ahat = off;
    off = align_up(off + (size_t)m * P.kw * 8);
  }
  if (stage_b) {
    P.bhat = off;
    off = align_up(off + (size_t)n * P.kw * 8);
  }
  // depth-first levels: all seven children of T, S and Q, or (lean) one of each
  P.lean = (o.flags & BMM_FLAG_LEAN_WORKSPACE) != 0;
  const size_t per = P.lean ? 1 : 7;
  for (int l = 1; l <= ds; ++l) {
    const int64_t M = m >> l, KW = P.kw >> l, N = n >> l, NW = P.nw >> l;
    Level L;
    L.T = off;
    off = align_up(off + per * M * KW * 8);
    L.S = off;
    off = align_up(off + per * N * KW * 8);
    L.Q = off;
    off = align_up(off + per * M * NW * 8);
    P.serial.push_back(L);
  }
  int left = dp - (P.shift ? 1 : 0), lvl = ds;  // levels expanded in HBM
  int64_t inst = 1;
  while (left > 0) {
    const int step = left >= 2 ? 2 : 1;
    lvl += step;
    left -= step;
    inst *= step == 2 ? 49 : 7;
    const int64_t M = m >> lvl, KW = P.kw >> lvl, N = n >> lvl, NW = P.nw >> lvl;
    Level L;
    L.T = off;
    off = align_up(off + (size_t)inst * M * KW * 8);
    L.S = off;
    off = align_up(off + (size_t)inst * N * KW * 8);
    L.Q = off;
    off = align_up(off + (size_t)inst * M * NW * 8);
    P.psteps.push_back(step);
    P.par.push_back(L);
  }
  P.bytes = std::max(off, (size_t)256);
  *plan = P;
  return BMM_OK;
}

struct StrassenRun {
  const StrassenPlan* P;
  char* ws;
  int leaf, tile;
  hipStream_t s;

  uint64_t* at(size_t off) const { return reinterpret_cast<uint64_t*>(ws + off); }

  // acc = 1: the result is XORed into Q (only ever set for the top-level output).
  int parallel(int level, const uint64_t* T, int64_t ldT, const uint64_t* S, int64_t ldS,
               uint64_t* Q, int64_t ldQ, int acc) const {
    const StrassenPlan& p = *P;
    const uint64_t* curT = T;
    const uint64_t* curS = S;
    int64_t pitchT = ldT, pitchS = ldS, strideT = 0, strideS = 0;
    int64_t inst = 1;
    int lvl = level;
    for (size_t i = 0; i < p.psteps.size(); ++i) {
      const int step = p.psteps[i];
      const int64_t M = p.m >> lvl, KW = p.kw >> lvl, N = p.n >> lvl;
      const Level& L = p.par[i];
      if (step == 2) {
        HIP_TRY(launch_expand2(0, curT, pitchT, strideT, at(L.T), M, KW, inst, s, p.scheme),
                "expand2 T");
        HIP_TRY(launch_expand2(1, curS, pitchS, strideS, at(L.S), N, KW, inst, s, p.scheme),
                "expand2 S");
      } else {
        HIP_TRY(launch_expand(0, curT, pitchT, strideT, at(L.T), M, KW, inst, s, p.scheme),
                "expand T");
        HIP_TRY(launch_expand(1, curS, pitchS, strideS, at(L.S), N, KW, inst, s, p.scheme),
                "expand S");
      }
      lvl += step;
      inst *= step == 2 ? 49 : 7;
      curT = at(L.T);
      curS = at(L.S);
      pitchT = pitchS = p.kw >> lvl;
      strideT = (p.m >> lvl) * pitchT;
      strideS = (p.n >> lvl) * pitchS;
    }
    // leaf products of all instances at the bottom level
    const int64_t M = p.m >> lvl, N = p.n >> lvl, NW = p.nw >> lvl;
    uint64_t* leafQ = p.par.empty() ? Q : at(p.par.back().Q);
    const int64_t ldLQ = p.par.empty() ? ldQ : NW;
    if (p.shift) {
      // the last level inside the leaf: the instances at this level are the parents
      // of the seven products each, their results this level's Q
      const int64_t cM = M >> 1, cN = N >> 1, cK = ((p.kw >> lvl) >> 1) * 64;
      if (!leaf_shift_fits(cM, pitchT) || !leaf_shift_fits(cN, pitchS))
        return fail(BMM_E_UNSUPPORTED, "shifted leaf: operand pitches too large");
      ShiftBatch sb{curT, pitchT, strideT, curS, pitchS, strideS, leafQ, ldLQ, M * NW,
                    cM, cK, cN, inst, p.par.empty() ? acc : 0};
      HIP_TRY(launch_leaf_shift(p.scheme, sb, p.shift == 2 ? 1 : 2, s), "shifted leaf");
    } else {
      LeafBatch lb{curT, pitchT, strideT, curS, pitchS, strideS, leafQ, ldLQ, M * NW,
                   M, (p.kw >> lvl) * 64, N, inst, p.par.empty() ? acc : 0};
      BMM_TRY(run_leaf(BMM_GF2, leaf, tile, lb, s));
    }
    // compress back up
    for (int i = (int)p.psteps.size() - 1; i >= 0; --i) {
      const int step = p.psteps[i];
      inst /= step == 2 ? 49 : 7;
      lvl -= step;
      const uint64_t* src = at(p.par[i].Q);
      uint64_t* dst;
      int64_t ldd, strideD;
      if (i == 0) {
        dst = Q;
        ldd = ldQ;
        strideD = 0;
      } else {
        dst = at(p.par[i - 1].Q);
        ldd = p.nw >> lvl;
        strideD = (p.m >> lvl) * ldd;
      }
      const int64_t M2 = p.m >> lvl, NW2 = p.nw >> lvl;
      const int a = i == 0 ? acc : 0;
      if (step == 2)
        HIP_TRY(launch_compress2(src, dst, ldd, strideD, M2, NW2, inst, s, a, p.scheme),
                "compress2");
      else
        HIP_TRY(launch_compress(src, dst, ldd, strideD, M2, NW2, inst, s, a, p.scheme),
                "compress");
    }
    return BMM_OK;
  }

  int solve(int level, const uint64_t* T, int64_t ldT, const uint64_t* S, int64_t ldS,
            uint64_t* Q, int64_t ldQ, int acc) const {
    const StrassenPlan& p = *P;
    if (level >= p.ds) return parallel(level, T, ldT, S, ldS, Q, ldQ, acc);
    const int64_t M = p.m >> level, KW = p.kw >> level, N = p.n >> level, NW = p.nw >> level;
    const Level& L = p.serial[level];
    if (p.lean) {
      // one child at a time: T_h and S_h from the parent quadrants alpha (beta) selects,
      // the product, then gamma adds it into the parent's result quadrants
      for (int h = 0; h < 7; ++h) {
        HIP_TRY(launch_child(p.scheme, 0, h, T, ldT, at(L.T), KW / 2, M, KW, s), "child T");
        HIP_TRY(launch_child(p.scheme, 1, h, S, ldS, at(L.S), KW / 2, N, KW, s), "child S");
        BMM_TRY(solve(level + 1, at(L.T), KW / 2, at(L.S), KW / 2, at(L.Q), NW / 2, 0));
        HIP_TRY(launch_gamma(p.scheme, h, at(L.Q), NW / 2, Q, ldQ, M, NW, acc, s), "gamma");
      }
      return BMM_OK;
    }
    HIP_TRY(launch_expand(0, T, ldT, 0, at(L.T), M, KW, 1, s, p.scheme), "serial expand T");
    HIP_TRY(launch_expand(1, S, ldS, 0, at(L.S), N, KW, 1, s, p.scheme), "serial expand S");
    const int64_t cT = (M / 2) * (KW / 2), cS = (N / 2) * (KW / 2), cQ = (M / 2) * (NW / 2);
    for (int h = 0; h < 7; ++h)
      BMM_TRY(solve(level + 1, at(L.T) + h * cT, KW / 2, at(L.S) + h * cS, KW / 2,
                    at(L.Q) + h * cQ, NW / 2, 0));
    HIP_TRY(launch_compress(at(L.Q), Q, ldQ, 0, M, NW, 1, s, acc, p.scheme), "serial compress");
    return BMM_OK;
  }
};

}  // namespace

extern "C" {

void bmm_options_init(bmm_options* opt) {
  if (!opt) return;
  opt->leaf = BMM_LEAF_AUTO;
  opt->tile = 0;
  opt->depth_serial = -1;
  opt->depth_parallel = -1;
  opt->block = 0;
  opt->flags = 0;
  opt->scheme = BMM_SCHEME_SELF_INVERSE;
  opt->shift = -1;
  opt->k_panel = 0;
}

int bmm_gf2(const uint64_t* A, int64_t lda, const uint64_t* B, int64_t ldb, uint64_t* C,
            int64_t ldc, int64_t m, int64_t k, int64_t n, const bmm_options* opt,
            void* hip_stream) {
  return cubic(BMM_GF2, A, lda, B, ldb, C, ldc, m, k, n, opt, hip_stream);
}

int bmm_boolean(const uint64_t* A, int64_t lda, const uint64_t* B, int64_t ldb, uint64_t* C,
                int64_t ldc, int64_t m, int64_t k, int64_t n, const bmm_options* opt,
                void* hip_stream) {
  return cubic(BMM_BOOLEAN, A, lda, B, ldb, C, ldc, m, k, n, opt, hip_stream);
}

int bmm_gf2_strassen_workspace(int64_t m, int64_t k, int64_t n, int depth,
                               const bmm_options* opt, size_t* bytes_out,
                               int* depth_serial_out, int* depth_parallel_out) {
  const bmm_options o = opt ? *opt : defaults();
  StrassenPlan P;
  const Staging st = staging_of(o);
  BMM_TRY(make_plan(m, k, n, depth, o, st.a, &P, st.b));
  if (bytes_out) *bytes_out = P.bytes;
  if (depth_serial_out) *depth_serial_out = P.ds;
  if (depth_parallel_out) *depth_parallel_out = P.dp;
  return BMM_OK;
}

int bmm_gf2_strassen(const uint64_t* A, int64_t lda, const uint64_t* B, int64_t ldb,
                     uint64_t* C, int64_t ldc, int64_t m, int64_t k, int64_t n, int depth,
                     void* workspace, size_t workspace_bytes, const bmm_options* opt,
                     void* hip_stream) {
  const bmm_options o = opt ? *opt : defaults();
  if (o.flags & BMM_FLAG_HOST_OPERANDS)
    return host_product(BMM_GF2, A, lda, B, ldb, C, ldc, m, k, n, o, hip_stream, false);
  const bool b_t = (o.flags & BMM_FLAG_B_TRANSPOSED) != 0;
  const bool alt = (o.flags & BMM_FLAG_ALT_BASIS_IO) != 0;
  const bool inplace = !alt && (o.flags & BMM_FLAG_INPLACE_BASIS) != 0;
  const int acc = (o.flags & BMM_FLAG_ACCUMULATE) ? 1 : 0;
  BMM_TRY(validate_product(A, lda, B, ldb, C, ldc, m, k, n, b_t));
  const Staging st = staging_of(o);
  StrassenPlan P;
  BMM_TRY(make_plan(m, k, n, depth, o, st.a, &P, st.b));
  if (m == 0 || n == 0) return BMM_OK;
  if (inplace && k > 0 &&
      overlaps(extent(A, m, lda, P.kw), b_t ? extent(B, n, ldb, P.kw) : extent(B, k, ldb, P.nw)))
    return fail(BMM_E_INVAL, "in-place basis changes need A and B not to overlap");
  hipStream_t s = (hipStream_t)hip_stream;
  if (k == 0) return acc ? BMM_OK : check_hip(launch_zero(C, ldc, m, P.nw, s), "zero");
  if (!workspace || workspace_bytes < P.bytes)
    return fail(BMM_E_WORKSPACE, "workspace of %zu bytes needed, %zu given", P.bytes,
                workspace_bytes);
  if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0)
    return fail(BMM_E_INVAL, "workspace must be 256-byte aligned");
  const Extent ew{reinterpret_cast<uintptr_t>(workspace),
                  reinterpret_cast<uintptr_t>(workspace) + P.bytes};
  if (overlaps(ew, extent(C, m, ldc, P.nw)) || overlaps(ew, extent(A, m, lda, P.kw)) ||
      overlaps(ew, b_t ? extent(B, n, ldb, P.kw) : extent(B, k, ldb, P.nw)))
    return fail(BMM_E_INVAL, "workspace overlaps an operand");
  char* ws = static_cast<char*>(workspace);
  // B^T: staged in the workspace (transposed, or copied when it will be changed), or
  // read where it lies (alternative-basis input, or changed in place)
  uint64_t* BT = const_cast<uint64_t*>(B);
  int64_t ldbt = ldb;
  if (st.b) {
    BT = reinterpret_cast<uint64_t*>(ws + P.bhat);
    ldbt = P.kw;
    if (b_t)
      HIP_TRY(launch_copy(B, ldb, BT, P.kw, n, P.kw, s), "copy B^T");
    else
      HIP_TRY(launch_transpose(B, ldb, 0, BT, P.kw, 0, k, n, 1, s), "transpose B");
  }
  uint64_t* Ah = const_cast<uint64_t*>(A);
  int64_t ldah = lda;
  if (st.a) {
    Ah = reinterpret_cast<uint64_t*>(ws + P.ahat);
    ldah = P.kw;
    HIP_TRY(launch_copy(A, lda, Ah, P.kw, m, P.kw, s), "copy A");
  }
  if (!alt) {
    // forward changes (eq. mb-fwdbasisrecurrence / ab-fwdbasisrecurrence), in the
    // workspace copies or in the caller's A and B^T (BMM_FLAG_INPLACE_BASIS)
    HIP_TRY(launch_basis(Ah, ldah, 0, m, P.kw, 1, P.depth, 0, s, P.scheme, 0), "basis A");
    HIP_TRY(launch_basis(BT, ldbt, 0, n, P.kw, 1, P.depth, 0, s, P.scheme, 1), "basis B");
  }
  const uint64_t* T0 = Ah;
  const int64_t ldT0 = ldah;
  int leaf, tile;
  const int64_t u = (int64_t)1 << P.depth;
  int64_t leaves = 1;
  for (int i = 0; i < P.dp; ++i) leaves *= 7;
  pick_leaf(BMM_GF2, m / u, k / u, n / u, leaves, o, &leaf, &tile);
  StrassenRun run{&P, ws, leaf, tile, s};
  // C ^= chi(core) is computed as chi(chi^-1(C) ^ core): C is taken to the
  // alternative basis and back (chi^-1 is chi itself for the self-inverse design
  // and the forward change for the chaining one).
  if (!alt && acc) HIP_TRY(to_alt_basis(C, ldc, m, P.nw, P.depth, P.scheme, s), "basis C");
  BMM_TRY(run.solve(0, T0, ldT0, BT, ldbt, C, ldc, acc));
  if (!alt) HIP_TRY(launch_basis(C, ldc, 0, m, P.nw, 1, P.depth, 1, s, P.scheme), "basis C");
  if (inplace) {
    // restore the caller's operands: the self-inverse change is an involution (its
    // forward change again), the chaining change is undone by its inverse (section 2.3)
    const int undo = P.scheme == BMM_SCHEME_CHAINING ? 1 : 0;
    if (!st.a)
      HIP_TRY(launch_basis(Ah, ldah, 0, m, P.kw, 1, P.depth, undo, s, P.scheme, 0), "restore A");
    if (!st.b)
      HIP_TRY(launch_basis(BT, ldbt, 0, n, P.kw, 1, P.depth, undo, s, P.scheme, 1), "restore B");
  }
  return BMM_OK;
}

}  // extern "C"

namespace bmm {

bool batched_tuned(int64_t count, double ops, int* leaf, int* tile, int* wg_per_cu) {
  std::lock_guard<std::mutex> lock(g_mu);
  auto it = g_batched.find({count, ops_bucket(ops)});
  if (it == g_batched.end()) return false;
  std::tie(*leaf, *tile, *wg_per_cu) = it->second;
  return true;
}

void batched_tune_set(int64_t count, double ops, int leaf, int tile, int wg_per_cu) {
  std::lock_guard<std::mutex> lock(g_mu);
  g_batched[{count, ops_bucket(ops)}] = {leaf, tile, wg_per_cu};
  ++g_batched_gen;
}

uint64_t batched_tune_generation() { return g_batched_gen.load(); }

bool batched_class_tuned(int64_t count, double ops, int kclass, int* leaf, int* tile) {
  std::lock_guard<std::mutex> lock(g_mu);
  auto it = g_bclass.find({count, ops_bucket(ops), kclass});
  if (it == g_bclass.end()) return false;
  std::tie(*leaf, *tile) = it->second;
  return true;
}

void batched_class_set(int64_t count, double ops, int kclass, int leaf, int tile) {
  std::lock_guard<std::mutex> lock(g_mu);
  g_bclass[{count, ops_bucket(ops), kclass}] = {leaf, tile};
  ++g_batched_gen;
}

void batched_class_clear(int64_t count, double ops) {
  std::lock_guard<std::mutex> lock(g_mu);
  const int b = ops_bucket(ops);
  for (auto it = g_bclass.begin(); it != g_bclass.end();)
    it = (std::get<0>(it->first) == count && std::get<1>(it->first) == b) ? g_bclass.erase(it)
                                                                           : std::next(it);
  ++g_batched_gen;
}

void choose_leaf(int semiring, int64_t m, int64_t k, int64_t n, int64_t batch,
                 const bmm_options& o, int* leaf, int* tile) {
  pick_leaf(semiring, m, k, n, batch, o, leaf, tile);
}

hipError_t to_alt_basis(uint64_t* C, int64_t ldc, int64_t rows, int64_t words, int depth,
                        int scheme, hipStream_t s) {
  // chaining: the forward change is the inverse of the result's change;
  // self-inverse: the result's change is its own inverse
  if (scheme == BMM_SCHEME_CHAINING)
    return launch_basis(C, ldc, 0, rows, words, 1, depth, 0, s, scheme, 0);
  return launch_basis(C, ldc, 0, rows, words, 1, depth, 1, s, scheme, 0);
}

int strassen_alt_plan(int64_t m, int64_t k, int64_t n, int depth, const bmm_options& o,
                      size_t* bytes, int* depth_out) {
  StrassenPlan P;
  BMM_TRY(make_plan(m, k, n, depth, o, false, &P, false));
  *bytes = P.bytes;
  *depth_out = P.depth;
  return BMM_OK;
}

int strassen_alt(const uint64_t* Ahat, int64_t lda, const uint64_t* BThat, int64_t ldbt,
                 uint64_t* C, int64_t ldc, int64_t m, int64_t k, int64_t n, int depth,
                 void* ws, size_t bytes, const bmm_options& o, int accumulate, hipStream_t s) {
  StrassenPlan P;
  BMM_TRY(make_plan(m, k, n, depth, o, false, &P, false));
  if (bytes < P.bytes) return fail(BMM_E_WORKSPACE, "workspace of %zu bytes needed", P.bytes);
  if (m == 0 || n == 0 || (k == 0 && accumulate)) return BMM_OK;
  if (k == 0) return check_hip(launch_zero(C, ldc, m, P.nw, s), "zero");
  int leaf, tile;
  const int64_t u = (int64_t)1 << P.depth;
  int64_t leaves = 1;
  for (int i = 0; i < P.dp; ++i) leaves *= 7;
  pick_leaf(BMM_GF2, m / u, k / u, n / u, leaves, o, &leaf, &tile);
  StrassenRun run{&P, static_cast<char*>(ws), leaf, tile, s};
  return run.solve(0, Ahat, lda, BThat, ldbt, C, ldc, accumulate);
}

}  // namespace bmm

extern "C" {

int bmm_transpose(const uint64_t* src, int64_t lds, uint64_t* dst, int64_t ldd, int64_t rows,
                  int64_t cols, void* hip_stream) {
  if (rows < 0 || cols < 0) return fail(BMM_E_INVAL, "negative size");
  if (rows == 0 || cols == 0) return BMM_OK;
  if (!src || !dst) return fail(BMM_E_INVAL, "null pointer");
  if (lds < words_of(cols) || ldd < words_of(rows)) return fail(BMM_E_INVAL, "pitch too small");
  if (overlaps(extent(src, rows, lds, words_of(cols)), extent(dst, cols, ldd, words_of(rows))))
    return fail(BMM_E_INVAL, "src and dst overlap");
  return check_hip(launch_transpose(src, lds, 0, dst, ldd, 0, rows, cols, 1,
                                    (hipStream_t)hip_stream),
                   "transpose");
}

int bmm_basis_change(uint64_t* X, int64_t ld, int64_t rows, int64_t row_words, int depth,
                     int inverse, int scheme, int transposed, void* hip_stream) {
  if (rows < 0 || row_words < 0 || depth < 0 || depth > 20)
    return fail(BMM_E_INVAL, "bad size or depth");
  if (scheme < BMM_SCHEME_SELF_INVERSE || scheme > BMM_SCHEME_WINOGRAD)
    return fail(BMM_E_INVAL, "unknown scheme %d", scheme);
  if (rows == 0 || row_words == 0 || depth == 0) return BMM_OK;
  if (!X || ld < row_words) return fail(BMM_E_INVAL, "null pointer or pitch too small");
  const int64_t u = (int64_t)1 << depth;
  if (rows % u || row_words % u)
    return fail(BMM_E_UNSUPPORTED, "rows and row words must be divisible by 2^depth");
  return check_hip(launch_basis(X, ld, 0, rows, row_words, 1, depth, inverse ? 1 : 0,
                                (hipStream_t)hip_stream, scheme, transposed ? 1 : 0),
                   "basis change");
}

int bmm_expand(int side, int levels, int scheme, const uint64_t* src, int64_t ldp,
               int64_t strideP, uint64_t* dst, int64_t rows, int64_t words, int64_t parents,
               void* hip_stream) {
  if ((side != 0 && side != 1) || (levels != 1 && levels != 2))
    return fail(BMM_E_INVAL, "side must be 0/1 and levels 1/2");
  if (scheme < BMM_SCHEME_SELF_INVERSE || scheme > BMM_SCHEME_WINOGRAD)
    return fail(BMM_E_INVAL, "unknown scheme %d", scheme);
  if (rows < 0 || words < 0 || parents < 0) return fail(BMM_E_INVAL, "negative size");
  if (rows == 0 || words == 0 || parents == 0) return BMM_OK;
  const int64_t u = levels == 2 ? 4 : 2;
  if (rows % u || words % u) return fail(BMM_E_UNSUPPORTED, "sizes must be divisible by %ld", (long)u);
  if (!src || !dst || ldp < words) return fail(BMM_E_INVAL, "null pointer or pitch too small");
  hipStream_t s = (hipStream_t)hip_stream;
  return check_hip(levels == 2 ? launch_expand2(side, src, ldp, strideP, dst, rows, words,
                                                parents, s, scheme)
                               : launch_expand(side, src, ldp, strideP, dst, rows, words,
                                               parents, s, scheme),
                   "expand");
}

int bmm_compress(int levels, int scheme, const uint64_t* src, uint64_t* dst, int64_t ldp,
                 int64_t strideP, int64_t rows, int64_t words, int64_t parents,
                 void* hip_stream) {
  if (levels != 1 && levels != 2) return fail(BMM_E_INVAL, "levels must be 1 or 2");
  if (scheme < BMM_SCHEME_SELF_INVERSE || scheme > BMM_SCHEME_WINOGRAD)
    return fail(BMM_E_INVAL, "unknown scheme %d", scheme);
  if (rows < 0 || words < 0 || parents < 0) return fail(BMM_E_INVAL, "negative size");
  if (rows == 0 || words == 0 || parents == 0) return BMM_OK;
  const int64_t u = levels == 2 ? 4 : 2;
  if (rows % u || words % u) return fail(BMM_E_UNSUPPORTED, "sizes must be divisible by %ld", (long)u);
  if (!src || !dst || ldp < words) return fail(BMM_E_INVAL, "null pointer or pitch too small");
  hipStream_t s = (hipStream_t)hip_stream;
  return check_hip(levels == 2 ? launch_compress2(src, dst, ldp, strideP, rows, words, parents,
                                                  s, 0, scheme)
                               : launch_compress(src, dst, ldp, strideP, rows, words, parents,
                                                 s, 0, scheme),
                   "compress");
}

int bmm_leaf_tiles(int leaf, int* count_out) {
  if (!count_out) return fail(BMM_E_INVAL, "null count_out");
  if (leaf == BMM_LEAF_VALU) *count_out = 2;
  else if (leaf == BMM_LEAF_MFMA_I8 || leaf == BMM_LEAF_MFMA_F4) *count_out = MFMA_NUM_TILES;
  else return fail(BMM_E_INVAL, "unknown leaf %d", leaf);
  return BMM_OK;
}

int bmm_leaf_choice(int semiring, int64_t m, int64_t k, int64_t n, int64_t batch,
                    const bmm_options* opt, int* leaf_out, int* tile_out) {
  if (semiring != BMM_GF2 && semiring != BMM_BOOLEAN) return fail(BMM_E_INVAL, "bad semiring");
  if (m < 0 || k < 0 || n < 0 || batch <= 0) return fail(BMM_E_INVAL, "bad shape");
  if (!leaf_out || !tile_out) return fail(BMM_E_INVAL, "null output");
  pick_leaf(semiring, m, k, n, batch, opt ? *opt : defaults(), leaf_out, tile_out);
  return BMM_OK;
}

int bmm_leaf_tile_shape(int leaf, int tile, int* rows_out, int* cols_out) {
  if (!rows_out || !cols_out) return fail(BMM_E_INVAL, "null output");
  if (leaf == BMM_LEAF_VALU && (tile == 1 || tile == 2)) {
    *rows_out = tile == 1 ? 128 : 512;
    *cols_out = tile == 1 ? 128 : 1024;
    return BMM_OK;
  }
  if ((leaf == BMM_LEAF_MFMA_I8 || leaf == BMM_LEAF_MFMA_F4) && tile >= 1 &&
      tile <= MFMA_NUM_TILES) {
    *rows_out = leaf_mfma_tile_rows(tile - 1);
    *cols_out = leaf_mfma_tile_cols(tile - 1);
    return BMM_OK;
  }
  return fail(BMM_E_INVAL, "unknown leaf %d / tile %d", leaf, tile);
}

int bmm_autotune_set(int semiring, int64_t m, int64_t k, int64_t n, int64_t batch, int leaf,
                     int tile) {
  int count = 0;
  if (semiring != BMM_GF2 && semiring != BMM_BOOLEAN) return fail(BMM_E_INVAL, "bad semiring");
  if (m <= 0 || k < 0 || n <= 0 || batch <= 0) return fail(BMM_E_INVAL, "bad shape");
  BMM_TRY(bmm_leaf_tiles(leaf, &count));
  if (tile < 1 || tile > count) return fail(BMM_E_INVAL, "bad tile %d", tile);
  std::lock_guard<std::mutex> lock(g_mu);
  TuneVal& v = g_tune[{semiring, m, k, n, batch_bucket(batch)}];
  v.best_leaf = leaf;
  v.tile[leaf] = tile;
  return BMM_OK;
}

int bmm_autotune_leaf(int semiring, int64_t m, int64_t k, int64_t n, int64_t batch,
                      int* leaf_out, int* tile_out, double* seconds_out) {
  if (semiring != BMM_GF2 && semiring != BMM_BOOLEAN) return fail(BMM_E_INVAL, "bad semiring");
  if (m <= 0 || k <= 0 || n <= 0 || batch <= 0) return fail(BMM_E_INVAL, "sizes must be positive");
  const int64_t kw = words_of(k), nw = words_of(n);
  const int64_t nb = batch_bucket(batch);  // time on the bucket's batch size
  uint64_t *A = nullptr, *BT = nullptr, *C = nullptr;
  // the right operand buffer serves as B^T (n x k) and, for the VALU leaf's
  // outer-product form, as B (k x n)
  const size_t ba = (size_t)m * kw * 8, bb = (size_t)std::max(n * kw, k * nw) * 8,
               bc = (size_t)m * nw * 8;
  if (dev_malloc((void**)&A, ba * nb) != hipSuccess || dev_malloc((void**)&BT, bb * nb) != hipSuccess ||
      dev_malloc((void**)&C, bc * nb) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipFree(A);
    (void)hipFree(BT);
    (void)hipFree(C);
    return fail(BMM_E_NOMEM, "autotune buffers");
  }
  int rc = BMM_OK;
  double best = 1e30;
  int best_leaf = BMM_LEAF_MFMA_I8, best_tile = 1;
  double best_of[4] = {1e30, 1e30, 1e30, 1e30};
  int tile_of[4] = {0, 0, 0, 0};
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  // dense random operands: the rate of the matrix cores depends on the bits they see
  rc = check_hip(launch_random(A, (int64_t)(ba * nb / 8), 0x5EED0001ull, nullptr), "tuning data");
  if (rc == BMM_OK)
    rc = check_hip(launch_random(BT, (int64_t)(bb * nb / 8), 0x5EED0002ull, nullptr), "tuning data");
  std::vector<std::pair<int, int>> cands = {{BMM_LEAF_VALU, 1}};
  if (nb == 1) cands.push_back({BMM_LEAF_VALU, 2});  // cubic products only
  for (int t = 1; t <= MFMA_NUM_TILES; ++t) cands.push_back({BMM_LEAF_MFMA_I8, t});
  if (k < ((int64_t)1 << 24))
    for (int t = 1; t <= MFMA_NUM_TILES; ++t) cands.push_back({BMM_LEAF_MFMA_F4, t});
  for (auto [leaf, tile] : cands) {
    if (rc != BMM_OK) break;
    LeafBatch p{A, kw, m * kw, BT, kw, n * kw, C, nw, m * nw, m, k, n, nb, 0};
    auto launch = [&, leaf = leaf, tile = tile]() {
      if (leaf == BMM_LEAF_VALU && tile == 2)
        return check_hip(launch_leaf_valu_outer(semiring, A, kw, BT, nw, C, nw, m, k, n, 0,
                                                nullptr), "leaf launch");
      return run_leaf(semiring, leaf, tile, p, nullptr);
    };
    // a timed warm-up; launches longer than 0.2 s are timed once, shorter ones 3 more times
    (void)hipEventRecord(e0, nullptr);
    rc = launch();
    (void)hipEventRecord(e1, nullptr);
    if (rc != BMM_OK) break;
    if (hipEventSynchronize(e1) != hipSuccess) {
      rc = check_hip(hipGetLastError(), "autotune sync");
      break;
    }
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    int reps = 1;
    if (ms < 200.f) {
      reps = 3;
      (void)hipEventRecord(e0, nullptr);
      for (int r = 0; r < reps && rc == BMM_OK; ++r) rc = launch();
      (void)hipEventRecord(e1, nullptr);
      if (rc != BMM_OK) break;
      if (hipEventSynchronize(e1) != hipSuccess) {
        rc = check_hip(hipGetLastError(), "autotune sync");
        break;
      }
      (void)hipEventElapsedTime(&ms, e0, e1);
    }
    const double sec = ms * 1e-3 / reps;
    if (sec < best_of[leaf]) {
      best_of[leaf] = sec;
      tile_of[leaf] = tile;
    }
    if (sec < best) {
      best = sec;
      best_leaf = leaf;
      best_tile = tile;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(A);
  (void)hipFree(BT);
  (void)hipFree(C);
  if (rc != BMM_OK) return rc;
  {
    std::lock_guard<std::mutex> lock(g_mu);
    TuneVal& v = g_tune[{semiring, m, k, n, nb}];
    v.best_leaf = best_leaf;
    for (int l = 1; l <= 3; ++l)
      if (tile_of[l]) v.tile[l] = tile_of[l];
  }
  if (leaf_out) *leaf_out = best_leaf;
  if (tile_out) *tile_out = best_tile;
  if (seconds_out) *seconds_out = best;
  return BMM_OK;
}

int bmm_autotune_cubic(int semiring, int64_t m, int64_t k, int64_t n, int* leaf_out,
                       int* tile_out, double* seconds_out) {
  return bmm_autotune_leaf(semiring, m, k, n, 1, leaf_out, tile_out, seconds_out);
}

int bmm_autotune_strassen(const uint64_t* A, int64_t lda, const uint64_t* B, int64_t ldb,
                          uint64_t* C, int64_t ldc, int64_t m, int64_t k, int64_t n,
                          void* workspace, size_t workspace_bytes, const bmm_options* opt,
                          int* depth_out, int* depth_serial_out, int* shift_out,
                          double* seconds_out) {
  const bmm_options o = opt ? *opt : defaults();
  int dmax = 0;
  while (dmax < 10) {
    const int64_t u = (int64_t)2 << dmax;
    if (m % u || k % (64 * u) || n % (64 * u) || m / u < 1024 || k / u < 1024 || n / u < 1024)
      break;
    ++dmax;
  }
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  double best = 1e30;
  int best_d = -1, best_ds = -1, best_sh = 0, rc = BMM_OK, tried = 0;
  for (int d = dmax; d >= std::max(0, dmax - 3); --d) {
    // the plain leaf, then the shifted leaf level with 16-byte and with 8-byte operand
    // loads, each with the fewest depth-first levels whose workspace fits
    for (int sh = 0; sh <= 2 && rc == BMM_OK; ++sh) {
      for (int ds = 0; ds <= d; ++ds) {
        bmm_options t = o;
        t.depth_serial = ds;
        t.depth_parallel = d - ds;
        t.shift = sh;
        StrassenPlan P;
        const Staging st = staging_of(t);
        if (make_plan(m, k, n, d, t, st.a, &P, st.b) != BMM_OK) continue;
        if (P.shift != sh) break;  // this shift does not apply at this depth
        if (P.bytes > workspace_bytes) continue;  // more breadth-first levels than memory allows
        rc = bmm_gf2_strassen(A, lda, B, ldb, C, ldc, m, k, n, d, workspace, workspace_bytes,
                              &t, nullptr);
        if (rc != BMM_OK) break;
        (void)hipEventRecord(e0, nullptr);
        rc = bmm_gf2_strassen(A, lda, B, ldb, C, ldc, m, k, n, d, workspace, workspace_bytes,
                              &t, nullptr);
        (void)hipEventRecord(e1, nullptr);
        if (rc != BMM_OK) break;
        if (hipEventSynchronize(e1) != hipSuccess) {
          rc = check_hip(hipGetLastError(), "autotune sync");
          break;
        }
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        ++tried;
        if (ms * 1e-3 < best) {
          best = ms * 1e-3;
          best_d = d;
          best_ds = ds;
          best_sh = sh;
        }
        break;  // the fewest serial levels that fit is the candidate for this depth
      }
    }
    if (rc != BMM_OK) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != BMM_OK) return rc;
  if (!tried) return fail(BMM_E_WORKSPACE, "no Strassen depth fits the workspace");
  {
    std::lock_guard<std::mutex> lock(g_mu);
    g_depth[{m, k, n}] = {best_d, best_ds, best_sh};
  }
  if (depth_out) *depth_out = best_d;
  if (depth_serial_out) *depth_serial_out = best_ds;
  if (shift_out) *shift_out = best_sh;
  if (seconds_out) *seconds_out = best;
  return BMM_OK;
}

int bmm_autotune_k_panel(int semiring, const uint64_t* A, int64_t lda, const uint64_t* B,
                         int64_t ldb, uint64_t* C, int64_t ldc, int64_t m, int64_t k, int64_t n,
                         const bmm_options* opt, const int64_t* candidates, int count,
                         int64_t* panel_out, double* seconds_out) {
  if (semiring != BMM_GF2 && semiring != BMM_BOOLEAN)
    return fail(BMM_E_INVAL, "unknown semiring %d", semiring);
  bmm_options o = opt ? *opt : defaults();
  if (o.flags & (BMM_FLAG_ACCUMULATE | BMM_FLAG_HOST_OPERANDS))
    return fail(BMM_E_INVAL, "k-panel tuning runs the product repeatedly on device "
                "operands: accumulation and host operands are not allowed");
  if (count < 0 || (count > 0 && !candidates)) return fail(BMM_E_INVAL, "bad candidate list");
  if (m <= 0 || n <= 0 || k <= 0) return fail(BMM_E_INVAL, "k-panel tuning needs a nonempty product");
  // candidates: the caller's, else one panel and every power of two from 8192 bits below k
  std::vector<int64_t> cand;
  if (count > 0) {
    for (int i = 0; i < count; ++i) {
      if (candidates[i] <= 0) return fail(BMM_E_INVAL, "candidate %d is not positive", i);
      cand.push_back(std::min<int64_t>((candidates[i] + 63) / 64 * 64, k));
    }
  } else {
    cand.push_back(k);
    for (int64_t b = (int64_t)1 << 40; b >= 8192; b >>= 1)
      if (b < k) cand.push_back(b);
  }
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0), "hipEventCreate");
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(BMM_E_DEVICE, "hipEventCreate failed");
  }
  double best = 1e30;
  int64_t best_bits = k;
  int rc = BMM_OK;
  auto product = [&](const bmm_options* t) {
    return cubic(semiring, A, lda, B, ldb, C, ldc, m, k, n, t, nullptr);
  };
  for (size_t i = 0; i < cand.size() && rc == BMM_OK; ++i) {
    bmm_options t = o;
    t.k_panel = cand[i];
    if (i == 0) rc = product(&t);  // warm-up (B^T scratch, code objects)
    if (rc != BMM_OK) break;
    (void)hipEventRecord(e0, nullptr);
    rc = product(&t);
    (void)hipEventRecord(e1, nullptr);
    if (rc != BMM_OK) break;
    if (hipEventSynchronize(e1) != hipSuccess) {
      rc = check_hip(hipGetLastError(), "autotune sync");
      break;
    }
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    if (ms * 1e-3 < best) {
      best = ms * 1e-3;
      best_bits = cand[i];
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != BMM_OK) return rc;
  {
    std::lock_guard<std::mutex> lock(g_mu);
    g_kpanel[{semiring, m, k, n}] = best_bits;
  }
  if (panel_out) *panel_out = best_bits;
  if (seconds_out) *seconds_out = best;
  return BMM_OK;
}

int bmm_autotune_save(const char* path) {
  if (!path) return fail(BMM_E_INVAL, "null path");
  std::ofstream f(path);
  if (!f) return fail(BMM_E_INVAL, "cannot write %s", path);
  std::lock_guard<std::mutex> lock(g_mu);
  f << "# bmm autotune table\n"
       "# leaf semiring m k n batch_bucket best_leaf tile_valu tile_mfma_i8 tile_mfma_f4\n"
       "# depth m k n depth depth_serial shift\n"
       "# batched count log2_ops leaf tile workgroups_per_cu\n"
       "# batched_class count log2_ops k_class leaf tile\n"
       "# kpanel semiring m k n panel_bits\n";
  for (auto& [key, val] : g_tune)
    f << "leaf " << key.semiring << ' ' << key.m << ' ' << key.k << ' ' << key.n << ' '
      << key.batch << ' ' << val.best_leaf << ' ' << val.tile[1] << ' ' << val.tile[2] << ' '
      << val.tile[3] << '\n';
  for (auto& [key, val] : g_depth)
    f << "depth " << std::get<0>(key) << ' ' << std::get<1>(key) << ' ' << std::get<2>(key)
      << ' ' << std::get<0>(val) << ' ' << std::get<1>(val) << ' ' << std::get<2>(val) << '\n';
  for (auto& [key, val] : g_batched)
    f << "batched " << key.first << ' ' << key.second << ' ' << std::get<0>(val) << ' '
      << std::get<1>(val) << ' ' << std::get<2>(val) << '\n';
  for (auto& [key, val] : g_bclass)
    f << "batched_class " << std::get<0>(key) << ' ' << std::get<1>(key) << ' '
      << std::get<2>(key) << ' ' << val.first << ' ' << val.second << '\n';
  for (auto& [key, val] : g_kpanel)
    f << "kpanel " << std::get<0>(key) << ' ' << std::get<1>(key) << ' ' << std::get<2>(key)
      << ' ' << std::get<3>(key) << ' ' << val << '\n';
  return f ? BMM_OK : fail(BMM_E_INVAL, "write failed: %s", path);
}

int bmm_autotune_load(const char* path) {
  if (!path) return fail(BMM_E_INVAL, "null path");
  std::ifstream f(path);
  if (!f) return fail(BMM_E_INVAL, "cannot read %s", path);
  std::string line;
  while (std::getline(f, line)) {
    if (line.empty() || line[0] == '#') continue;
    int sr, leaf, t1, t2, t3, d, ds;
    long long m, k, n, b;
    if (sscanf(line.c_str(), "leaf %d %lld %lld %lld %lld %d %d %d %d", &sr, &m, &k, &n, &b,
               &leaf, &t1, &t2, &t3) == 9) {
      int cnt = 0;
      if ((sr != BMM_GF2 && sr != BMM_BOOLEAN) || m <= 0 || n <= 0 || k < 0 || b <= 0 ||
          leaf < 1 || leaf > 3 || t1 < 0 || t1 > 2 || t2 < 0 || t3 < 0 ||
          bmm_leaf_tiles(BMM_LEAF_MFMA_I8, &cnt) != BMM_OK || t2 > cnt || t3 > cnt)
        return fail(BMM_E_INVAL, "bad leaf line: %s", line.c_str());
      std::lock_guard<std::mutex> lock(g_mu);
      TuneVal& v = g_tune[{sr, m, k, n, batch_bucket(b)}];
      v.best_leaf = leaf;
      v.tile[1] = t1;
      v.tile[2] = t2;
      v.tile[3] = t3;
    } else if (sscanf(line.c_str(), "depth %lld %lld %lld %d %d", &m, &k, &n, &d, &ds) == 5) {
      int sh = 0;  // lines without the shift column: the plain leaf
      if (sscanf(line.c_str(), "depth %lld %lld %lld %d %d %d", &m, &k, &n, &d, &ds, &sh) < 5 ||
          d < 0 || ds < 0 || ds > d || sh < 0 || sh > 2)
        return fail(BMM_E_INVAL, "bad depth line: %s", line.c_str());
      std::lock_guard<std::mutex> lock(g_mu);
      g_depth[{m, k, n}] = {d, ds, sh};
    } else if (sscanf(line.c_str(), "kpanel %d %lld %lld %lld %lld", &sr, &m, &k, &n, &b) == 5) {
      if ((sr != BMM_GF2 && sr != BMM_BOOLEAN) || m <= 0 || k <= 0 || n <= 0 || b <= 0 ||
          b % 64 != 0)
        return fail(BMM_E_INVAL, "bad kpanel line: %s", line.c_str());
      std::lock_guard<std::mutex> lock(g_mu);
      g_kpanel[{sr, m, k, n}] = b;
    } else if (sscanf(line.c_str(), "batched_class %lld %d %d %d %d", &m, &d, &ds, &leaf, &t1) ==
               5) {
      if (m <= 0 || d < 0 || ds < 0 || ds > 2 || leaf < BMM_LEAF_VALU || leaf > BMM_LEAF_MFMA_F4 ||
          t1 < 1 || t1 > 4)
        return fail(BMM_E_INVAL, "bad batched_class line: %s", line.c_str());
      std::lock_guard<std::mutex> lock(g_mu);
      g_bclass[{m, d, ds}] = {leaf, t1};
      ++g_batched_gen;
    } else if (sscanf(line.c_str(), "batched %lld %d %d %d %d", &m, &d, &leaf, &t1, &t2) >= 4) {
      if (sscanf(line.c_str(), "batched %lld %d %d %d %d", &m, &d, &leaf, &t1, &t2) == 4) t2 = 4;
      if (m <= 0 || d < 0 || (leaf != BMM_LEAF_MFMA_I8 && leaf != BMM_LEAF_MFMA_F4) ||
          t1 < 1 || t1 > 4 || t2 < 1 || t2 > 64)
        return fail(BMM_E_INVAL, "bad batched line: %s", line.c_str());
      std::lock_guard<std::mutex> lock(g_mu);
      g_batched[{m, d}] = {leaf, t1, t2};
      ++g_batched_gen;
    } else {
      return fail(BMM_E_INVAL, "bad line in %s: %s", path, line.c_str());
    }
  }
  return BMM_OK;
}

const char* bmm_status_string(int status) {
  switch (status) {
    case BMM_OK: return "ok";
    case BMM_E_INVAL: return "invalid argument";
    case BMM_E_UNSUPPORTED: return "unsupported";
    case BMM_E_WORKSPACE: return "workspace too small";
    case BMM_E_NOMEM: return "out of memory";
    case BMM_E_DEVICE: return "device error";
    default: return "unknown status";
  }
}

const char* bmm_last_error(void) { return g_last_error.c_str(); }

const char* bmm_version(void) { return "bmm 0.1 (gfx950)"; }

int bmm_debug_fail_allocations(int64_t count) {
  g_fail_allocs.store(count > 0 ? count : 0);
  return BMM_OK;
}

void bmm_finalize(void) {
  batched_cache_clear();
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch.empty()) (void)hipDeviceSynchronize();
  int cur = 0;
  (void)hipGetDevice(&cur);
  for (auto& [dev, slot] : g_scratch) {
    if (slot.first) {
      (void)hipSetDevice(dev);
      (void)hipFree(slot.first);
    }
  }
  (void)hipSetDevice(cur);
  g_scratch.clear();
  g_tune.clear();
  g_depth.clear();
  g_batched.clear();
  g_bclass.clear();
  ++g_batched_gen;
}

}  // extern "C"
