// Cubic leaf on the matrix cores with operand panels shared through LDS.
//
// Same arithmetic as leaf_mfma.hip (bits expanded in registers to int8 or
// E2M1 operands, exact counts, ballot repacking; see mfma_tile.h), but an
// 8-wave workgroup owns a 256 x 256 tile of C (2 x 4 waves of 128 x 64) and
// stages, per step of 8 words of k, its 256 rows of A and 256 rows of B^T in
// LDS with 64-byte coalesced loads.  Each operand row is then fetched from
// L2 once per workgroup instead of once per wave that uses it (3x less
// traffic than independent waves), which keeps the matrix cores fed at the
// fp4 rate.  LDS rows are padded to 80 bytes so that the eight lanes served
// together by a 16-byte LDS read hit distinct banks.  The next stage's words
// are loaded into registers while the current stage computes (one LDS buffer
// pair, double buffered).
#include "mfma_tile.h"

namespace bmm {
namespace {

constexpr int LW = 8;             // waves per workgroup
constexpr int LT = 64 * LW;       // threads
constexpr int L_RA = 4, L_RB = 2; // wave tile 128 x 64
constexpr int L_TM = 256, L_TN = 256;
constexpr int KS = 8;             // words of k per stage
constexpr int ROWB = 80;          // padded LDS row, bytes (64 data + 16)
constexpr int PANEL = (L_TM + L_TN) * ROWB;  // bytes per stage buffer

template <int SEMI, int FMT>
__global__ __launch_bounds__(LT) __attribute__((amdgpu_waves_per_eu(2))) void leaf_mfma_lds_kernel(
    LeafBatch p, int64_t grid_m, int64_t grid_n) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  const TileCoord c = xcd_tile(blockIdx.x, gridDim.x, grid_m, grid_n);
  if (c.b >= p.batch) return;  // uniform per workgroup
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wy = wave >> 2, wx = wave & 3;  // 2 x 4 waves
  const int half = lane >> 5, li = lane & 31;
  const uint64_t* A = p.A + c.b * p.strideA;
  const uint64_t* BT = p.BT + c.b * p.strideB;
  const int64_t kw = (p.k + 63) >> 6;
  const int64_t row0 = c.tm * L_TM, col0 = c.tn * L_TN;

  // Global -> register staging: 512 rows (256 of A, then 256 of B^T) x 64 bytes per
  // stage = 2048 chunks of 16 bytes, 4 per thread; chunk q: row q >> 2, part q & 3.
  const uint64_t* src[4];
  int soff[4], spart[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int q = tid + i * LT;
    const int r = q >> 2, part = q & 3;
    spart[i] = part;
    if (r < L_TM) {
      int64_t g = row0 + r;
      g = g < p.m ? g : p.m - 1;
      src[i] = A + g * p.lda + 2 * part;
    } else {
      int64_t g = col0 + (r - L_TM);
      g = g < p.n ? g : p.n - 1;
      src[i] = BT + g * p.ldbt + 2 * part;
    }
    soff[i] = r * ROWB + part * 16;
  }
  const bool aligned = ((reinterpret_cast<uintptr_t>(p.A) | reinterpret_cast<uintptr_t>(p.BT)) & 15) == 0 &&
                       ((p.lda | p.ldbt | p.strideA | p.strideB) & 1) == 0;
  ulonglong2 stage[4];
  auto load = [&](int64_t w0) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t w = w0 + 2 * spart[i];
      if (aligned && w + 1 < kw) {
        stage[i] = *reinterpret_cast<const ulonglong2*>(src[i] + w0);
      } else {
        stage[i].x = w < kw ? src[i][w0] : 0ull;
        stage[i].y = w + 1 < kw ? src[i][w0 + 1] : 0ull;
      }
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
      *reinterpret_cast<ulonglong2*>(smem + buf * PANEL + soff[i]) = stage[i];
  };

  using AccV = typename mfma::Acc<FMT>::type;
  AccV acc[L_RA][L_RB];
#pragma unroll
  for (int f = 0; f < L_RA; ++f)
#pragma unroll
    for (int g = 0; g < L_RB; ++g) acc[f][g] = AccV{};

  // LDS rows this lane reads: A rows wy*128 + 32f + li, B^T rows 256 + wx*64 + 32g + li
  int aoff[L_RA], boff[L_RB];
#pragma unroll
  for (int f = 0; f < L_RA; ++f) aoff[f] = (wy * 128 + 32 * f + li) * ROWB + 16 * half;
#pragma unroll
  for (int g = 0; g < L_RB; ++g) boff[g] = (L_TM + wx * 64 + 32 * g + li) * ROWB + 16 * half;

  const int64_t stages = (kw + KS - 1) / KS;
  if (stages > 0) {
    load(0);
    store(0);
  }
  __syncthreads();
  for (int64_t st = 0; st < stages; ++st) {
    const int cur = (int)(st & 1);
    if (st + 1 < stages) load((st + 1) * KS);
    const unsigned char* base = smem + cur * PANEL;
    // two steps per stage: lane half h takes words 4s + 2h and 4s + 2h + 1
#pragma unroll
    for (int s = 0; s < KS / 4; ++s) {
      uint64_t xa[2][L_RA], xb[2][L_RB];
#pragma unroll
      for (int f = 0; f < L_RA; ++f) {
        const ulonglong2 v = *reinterpret_cast<const ulonglong2*>(base + aoff[f] + 32 * s);
        xa[0][f] = v.x;
        xa[1][f] = v.y;
      }
#pragma unroll
      for (int g = 0; g < L_RB; ++g) {
        const ulonglong2 v = *reinterpret_cast<const ulonglong2*>(base + boff[g] + 32 * s);
        xb[0][g] = v.x;
        xb[1][g] = v.y;
      }
      mfma::mfma_word<SEMI, L_RA, L_RB, FMT>(xa[0], xb[0], acc);
      mfma::mfma_word<SEMI, L_RA, L_RB, FMT>(xa[1], xb[1], acc);
    }
    if (st + 1 < stages) store(cur ^ 1);
    __syncthreads();
  }

  const int64_t tm = c.tm * 2 + wy, tn = c.tn * 4 + wx;  // wave tile (128 x 64) coordinates
  if (tm * 128 >= p.m || tn * 64 >= (((p.n + 63) >> 6) << 6)) return;
  mfma::epilogue<SEMI, L_RA, L_RB, FMT>(acc, p.C + c.b * p.strideC, p.ldc, p.m, p.n, tm, tn,
                                        p.accumulate);
}

template <int SEMI, int FMT>
hipError_t launch_sf(const LeafBatch& p, hipStream_t s) {
  const int64_t grid_m = (p.m + L_TM - 1) / L_TM;
  const int64_t grid_n = (p.n + L_TN - 1) / L_TN;
  const int64_t blocks = grid_m * grid_n * p.batch;
  if (blocks == 0) return hipSuccess;
  if (!grid_fits(blocks, LT)) return kGridTooLarge;
  static bool configured = false;
  if (!configured) {
    hipError_t e = hipFuncSetAttribute(
        reinterpret_cast<const void*>(&leaf_mfma_lds_kernel<SEMI, FMT>),
        hipFuncAttributeMaxDynamicSharedMemorySize, 2 * PANEL);
    if (e != hipSuccess) return e;
    configured = true;
  }
  hipLaunchKernelGGL((leaf_mfma_lds_kernel<SEMI, FMT>), dim3((unsigned)blocks), dim3(LT),
                     2 * PANEL, s, p, grid_m, grid_n);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_leaf_mfma_lds(int semiring, int fmt, const LeafBatch& p, hipStream_t s) {
  if (p.m <= 0 || p.n <= 0 || p.batch <= 0) return hipSuccess;
  if (fmt == mfma::FMT_F4)
    return semiring == GF2 ? launch_sf<GF2, mfma::FMT_F4>(p, s)
                           : launch_sf<BOOLEAN, mfma::FMT_F4>(p, s);
  return semiring == GF2 ? launch_sf<GF2, mfma::FMT_I8>(p, s)
                         : launch_sf<BOOLEAN, mfma::FMT_I8>(p, s);
}

}  // namespace bmm
