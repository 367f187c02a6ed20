// Issue-rate calibration of the vector ALU, for the bit-operation roofline of the
// VALU leaf.
//
// The paper counts one 32-bit lane operation as 32 bit operations and takes the
// bit-operation peak of a device as its lane operations per second times the
// word width (section 1.2; the peak figures of section 4).  What that rate is
// for the three-input v_bitop3_b32 on gfx950 (which can issue two VALU
// instructions per SIMD in one quad-cycle) is measured here instead of assumed:
// every lane folds CH independent 32-bit accumulators, one v_bitop3_b32 each per
// round, with no memory traffic inside the timed loop, and every wave records
// its own start and end on the core-clock counter (s_memtime) and on the
// constant-rate counter.  Lane operations per core clock per CU then follow from
// the instruction count and the per-wave cycle counts, independent of the clock
// frequency the chip chose.
#include "bmm_internal.h"

namespace bmm {
namespace {

constexpr int kCalibChains = 16;

// Every round: one v_bitop3_b32 (the GF(2) fold's truth table, (a & b) ^ c) per
// chain; chain j reads chains j+1 and j+2 of the previous round, so a round's
// instructions are independent of each other.
__global__ __launch_bounds__(256) void valu_rate_kernel(uint32_t seed, int64_t rounds,
                                                        uint32_t* __restrict__ sink,
                                                        long long* __restrict__ stamps) {
  const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t x[kCalibChains];
#pragma unroll
  for (int j = 0; j < kCalibChains; ++j) x[j] = seed * (2u * j + 1u) ^ (tid * 0x9E3779B9u);
  const long long c0 = clock64();
  const long long r0 = wall_clock64();
  for (int64_t r = 0; r < rounds; r += 4) {
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int j = 0; j < kCalibChains; ++j)
        x[j] = __builtin_amdgcn_bitop3_b32(x[(j + 1) % kCalibChains],
                                           x[(j + 2) % kCalibChains], x[j], 0x6A);
  }
  const long long c1 = clock64();
  const long long r1 = wall_clock64();
  uint32_t acc = 0;
#pragma unroll
  for (int j = 0; j < kCalibChains; ++j) acc ^= x[j];
  sink[tid] = acc;
  if ((threadIdx.x & 63) == 0) {
    const uint32_t wave = tid >> 6;
    stamps[4 * wave + 0] = c0;
    stamps[4 * wave + 1] = c1;
    stamps[4 * wave + 2] = r0;
    stamps[4 * wave + 3] = r1;
  }
}

}  // namespace

int calib_chains() { return kCalibChains; }

// rounds: a multiple of 4 (the loop is unrolled by 4).
hipError_t launch_valu_rate(uint32_t seed, int64_t rounds, int blocks, uint32_t* sink,
                            long long* stamps, hipStream_t s) {
  if (blocks <= 0 || rounds <= 0) return hipSuccess;
  if (!grid_fits(blocks, 256)) return kGridTooLarge;
  hipLaunchKernelGGL(valu_rate_kernel, dim3((unsigned)blocks), dim3(256), 0, s, seed, rounds,
                     sink, stamps);
  return hipGetLastError();
}

}  // namespace bmm

// ---- C ABI -----------------------------------------------------------------

#include <algorithm>
#include <vector>

#include "../../include/bmm.h"

extern "C" int bmm_calibrate_valu(int waves_per_simd, int64_t rounds, double* lane_ops_per_clk_cu,
                                  double* clock_ghz, double* seconds, double* aggregate_bops) {
  using namespace bmm;
  if (waves_per_simd < 1 || waves_per_simd > 8 || rounds <= 0 || rounds % 4 != 0)
    return set_error(BMM_E_INVAL, "waves_per_simd must be 1..8 and rounds a positive multiple of 4");
  int dev = 0, cus = 0, wall_khz = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess)
    return set_error(BMM_E_DEVICE, "device query: %s", hipGetErrorString(hipGetLastError()));
  // one 256-thread workgroup puts one wave on each of a CU's four SIMDs
  const int blocks = cus * waves_per_simd;
  const int waves = blocks * 4;
  uint32_t* sink = nullptr;
  long long* stamps = nullptr;
  if (bmm::dev_malloc((void**)&sink, (size_t)blocks * 256 * 4) != hipSuccess ||
      bmm::dev_malloc((void**)&stamps, (size_t)waves * 4 * sizeof(long long)) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipFree(sink);
    return set_error(BMM_E_NOMEM, "calibration buffers");
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = BMM_OK;
  float ms = 0.f;
  std::vector<long long> st((size_t)waves * 4);
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    rc = set_error(BMM_E_DEVICE, "event create");
  } else {
    // a short warm-up launch raises the clock, then the timed one
    hipError_t e = launch_valu_rate(0x5EEDu, 4 * 64, blocks, sink, stamps, nullptr);
    if (e == hipSuccess) e = hipEventRecord(e0, nullptr);
    if (e == hipSuccess) e = launch_valu_rate(0x5EEDu, rounds, blocks, sink, stamps, nullptr);
    if (e == hipSuccess) e = hipEventRecord(e1, nullptr);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e == hipSuccess)
      e = hipMemcpy(st.data(), stamps, st.size() * sizeof(long long), hipMemcpyDeviceToHost);
    if (e != hipSuccess) rc = set_error(BMM_E_DEVICE, "calibration: %s", hipGetErrorString(e));
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(sink);
  (void)hipFree(stamps);
  if (rc != BMM_OK) return rc;
  // core clock: per wave, core cycles over constant-rate time; the median over waves
  const double insts = (double)rounds * calib_chains();
  std::vector<double> clk;
  for (int w = 0; w < waves; ++w) {
    const double cyc = (double)(st[4 * w + 1] - st[4 * w]);
    const double sec = (double)(st[4 * w + 3] - st[4 * w + 2]) / (wall_khz * 1e3);
    if (cyc > 0 && sec > 0) clk.push_back(cyc / sec);
  }
  if (clk.empty() || ms <= 0.f) return set_error(BMM_E_DEVICE, "calibration: no valid timings");
  std::sort(clk.begin(), clk.end());
  const double c_med = clk[clk.size() / 2];
  const double sec = ms * 1e-3;
  // the whole launch: every wave's instructions over the launch's core cycles (waves
  // need not all be resident at once, so per-wave rates would overstate a SIMD's)
  const double lane_ops = insts * waves * 64.0;
  if (lane_ops_per_clk_cu) *lane_ops_per_clk_cu = lane_ops / (sec * c_med * cus);
  if (clock_ghz) *clock_ghz = c_med * 1e-9;
  if (seconds) *seconds = sec;
  // 2 bit operations on each of 32 bit positions per lane operation
  if (aggregate_bops) *aggregate_bops = lane_ops * 64.0 / sec;
  return BMM_OK;
}
