// ps_check_finite: opt-in scan of float arrays for NaN and infinity.  The
// hot-path calls never test their inputs; a caller who wants to know runs
// this on parameters, gradients or rendered maps between steps.
#include <algorithm>

#include "ps_internal.h"

using namespace ps;

namespace {

constexpr int kBlock = 256;

__global__ void check_clear_kernel(unsigned long long* count) { *count = 0ull; }

// Grid-stride count of non-finite values; one atomic per wave.
__global__ __launch_bounds__(kBlock) void check_finite_kernel(const float* x, int64_t n,
                                                              unsigned long long* count) {
  int bad = 0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
    bad += !isfinite(x[i]);
  const uint64_t m = ballot(bad != 0);
  if (m == 0) return;
  for (int o = 32; o >= 1; o >>= 1) bad += __shfl_xor(bad, o, 64);
  if ((threadIdx.x & 63) == 0) atomicAdd(count, (unsigned long long)bad);
}

}  // namespace

extern "C" int ps_check_finite(const float* x, int64_t n, int64_t* d_count, int64_t* h_count, void* stream) {
  if (n < 0 || !d_count || (n > 0 && !x)) return ps_set_error(PS_ERR_INVALID, "ps_check_finite: bad argument");
  hipStream_t st = (hipStream_t)stream;
  unsigned long long* c = reinterpret_cast<unsigned long long*>(d_count);
  hipLaunchKernelGGL(check_clear_kernel, dim3(1), dim3(1), 0, st, c);
  if (n > 0) {
    const int64_t blocks = std::min<int64_t>((n + kBlock - 1) / kBlock, 4096);
    hipLaunchKernelGGL(check_finite_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, st, x, n, c);
  }
  PS_HIP_CHECK(hipGetLastError());
  if (h_count) {
    PS_HIP_CHECK(hipMemcpyAsync(h_count, d_count, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    PS_HIP_CHECK(hipStreamSynchronize(st));
  }
  return PS_OK;
}
