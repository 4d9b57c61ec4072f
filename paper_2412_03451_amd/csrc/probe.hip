// ps_valu_probe: the vector ALU's issue rate, measured.  The render kernels
// are priced in lane operations against the non-packed issue rate (one fp32
// or fp64 operation per lane per cycle); this kernel runs eight independent
// chains of fused multiply-adds per lane, enough to hide the operation
// latency with four waves per SIMD, so its launch time gives that rate for
// either precision on the chip at hand.
#include "ps_internal.h"

namespace {

constexpr int kBlock = 256;
constexpr int kChains = 8;

template <typename T>
__global__ __launch_bounds__(kBlock) void valu_probe_kernel(T* sink, int iters, T a, T b) {
  T x[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) x[c] = (T)(threadIdx.x + c) * (T)1e-3;
#pragma unroll 4
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < kChains; ++c) x[c] = fma(x[c], a, b);
  }
  T s = 0;
#pragma unroll
  for (int c = 0; c < kChains; ++c) s += x[c];
  sink[(size_t)blockIdx.x * kBlock + threadIdx.x] = s;
}

}  // namespace

extern "C" int ps_valu_probe(int kind, int blocks, int iters, void* sink, size_t sink_bytes, void* stream) {
  if ((kind != 0 && kind != 1) || blocks < 1 || iters < 1 || !sink)
    return ps_set_error(PS_ERR_INVALID, "ps_valu_probe: bad argument");
  const size_t need = (size_t)blocks * kBlock * (kind == 0 ? sizeof(float) : sizeof(double));
  if (sink_bytes < need)
    return ps_set_error(PS_ERR_INVALID, "ps_valu_probe: sink of %zu bytes, %zu needed", sink_bytes, need);
  hipStream_t st = (hipStream_t)stream;
  if (kind == 0)
    hipLaunchKernelGGL(valu_probe_kernel<float>, dim3(blocks), dim3(kBlock), 0, st, (float*)sink, iters, 0.999999f,
                       1e-6f);
  else
    hipLaunchKernelGGL(valu_probe_kernel<double>, dim3(blocks), dim3(kBlock), 0, st, (double*)sink, iters, 0.999999,
                       1e-6);
  PS_HIP_CHECK(hipGetLastError());
  return PS_OK;
}
