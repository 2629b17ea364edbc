// Vector-ALU throughput probe: independent fused multiply-add chains with no memory traffic, so that
// the FP64 and FP32 rates the stencil kernels are compared against are measured on the device rather
// than taken from a datasheet.
#include "gf_internal.h"

#include <algorithm>

namespace gf {

constexpr int kProbeChains = 8;   // independent chains per lane
constexpr int kProbeUnroll = 16;  // multiply-adds per chain per loop trip

// each lane runs kProbeChains chains of iters * kProbeUnroll dependent multiply-adds; the sum of the
// chains is stored so that none of the arithmetic is dead
template <typename T>
__global__ __launch_bounds__(256) void k_fma_probe(T *out, int iters, T a, T b) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  T v[kProbeChains];
#pragma unroll
  for (int c = 0; c < kProbeChains; ++c) v[c] = (T)(tid & 1023) * (T)1e-6 + (T)c;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int u = 0; u < kProbeUnroll; ++u)
#pragma unroll
      for (int c = 0; c < kProbeChains; ++c) v[c] = fma(v[c], a, b);
  }
  T s = 0;
#pragma unroll
  for (int c = 0; c < kProbeChains; ++c) s += v[c];
  out[tid] = s;
}

template <typename T>
static double fma_probe_t(hipStream_t s) {
  int dev = 0, ncu = 0;
  HIPCHK(hipGetDevice(&dev));
  HIPCHK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  const int blocks = 8 * std::max(ncu, 1), threads = 256, iters = 1000;
  DBuf<T> out;
  out.alloc((size_t)blocks * threads);
  // a = 1 - 2^-20, b = 2^-20: the chains stay bounded (they converge to 1)
  const T a = (T)(1.0 - 1.0 / 1048576.0), b = (T)(1.0 / 1048576.0);
  hipLaunchKernelGGL(k_fma_probe<T>, dim3(blocks), dim3(threads), 0, s, out.p, iters, a, b);
  HIPCHK(hipGetLastError());
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  HIPCHK(hipEventRecord(e0, s));
  hipLaunchKernelGGL(k_fma_probe<T>, dim3(blocks), dim3(threads), 0, s, out.p, iters, a, b);
  HIPCHK(hipGetLastError());
  HIPCHK(hipEventRecord(e1, s));
  HIPCHK(hipEventSynchronize(e1));
  float ms = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  const double flops = 2.0 * (double)blocks * threads * iters * kProbeUnroll * kProbeChains;
  return flops / (ms * 1e-3) / 1e12;
}

double fma_probe(bool fp64, hipStream_t s) { return fp64 ? fma_probe_t<double>(s) : fma_probe_t<float>(s); }

}  // namespace gf
