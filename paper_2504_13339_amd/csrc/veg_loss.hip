// L1 image loss and its gradient (paper, section "Training": the image loss mixes L1 and
// SSIM; this is the L1 term).
#include "veg_internal.h"

namespace veg {
namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ double wave_sum_f64(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

__global__ __launch_bounds__(kThreads) void l1_kernel(const float* __restrict__ img, const float* __restrict__ tgt,
                                                      int64_t n, float scale, double* __restrict__ loss,
                                                      float* __restrict__ dimg) {
  __shared__ double s_part[kThreads / 64];
  double acc = 0.0;
  const int64_t stride = (int64_t)gridDim.x * kThreads;
  const bool vec = (n & 3) == 0 && ((reinterpret_cast<uintptr_t>(img) | reinterpret_cast<uintptr_t>(tgt) |
                                       reinterpret_cast<uintptr_t>(dimg)) & 15u) == 0;
  if (vec) {   // 16-byte loads and stores: four elements per lane and instruction
    const float4* img4 = reinterpret_cast<const float4*>(img);
    const float4* tgt4 = reinterpret_cast<const float4*>(tgt);
    float4* dimg4 = reinterpret_cast<float4*>(dimg);
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n / 4; i += stride) {
      const float4 a = img4[i], b = tgt4[i];
      const float d[4] = {a.x - b.x, a.y - b.y, a.z - b.z, a.w - b.w};
      float g[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        acc += (double)fabsf(d[k]);
        g[k] = d[k] > 0.0f ? scale : (d[k] < 0.0f ? -scale : 0.0f);
      }
      dimg4[i] = make_float4(g[0], g[1], g[2], g[3]);
    }
  } else {
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += stride) {
      const float d = img[i] - tgt[i];
      acc += (double)fabsf(d);
      dimg[i] = d > 0.0f ? scale : (d < 0.0f ? -scale : 0.0f);
    }
  }
  acc = wave_sum_f64(acc);
  if ((threadIdx.x & 63) == 0) s_part[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int k = 0; k < kThreads / 64; ++k) t += s_part[k];
    if (t != 0.0) unsafeAtomicAdd(loss, t * (double)scale);
  }
}

}  // namespace

hipError_t launch_l1(const float* image, const float* target, int64_t count, float scale, double* loss, float* dimage,
                     hipStream_t stream) {
  if (count <= 0) return hipSuccess;
  int64_t blocks = (count + kThreads * 8 - 1) / (kThreads * 8);
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL(l1_kernel, dim3((unsigned)blocks), dim3(kThreads), 0, stream, image, target, count, scale, loss,
                     dimage);
  return hipGetLastError();
}

}  // namespace veg
