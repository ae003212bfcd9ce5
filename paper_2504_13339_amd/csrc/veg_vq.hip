// Decode of vector-quantised model attributes: trained models are stored with most
// parameters clustered into a codebook (paper, related work on compact Gaussian models);
// this expands the per-Gaussian codebook indices into the structure-of-arrays model the
// projection reads.
#include "veg_internal.h"

#include <cmath>

namespace veg {
namespace {

// One thread per Gaussian: its codeword row is split, in order, into the fields; an index
// outside the codebook writes NaN (a Gaussian with a non-finite attribute is culled).
__global__ __launch_bounds__(256) void vq_decode_kernel(const uint16_t* __restrict__ idx, int64_t n,
                                                        const float* __restrict__ book, int k, int dim,
                                                        VqFields fl) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const int r = idx[i];
    const bool ok = r < k;
    const float* row = book + (size_t)(ok ? r : 0) * dim;
    int c = 0;
    for (int f = 0; f < fl.n_fields; ++f) {
      const int w = fl.width[f];
      float* dst = fl.dst[f] + (size_t)i * w;
      for (int j = 0; j < w; ++j) dst[j] = ok ? row[c + j] : __builtin_nanf("");
      c += w;
    }
  }
}

}  // namespace

hipError_t launch_vq_decode(const uint16_t* idx, int64_t n, const float* book, int k, int dim, const VqFields& fl,
                            hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65535) blocks = 65535;
  hipLaunchKernelGGL(vq_decode_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, idx, n, book, k, dim, fl);
  return hipGetLastError();
}

}  // namespace veg
