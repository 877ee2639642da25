// Isotropic low-pass filter of Section 2 (matching is applied to f * h and
// t * h, with h * 1 = 1): a sampled Gaussian, separable, applied one axis at a
// time, out(x) = sum_k h(k) in(x - k), indices modulo the extent (periodic, as
// the FFT correlation treats the image) or with zeros outside (the template
// box).  Float32 with float32 accumulation over at most 2 * 32 + 1 taps.
#include <algorithm>
#include <cmath>

#include "ttm_device.h"
#include "ttm_internal.h"

namespace ttm {

__global__ void __launch_bounds__(256) k_lowpass_axis(const float* __restrict__ in, float* __restrict__ out,
                                                      long total, int n_axis, long stride, int periodic,
                                                      FilterTaps taps) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (long)gridDim.x * blockDim.x) {
    const int x = (int)((i / stride) % n_axis);
    const long base = i - (long)x * stride;
    float acc = 0.0f;
    for (int k = -taps.R; k <= taps.R; ++k) {
      int s = x - k;
      if (periodic) {
        s %= n_axis;
        if (s < 0) s += n_axis;
      } else if (s < 0 || s >= n_axis) {
        continue;
      }
      acc += taps.h[k + taps.R] * in[base + (long)s * stride];
    }
    out[i] = acc;
  }
}

hipError_t launch_lowpass(const float* in, float* out, float* tmp_a, float* tmp_b, int n0, int n1, int n2,
                          int periodic, const FilterTaps& taps, hipStream_t s) {
  const long total = (long)n0 * n1 * n2;
  const unsigned nb = (unsigned)std::min<long>((total + 255) / 256, 8192);
  hipLaunchKernelGGL(k_lowpass_axis, dim3(nb), dim3(256), 0, s, in, tmp_a, total, n2, 1L, periodic, taps);
  hipLaunchKernelGGL(k_lowpass_axis, dim3(nb), dim3(256), 0, s, tmp_a, tmp_b, total, n1, (long)n2, periodic,
                     taps);
  hipLaunchKernelGGL(k_lowpass_axis, dim3(nb), dim3(256), 0, s, tmp_b, out, total, n0, (long)n1 * n2, periodic,
                     taps);
  return hipGetLastError();
}

}  // namespace ttm
