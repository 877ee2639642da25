// Gradient of the Frobenius score at fixed positions (the adjoint of the
// tensor build, the window correlation, the local normalisation and the
// Frobenius norm of Sections 2, 3.2 and 3.4) with respect to the raw template
// and the image.  For L = sum_p gF_p F(x_p), C_alpha = w G_alpha,
// G_alpha = <tau_x f, T_alpha>, F = sqrt(sum_alpha mu_alpha C_alpha^2):
//
//   dC_alpha(p)    = gF_p mu_alpha C_alpha / F
//   dT_alpha(u)    = sum_p dC_alpha(p) w_p f(x_p + u - c)
//   df(x_p+u-c)   += w_p sum_alpha dC_alpha T_alpha(u)
//                    - w_p^3 m(u) (f - mu_p) sum_alpha dC_alpha G_alpha
//   (w = v^-1/2 with v = sum m (f - mu)^2, so dw/df = -w^3 m (f - mu))
//
// and, through T_alpha = sum_j coef_j,alpha m (g_j - mean_j) with
// coef = omega_j Q_j^alpha scale_j, scale_j = 1/sigma_j and g_j the template
// rotated by R_j (trilinear):
//
//   h_j(u)  = sum_alpha coef_j,alpha dT_alpha(u)
//   dg_j(u) = m(u) (h_j(u) - H1_j / M - (g_j(u) - mean_j) H2_j scale_j^2),
//   H1_j = sum_u m h_j, H2_j = sum_u m h_j (g_j - mean_j), M = sum m,
//
// then the trilinear weights of every sample scattered back to its corners.
// Window sums and the per-position quantities are float64; the rotation
// passes accumulate in float32 with float64 per-rotation sums.
#include <algorithm>

#include "ttm_device.h"
#include "ttm_internal.h"
#include "ttm_rotate.h"

namespace ttm {

namespace {

__device__ __forceinline__ double block_sum_d(double v, double* sh /* 4 */) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  return sh[0] + sh[1] + sh[2] + sh[3];
}

}  // namespace

// Per position (one 256-thread block): window mean, w, G_alpha in float64,
// then F, dC_alpha and a = sum_alpha dC_alpha G_alpha.  Positions outside
// the valid region, or with w = 0 or F = 0, get dC = 0.
__global__ void __launch_bounds__(256) k_grad_field(GradGeo g, const float* __restrict__ image,
                                                    const float* __restrict__ comps,
                                                    const float* __restrict__ mask, int order_n, int K,
                                                    const double* __restrict__ img_stats, float eps_v,
                                                    const int* __restrict__ pos, const float* __restrict__ grad_F,
                                                    double* __restrict__ wv, double* __restrict__ meanv,
                                                    double* __restrict__ dC, double* __restrict__ av) {
  __shared__ double sh[4];
  __shared__ double Gs[kMaxK];
  const int p = blockIdx.x, tid = threadIdx.x;
  const int x0 = pos[3 * p], x1 = pos[3 * p + 1], x2 = pos[3 * p + 2];
  const bool inside = x0 >= g.lo0 && x0 <= g.hi0 && x1 >= g.lo1 && x1 <= g.hi1 && x2 >= g.lo2 && x2 <= g.hi2;
  if (!inside) {
    for (int k = tid; k < K; k += 256) dC[(long)p * K + k] = 0.0;
    if (tid == 0) {
      wv[p] = 0.0;
      meanv[p] = 0.0;
      av[p] = 0.0;
    }
    return;
  }
  const int L0 = g.L0, L1 = g.L1, L2 = g.L2, nL = L0 * L1 * L2;
  const float* base = image + ((long)(x0 - L0 / 2) * g.n1 + (x1 - L1 / 2)) * g.n2 + (x2 - L2 / 2);
  auto img_at = [&](int u) -> double {
    const int u2 = u % L2, u1 = (u / L2) % L1, u0 = u / (L1 * L2);
    return (double)base[((long)u0 * g.n1 + u1) * g.n2 + u2];
  };
  double s0 = 0.0, s1 = 0.0;
  for (int u = tid; u < nL; u += 256) {
    const double mv = mask[u];
    if (mv != 0.0) {
      s0 += mv;
      s1 += mv * img_at(u);
    }
  }
  const double msum = block_sum_d(s0, sh);
  const double mean = block_sum_d(s1, sh) / msum;
  double s2 = 0.0;
  for (int u = tid; u < nL; u += 256) {
    const double mv = mask[u];
    if (mv != 0.0) {
      const double d = img_at(u) - mean;
      s2 += mv * d * d;
    }
  }
  const double var = block_sum_d(s2, sh);
  const double w = var > (double)eps_v * msum * img_stats[1] ? 1.0 / sqrt(var) : 0.0;
  for (int k = 0; k < K; ++k) {
    double acc = 0.0;
    const float* ck = comps + (long)k * nL;
    for (int u = tid; u < nL; u += 256) acc += img_at(u) * (double)ck[u];
    const double G = block_sum_d(acc, sh);
    if (tid == 0) Gs[k] = G;
  }
  __syncthreads();
  if (tid == 0) {
    double F2 = 0.0;
    for (int k = 0; k < K; ++k) {
      int al[4];
      alpha_of_dev(order_n, k, al);
      double mu = 1.0;
      for (int i = 2; i <= order_n; ++i) mu *= i;
      for (int d = 0; d < 4; ++d)
        for (int i = 2; i <= al[d]; ++i) mu /= i;
      const double C = w * Gs[k];
      F2 += mu * C * C;
    }
    const double F = sqrt(F2);
    const bool ok = w > 0.0 && F > 0.0;
    double a = 0.0;
    for (int k = 0; k < K; ++k) {
      int al[4];
      alpha_of_dev(order_n, k, al);
      double mu = 1.0;
      for (int i = 2; i <= order_n; ++i) mu *= i;
      for (int d = 0; d < 4; ++d)
        for (int i = 2; i <= al[d]; ++i) mu /= i;
      const double d = ok ? (double)grad_F[p] * mu * w * Gs[k] / F : 0.0;
      dC[(long)p * K + k] = d;
      a += d * Gs[k];
    }
    wv[p] = ok ? w : 0.0;
    meanv[p] = mean;
    av[p] = a;
  }
}

// dT_alpha(u) = sum_p dC_alpha(p) w_p f(x_p + u - c): one thread per (alpha, u)
__global__ void __launch_bounds__(256) k_grad_dT(GradGeo g, const float* __restrict__ image, int K,
                                                 const int* __restrict__ pos, int n_pos,
                                                 const double* __restrict__ wv, const double* __restrict__ dC,
                                                 float* __restrict__ dT) {
  const int L0 = g.L0, L1 = g.L1, L2 = g.L2, nL = L0 * L1 * L2;
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long)K * nL) return;
  const int k = (int)(i / nL), u = (int)(i % nL);
  const int u2 = u % L2, u1 = (u / L2) % L1, u0 = u / (L1 * L2);
  double acc = 0.0;
  for (int p = 0; p < n_pos; ++p) {
    const double wd = wv[p] * dC[(long)p * K + k];
    if (wd == 0.0) continue;
    const long y0 = pos[3 * p] + u0 - L0 / 2, y1 = pos[3 * p + 1] + u1 - L1 / 2, y2 = pos[3 * p + 2] + u2 - L2 / 2;
    acc += wd * (double)image[(y0 * g.n1 + y1) * g.n2 + y2];
  }
  dT[i] = (float)acc;
}

// image gradient on the windows (grad_image zeroed beforehand; overlapping
// windows add): grid (n_pos, ceil(L^3 / 256))
__global__ void __launch_bounds__(256) k_grad_image(GradGeo g, const float* __restrict__ image,
                                                    const float* __restrict__ comps,
                                                    const float* __restrict__ mask, int K,
                                                    const int* __restrict__ pos, const double* __restrict__ wv,
                                                    const double* __restrict__ meanv,
                                                    const double* __restrict__ dC, const double* __restrict__ av,
                                                    float* __restrict__ grad_image) {
  const int p = blockIdx.x;
  const double w = wv[p];
  if (!(w > 0.0)) return;
  const int L0 = g.L0, L1 = g.L1, L2 = g.L2, nL = L0 * L1 * L2;
  const int u = blockIdx.y * 256 + threadIdx.x;
  if (u >= nL) return;
  const int u2 = u % L2, u1 = (u / L2) % L1, u0 = u / (L1 * L2);
  const long y = ((long)(pos[3 * p] + u0 - L0 / 2) * g.n1 + (pos[3 * p + 1] + u1 - L1 / 2)) * g.n2 +
                 (pos[3 * p + 2] + u2 - L2 / 2);
  double b = 0.0;
  for (int k = 0; k < K; ++k) b += dC[(long)p * K + k] * (double)comps[(long)k * nL + u];
  const double d = w * b - w * w * w * (double)mask[u] * ((double)image[y] - meanv[p]) * av[p];
  if (d != 0.0) atomicAdd(grad_image + y, (float)d);
}

// Pass A over (voxel tile, rotation chunk): per rotation j the partial sums
// over this tile of m h_j and m h_j g_j.  Each thread holds its voxel's dT in
// registers; the rotations' coefficients are uniform across the block.
template <int N>
__global__ void __launch_bounds__(256) k_grad_rot_sums(GradGeo g, const float* __restrict__ tmpl,
                                                       const float* __restrict__ mask,
                                                       const float* __restrict__ quats,
                                                       const double* __restrict__ coef, int nrot, int jchunk,
                                                       const float* __restrict__ dT,
                                                       double* __restrict__ part /* [ntiles][nrot][2] */) {
  constexpr int K = (N + 1) * (N + 2) * (N + 3) / 6;
  __shared__ double red[4][2];
  const int L0 = g.L0, L1 = g.L1, L2 = g.L2, nL = L0 * L1 * L2;
  const int tile = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int u = tile * 256 + tid;
  const bool on = u < nL;
  float d[K];
#pragma unroll
  for (int k = 0; k < K; ++k) d[k] = on ? dT[(long)k * nL + u] : 0.0f;
  const float mv = on ? mask[u] : 0.0f;
  const int u2 = on ? u % L2 : 0, u1 = on ? (u / L2) % L1 : 0, u0 = on ? u / (L1 * L2) : 0;
  const int j0 = blockIdx.y * jchunk, j1 = min(nrot, j0 + jchunk);
  for (int j = j0; j < j1; ++j) {
    float h = 0.0f;
    const double* cj = coef + (long)j * K;
#pragma unroll
    for (int k = 0; k < K; ++k) h += (float)cj[k] * d[k];
    float mh = 0.0f, mhg = 0.0f;
    if (on && mv != 0.0f) {
      const Rot R = quat_rot(quats + 4 * j);
      const float gv = sample_rotated(tmpl, L0, L1, L2, R, u0, u1, u2);
      mh = mv * h;
      mhg = mh * gv;
    }
    double a = mh, b = mhg;
    for (int off = 32; off > 0; off >>= 1) {
      a += __shfl_xor(a, off);
      b += __shfl_xor(b, off);
    }
    __syncthreads();
    if (lane == 0) {
      red[wave][0] = a;
      red[wave][1] = b;
    }
    __syncthreads();
    if (tid == 0) {
      double* o = part + ((long)tile * nrot + j) * 2;
      o[0] = red[0][0] + red[1][0] + red[2][0] + red[3][0];
      o[1] = red[0][1] + red[1][1] + red[2][1] + red[3][1];
    }
  }
}

// H1_j = sum over tiles, H2_j = sum of (m h g) - mean_j H1_j
__global__ void k_grad_rot_reduce(const double* __restrict__ part, int ntiles, int nrot,
                                  const double* __restrict__ rstats, double* __restrict__ H) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nrot) return;
  double a = 0.0, b = 0.0;
  for (int t = 0; t < ntiles; ++t) {
    a += part[((long)t * nrot + j) * 2];
    b += part[((long)t * nrot + j) * 2 + 1];
  }
  H[2 * j] = a;
  H[2 * j + 1] = b - rstats[2 * j] * a;
}

// Pass B: dg_j(u) scattered through the trilinear weights into an LDS copy of
// the template gradient (L^3 <= kGradLdsCap floats), flushed with atomics.
constexpr int kGradLdsCap = kGradMaxTemplate;
template <int N>
__global__ void __launch_bounds__(256) k_grad_rot_scatter(GradGeo g, const float* __restrict__ tmpl,
                                                          const float* __restrict__ mask,
                                                          const float* __restrict__ quats,
                                                          const double* __restrict__ coef,
                                                          const double* __restrict__ rstats,
                                                          const double* __restrict__ H,
                                                          const double* __restrict__ stats, int nrot,
                                                          int jchunk, const float* __restrict__ dT,
                                                          float* __restrict__ grad_tmpl) {
  constexpr int K = (N + 1) * (N + 2) * (N + 3) / 6;
  __shared__ float acc[kGradLdsCap];
  const int L0 = g.L0, L1 = g.L1, L2 = g.L2, nL = L0 * L1 * L2;
  const int tile = blockIdx.x, tid = threadIdx.x;
  for (int i = tid; i < nL; i += 256) acc[i] = 0.0f;
  __syncthreads();
  const int u = tile * 256 + tid;
  const bool on = u < nL;
  float d[K];
#pragma unroll
  for (int k = 0; k < K; ++k) d[k] = on ? dT[(long)k * nL + u] : 0.0f;
  const float mv = on ? mask[u] : 0.0f;
  const int u2 = on ? u % L2 : 0, u1 = on ? (u / L2) % L1 : 0, u0 = on ? u / (L1 * L2) : 0;
  const int c0 = L0 / 2, c1 = L1 / 2, c2 = L2 / 2;
  const int j0 = blockIdx.y * jchunk, j1 = min(nrot, j0 + jchunk);
  const double msum = stats[2];
  if (on && mv != 0.0f) {
    for (int j = j0; j < j1; ++j) {
      const double sc = rstats[2 * j + 1];
      if (sc == 0.0) continue;
      float h = 0.0f;
      const double* cj = coef + (long)j * K;
#pragma unroll
      for (int k = 0; k < K; ++k) h += (float)cj[k] * d[k];
      const Rot R = quat_rot(quats + 4 * j);
      const float gv = sample_rotated(tmpl, L0, L1, L2, R, u0, u1, u2);
      const float dg = mv * (h - (float)(H[2 * j] / msum) - (gv - (float)rstats[2 * j]) * (float)(H[2 * j + 1] * sc * sc));
      // the sample's position and trilinear weights, as in sample_rotated
      const float v0 = (float)(u0 - c0), v1 = (float)(u1 - c1), v2 = (float)(u2 - c2);
      const float p0 = c0 + R.r[0] * v0 + R.r[3] * v1 + R.r[6] * v2;
      const float p1 = c1 + R.r[1] * v0 + R.r[4] * v1 + R.r[7] * v2;
      const float p2 = c2 + R.r[2] * v0 + R.r[5] * v1 + R.r[8] * v2;
      const float f0 = floorf(p0), f1 = floorf(p1), f2 = floorf(p2);
      const int i0 = (int)f0, i1 = (int)f1, i2 = (int)f2;
      const float w0 = p0 - f0, w1 = p1 - f1, w2 = p2 - f2;
#pragma unroll
      for (int e0 = 0; e0 < 2; ++e0) {
        const int k0 = i0 + e0;
        if (k0 < 0 || k0 >= L0) continue;
        const float a0 = e0 ? w0 : 1.0f - w0;
#pragma unroll
        for (int e1 = 0; e1 < 2; ++e1) {
          const int k1 = i1 + e1;
          if (k1 < 0 || k1 >= L1) continue;
          const float a1 = a0 * (e1 ? w1 : 1.0f - w1);
#pragma unroll
          for (int e2 = 0; e2 < 2; ++e2) {
            const int k2 = i2 + e2;
            if (k2 < 0 || k2 >= L2) continue;
            atomicAdd(&acc[(k0 * L1 + k1) * L2 + k2], a1 * (e2 ? w2 : 1.0f - w2) * dg);
          }
        }
      }
    }
  }
  __syncthreads();
  for (int i = tid; i < nL; i += 256) {
    const float v = acc[i];
    if (v != 0.0f) atomicAdd(grad_tmpl + i, v);
  }
}

hipError_t launch_grad_field(const GradGeo& g, const float* image, const float* comps, const float* mask,
                             int order_n, const double* img_stats, float eps_v, const int* pos, int n_pos,
                             const float* grad_F, const GradWs& w, hipStream_t s) {
  const int K = num_components(order_n);
  hipLaunchKernelGGL(k_grad_field, dim3((unsigned)n_pos), dim3(256), 0, s, g, image, comps, mask, order_n, K,
                     img_stats, eps_v, pos, grad_F, w.wv, w.mean, w.dC, w.a);
  return hipGetLastError();
}

hipError_t launch_grad_image(const GradGeo& g, const float* image, const float* comps, const float* mask,
                             int order_n, const int* pos, int n_pos, const GradWs& w, float* grad_image,
                             hipStream_t s) {
  const int K = num_components(order_n);
  const int nL = g.L0 * g.L1 * g.L2;
  hipLaunchKernelGGL(k_grad_image, dim3((unsigned)n_pos, (unsigned)((nL + 255) / 256)), dim3(256), 0, s, g,
                     image, comps, mask, K, pos, w.wv, w.mean, w.dC, w.a, grad_image);
  return hipGetLastError();
}

template <int N>
static hipError_t grad_tmpl_n(const GradGeo& g, const float* image, const float* tmpl, const float* mask,
                              const float* quats, int nrot, const double* coef, const double* rstats,
                              const double* stats, const int* pos, int n_pos, const GradWs& w, float* grad_tmpl,
                              hipStream_t s) {
  constexpr int K = (N + 1) * (N + 2) * (N + 3) / 6;
  const int nL = g.L0 * g.L1 * g.L2;
  hipLaunchKernelGGL(k_grad_dT, dim3((unsigned)(((long)K * nL + 255) / 256)), dim3(256), 0, s, g, image, K, pos,
                     n_pos, w.wv, w.dC, w.dT);
  const int ntiles = (nL + 255) / 256;
  const int nchunks = std::max(1, std::min(nrot, 512 / ntiles));
  const int jchunk = (nrot + nchunks - 1) / nchunks;
  hipLaunchKernelGGL((k_grad_rot_sums<N>), dim3((unsigned)ntiles, (unsigned)nchunks), dim3(256), 0, s, g, tmpl,
                     mask, quats, coef, nrot, jchunk, w.dT, w.part);
  hipLaunchKernelGGL(k_grad_rot_reduce, dim3((unsigned)((nrot + 255) / 256)), dim3(256), 0, s, w.part, ntiles,
                     nrot, rstats, w.H);
  hipLaunchKernelGGL((k_grad_rot_scatter<N>), dim3((unsigned)ntiles, (unsigned)nchunks), dim3(256), 0, s, g,
                     tmpl, mask, quats, coef, rstats, w.H, stats, nrot, jchunk, w.dT, grad_tmpl);
  return hipGetLastError();
}

hipError_t launch_grad_tmpl(const GradGeo& g, const float* image, const float* tmpl, const float* mask,
                            int order_n, const float* quats, int nrot, const double* coef, const double* rstats,
                            const double* stats, const int* pos, int n_pos, const GradWs& w, float* grad_tmpl,
                            hipStream_t s) {
  if ((long)g.L0 * g.L1 * g.L2 > kGradLdsCap) return hipErrorInvalidValue;
  switch (order_n) {
    case 2: return grad_tmpl_n<2>(g, image, tmpl, mask, quats, nrot, coef, rstats, stats, pos, n_pos, w, grad_tmpl, s);
    case 4: return grad_tmpl_n<4>(g, image, tmpl, mask, quats, nrot, coef, rstats, stats, pos, n_pos, w, grad_tmpl, s);
    case 6: return grad_tmpl_n<6>(g, image, tmpl, mask, quats, nrot, coef, rstats, stats, pos, n_pos, w, grad_tmpl, s);
    case 8: return grad_tmpl_n<8>(g, image, tmpl, mask, quats, nrot, coef, rstats, stats, pos, n_pos, w, grad_tmpl, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace ttm
