// Tensor template construction (Section 3.2) and the rotated, normalised
// templates of classical matching (Algorithm 1).
//
//   s_j(u) = m(u) (g_j(u) - mean_j) scale_j,  g_j(u) = t(c + R_j^-1 (u - c))
//   mean_j = <g_j, m> / m_sum,  scale_j = 1 / sqrt(<g_j^2, m> - <g_j, m>^2 / m_sum)
//   T_alpha(u) = sum_j omega_j Q_j^alpha s_j(u)
//
// Rotation R(Q) of Q = (a,b,c,d): the active Hamilton rotation v -> Q v Q*,
// vector part on axes (0,1,2).  Sampling is trilinear with zero outside the
// box.  Masked sums and the tensor accumulation are float64.
#include "ttm_device.h"
#include "ttm_internal.h"
#include "ttm_rotate.h"

namespace ttm {

// ----------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_rot_stats(const float* __restrict__ t, const float* __restrict__ m,
                                                   int L0, int L1, int L2, const float* __restrict__ quats,
                                                   double* __restrict__ rstats) {
  __shared__ double sh[3 * 256];
  const int j = blockIdx.x;
  const Rot R = quat_rot(quats + 4 * j);
  const int n = L0 * L1 * L2;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  for (int u = threadIdx.x; u < n; u += blockDim.x) {
    const float mv = m[u];
    if (mv == 0.0f) continue;
    const int u2 = u % L2, u1 = (u / L2) % L1, u0 = u / (L1 * L2);
    const double gv = sample_rotated(t, L0, L1, L2, R, u0, u1, u2);
    s0 += mv;
    s1 += mv * gv;
    s2 += mv * gv * gv;
  }
  const int tid = threadIdx.x;
  sh[tid] = s0; sh[256 + tid] = s1; sh[512 + tid] = s2;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) {
      sh[tid] += sh[tid + s];
      sh[256 + tid] += sh[256 + tid + s];
      sh[512 + tid] += sh[512 + tid + s];
    }
    __syncthreads();
  }
  if (tid == 0) {
    const double msum = sh[0], a1 = sh[256], a2 = sh[512];
    const double mean = msum > 0.0 ? a1 / msum : 0.0;
    const double var = msum > 0.0 ? a2 - a1 * a1 / msum : 0.0;
    rstats[2 * j] = mean;
    rstats[2 * j + 1] = (var > 1e-12 * (a2 > 0.0 ? a2 : 1.0)) ? 1.0 / sqrt(var) : 0.0;
  }
}

// The same statistics with the template box held in LDS (the padded layout
// of sample_rotated_lds): one 1024-thread block takes kStatRots rotations in
// turn, so the box is loaded once for all of them.
constexpr int kStatRots = 16;

__global__ void __launch_bounds__(1024) k_rot_stats_lds(const float* __restrict__ t, const float* __restrict__ m,
                                                        int L0, int L1, int L2, const float* __restrict__ quats,
                                                        int nrot, double* __restrict__ rstats) {
  extern __shared__ float tl[];
  __shared__ double red[3][16];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int P2 = ncc_lds_p2(L2), P01 = ncc_lds_p01(L1, L2);
  fill_lds_box(tl, t, L0, L1, L2, P2, P01, tid, 1024);
  __syncthreads();
  const int n = L0 * L1 * L2;
  for (int jj = 0; jj < kStatRots; ++jj) {
    const int j = blockIdx.x * kStatRots + jj;
    if (j >= nrot) break;
    const Rot R = quat_rot(quats + 4 * j);
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int u = tid; u < n; u += 1024) {
      const float mv = m[u];
      if (mv == 0.0f) continue;
      const int u2 = u % L2, u1 = (u / L2) % L1, u0 = u / (L1 * L2);
      const double gv = sample_rotated_lds<false>(tl, L0, L1, L2, P2, P01, R, u0, u1, u2);
      s0 += mv;
      s1 += mv * gv;
      s2 += mv * gv * gv;
    }
    for (int off = 32; off > 0; off >>= 1) {
      s0 += __shfl_xor(s0, off);
      s1 += __shfl_xor(s1, off);
      s2 += __shfl_xor(s2, off);
    }
    if (lane == 0) {
      red[0][wave] = s0;
      red[1][wave] = s1;
      red[2][wave] = s2;
    }
    __syncthreads();
    if (tid == 0) {
      double msum = 0.0, a1 = 0.0, a2 = 0.0;
      for (int w = 0; w < 16; ++w) {
        msum += red[0][w];
        a1 += red[1][w];
        a2 += red[2][w];
      }
      const double mean = msum > 0.0 ? a1 / msum : 0.0;
      const double var = msum > 0.0 ? a2 - a1 * a1 / msum : 0.0;
      rstats[2 * j] = mean;
      rstats[2 * j + 1] = (var > 1e-12 * (a2 > 0.0 ? a2 : 1.0)) ? 1.0 / sqrt(var) : 0.0;
    }
    __syncthreads();
  }
}

hipError_t launch_rot_stats(const float* tmpl, const float* mask, int L0, int L1, int L2,
                            const float* quats, int nrot, double* rstats, hipStream_t s) {
  const long lds = ncc_lds_floats(L0, L1, L2);
  if (lds <= kNccLdsCap) {
    hipLaunchKernelGGL(k_rot_stats_lds, dim3((unsigned)((nrot + kStatRots - 1) / kStatRots)), dim3(1024),
                       sizeof(float) * lds, s, tmpl, mask, L0, L1, L2, quats, nrot, rstats);
  } else {
    hipLaunchKernelGGL(k_rot_stats, dim3(nrot), dim3(256), 0, s, tmpl, mask, L0, L1, L2, quats, rstats);
  }
  return hipGetLastError();
}

// ----------------------------------------------------------------------------
__device__ __forceinline__ double ipow(double x, int e) {
  double r = 1.0;
  for (int i = 0; i < e; ++i) r *= x;
  return r;
}

__global__ void k_build_coef(const float* __restrict__ quats, const double* __restrict__ weights,
                             const double* __restrict__ rstats, int nrot, int order_n, int K,
                             double* __restrict__ coef) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long)nrot * K) return;
  const int j = (int)(i / K), k = (int)(i % K);
  int al[4];
  alpha_of_dev(order_n, k, al);
  double q[4] = {quats[4 * j], quats[4 * j + 1], quats[4 * j + 2], quats[4 * j + 3]};
  const double nrm = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  double mono = 1.0;
  for (int d = 0; d < 4; ++d) mono *= ipow(q[d] / nrm, al[d]);
  coef[i] = weights[j] * mono * rstats[2 * j + 1];
}

hipError_t launch_build_coef(const float* quats, const double* weights, const double* rstats,
                             int nrot, int order_n, double* coef, hipStream_t s) {
  const int K = num_components(order_n);
  const long n = (long)nrot * K;
  hipLaunchKernelGGL(k_build_coef, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, quats, weights,
                     rstats, nrot, order_n, K, coef);
  return hipGetLastError();
}

__global__ void k_multiplicities(int order_n, int K, float* mu) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  int al[4];
  alpha_of_dev(order_n, k, al);
  double f = 1.0;
  for (int i = 2; i <= order_n; ++i) f *= i;
  for (int d = 0; d < 4; ++d)
    for (int i = 2; i <= al[d]; ++i) f /= i;
  mu[k] = (float)f;
}

hipError_t launch_multiplicities(int order_n, float* mu, hipStream_t s) {
  const int K = num_components(order_n);
  hipLaunchKernelGGL(k_multiplicities, dim3((K + 255) / 256), dim3(256), 0, s, order_n, K, mu);
  return hipGetLastError();
}

// ----------------------------------------------------------------------------
// T_alpha(u) for a chunk of KC components (blockIdx.y selects the chunk)
constexpr int kKC = 36;

__global__ void k_rot_table(const float* __restrict__ quats, int nrot, float* __restrict__ rtab) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nrot) return;
  const Rot R = quat_rot(quats + 4 * j);
  for (int i = 0; i < 9; ++i) rtab[9 * j + i] = R.r[i];
}

__global__ void __launch_bounds__(256) k_build_accum(const float* __restrict__ t, const float* __restrict__ m,
                                                     int L0, int L1, int L2, const float* __restrict__ rtab,
                                                     const double* __restrict__ rstats,
                                                     const double* __restrict__ coef, int nrot, int K,
                                                     float* __restrict__ comps) {
  const int n = L0 * L1 * L2;
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  const int k0 = blockIdx.y * kKC;
  const int kc = min(kKC, K - k0);
  double acc[kKC];
#pragma unroll
  for (int i = 0; i < kKC; ++i) acc[i] = 0.0;
  float mv = 0.0f;
  int u0 = 0, u1 = 0, u2 = 0;
  if (u < n) {
    mv = m[u];
    u2 = u % L2; u1 = (u / L2) % L1; u0 = u / (L1 * L2);
  }
  if (mv != 0.0f) {
#pragma unroll 1
    for (int j = 0; j < nrot; ++j) {
      Rot R;
#pragma unroll
      for (int i = 0; i < 9; ++i) R.r[i] = rtab[9 * j + i];
      const double g = sample_rotated(t, L0, L1, L2, R, u0, u1, u2);
      const double sv = (double)mv * (g - rstats[2 * j]);
      const double* cj = coef + (long)j * K + k0;
#pragma unroll
      for (int i = 0; i < kKC; ++i)
        if (i < kc) acc[i] += cj[i] * sv;
    }
  }
  if (u < n) {
#pragma unroll
    for (int i = 0; i < kKC; ++i)
      if (i < kc) comps[(long)(k0 + i) * n + u] = (float)acc[i];
  }
}

// The same sum as a matrix product on the matrix cores: T[alpha][u] =
// sum_j coef[j][alpha] S[j][u], S[j][u] = m(u) (g_j(u) - mean_j), with
// v_mfma_f64_16x16x4f64 (float64 in and out).  One wavefront owns 16
// positions u and all components (NT tiles of 16); each step takes four
// rotations: every lane samples its own S[j][u] (the B operand, j = j0 +
// lane / 16, u = lane % 16) and loads coef[j][alpha] (the A operand, alpha =
// 16 t + lane % 16), then one MFMA per component tile.  Result lane l,
// register i holds alpha = 16 t + 4 i + l / 16 at u = l % 16.  Tiles of 16
// positions that lie wholly outside the mask are skipped (S = 0 there).
typedef double d4_t __attribute__((ext_vector_type(4)));

// LDS = true: the template box is staged in LDS (padded layout) by the
// block's 512 threads, 8 wavefronts of 16 positions each.
template <int NT, bool LDS>
__global__ void __launch_bounds__(LDS ? 512 : 256) k_build_mfma(const float* __restrict__ t,
                                                                const float* __restrict__ m, int L0, int L1,
                                                                int L2, const float* __restrict__ rtab,
                                                                const double* __restrict__ rstats,
                                                                const double* __restrict__ coef, int nrot, int K,
                                                                float* __restrict__ comps) {
  extern __shared__ float tl[];
  constexpr int WPB = LDS ? 8 : 4;   // wavefronts (tiles) per block
  const int P2 = ncc_lds_p2(L2), P01 = ncc_lds_p01(L1, L2);
  if (LDS) {
    fill_lds_box(tl, t, L0, L1, L2, P2, P01, threadIdx.x, 64 * WPB);
    __syncthreads();
  }
  const int n = L0 * L1 * L2;
  const int lane = threadIdx.x & 63;
  const int tile = blockIdx.x * WPB + (threadIdx.x >> 6);
  const int u = tile * 16 + (lane & 15);
  const int jl = lane >> 4;
  const bool uin = u < n;
  const float mv = uin ? m[uin ? u : 0] : 0.0f;
  int u0 = 0, u1 = 0, u2 = 0;
  if (uin) {
    u2 = u % L2; u1 = (u / L2) % L1; u0 = u / (L1 * L2);
  }
  d4_t acc[NT];
#pragma unroll
  for (int tt = 0; tt < NT; ++tt) acc[tt] = d4_t{0.0, 0.0, 0.0, 0.0};
  // the whole wavefront skips a tile with no masked position
  if (__any(mv != 0.0f)) {
#pragma unroll 1
    for (int j0 = 0; j0 < nrot; j0 += 4) {
      const int j = j0 + jl;
      const bool jin = j < nrot;
      double sv = 0.0;
      if (jin && mv != 0.0f) {
        Rot R;
#pragma unroll
        for (int i = 0; i < 9; ++i) R.r[i] = rtab[9 * j + i];
        const double g = LDS ? (double)sample_rotated_lds<false>(tl, L0, L1, L2, P2, P01, R, u0, u1, u2)
                             : (double)sample_rotated(t, L0, L1, L2, R, u0, u1, u2);
        sv = (double)mv * (g - rstats[2 * j]);
      }
      const double* cj = coef + (long)(jin ? j : 0) * K;
#pragma unroll
      for (int tt = 0; tt < NT; ++tt) {
        const int al = 16 * tt + (lane & 15);
        const double cv = cj[al < K ? al : 0];
        const double a = jin && al < K ? cv : 0.0;
        acc[tt] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, sv, acc[tt], 0, 0, 0);
      }
    }
  }
  if (uin) {
#pragma unroll
    for (int tt = 0; tt < NT; ++tt)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int al = 16 * tt + 4 * i + jl;
        if (al < K) comps[(long)al * n + u] = (float)acc[tt][i];
      }
  }
}

hipError_t launch_build_accum(const float* tmpl, const float* mask, int L0, int L1, int L2,
                              const float* quats, const double* rstats, const double* coef,
                              int nrot, int K, float* comps, float* rtab, hipStream_t s) {
  const int n = L0 * L1 * L2;
  hipLaunchKernelGGL(k_rot_table, dim3((nrot + 255) / 256), dim3(256), 0, s, quats, nrot, rtab);
  const int nt = (K + 15) / 16;
  const long lds = ncc_lds_floats(L0, L1, L2);
  const bool use_lds = lds <= kNccLdsCap;
  const dim3 grid((unsigned)(use_lds ? (n + 127) / 128 : (n + 63) / 64));
#define TTM_BUILD(NT)                                                                                          \
  if (use_lds)                                                                                                 \
    hipLaunchKernelGGL((k_build_mfma<NT, true>), grid, dim3(512), sizeof(float) * lds, s, tmpl, mask, L0, L1, L2, \
                       rtab, rstats, coef, nrot, K, comps);                                                    \
  else                                                                                                         \
    hipLaunchKernelGGL((k_build_mfma<NT, false>), grid, dim3(256), 0, s, tmpl, mask, L0, L1, L2, rtab, rstats,   \
                       coef, nrot, K, comps)
  switch (nt) {
    case 1: TTM_BUILD(1); break;
    case 3: TTM_BUILD(3); break;
    case 6: TTM_BUILD(6); break;
    case 11: TTM_BUILD(11); break;
    default: {
      dim3 g2((unsigned)((n + 255) / 256), (unsigned)((K + kKC - 1) / kKC));
      hipLaunchKernelGGL(k_build_accum, g2, dim3(256), 0, s, tmpl, mask, L0, L1, L2, rtab, rstats, coef, nrot,
                         K, comps);
    }
  }
#undef TTM_BUILD
  return hipGetLastError();
}

// ----------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_rot_write(const float* __restrict__ t, const float* __restrict__ m,
                                                   int L0, int L1, int L2, const float* __restrict__ quats,
                                                   const double* __restrict__ rstats, int j0,
                                                   float* __restrict__ out) {
  const int n = L0 * L1 * L2;
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y;
  const int j = j0 + b;
  if (u >= n) return;
  const float mv = m[u];
  float v = 0.0f;
  if (mv != 0.0f) {
    const Rot R = quat_rot(quats + 4 * j);
    const int u2 = u % L2, u1 = (u / L2) % L1, u0 = u / (L1 * L2);
    const double g = sample_rotated(t, L0, L1, L2, R, u0, u1, u2);
    v = (float)((double)mv * (g - rstats[2 * j]) * rstats[2 * j + 1]);
  }
  out[(long)b * n + u] = v;
}

hipError_t launch_rot_write(const float* tmpl, const float* mask, int L0, int L1, int L2,
                            const float* quats, const double* rstats, int j0, int nb, float* out,
                            hipStream_t s) {
  const int n = L0 * L1 * L2;
  dim3 grid((unsigned)((n + 255) / 256), (unsigned)nb);
  hipLaunchKernelGGL(k_rot_write, grid, dim3(256), 0, s, tmpl, mask, L0, L1, L2, quats, rstats, j0, out);
  return hipGetLastError();
}

}  // namespace ttm
