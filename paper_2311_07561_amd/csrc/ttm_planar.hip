// Two-dimensional TTM (Sections 2 and 3 with d = 2): the small kernels that
// connect the planar entry points to the volume passes.
//
// A plane rotation is described by the unit complex number z = (a, b) of half
// its angle; as a quaternion it is (a, b, 0, 0), the rotation about axis 0, so
// a template box of depth 1 rotated by it is the planar template rotated
// bilinearly.  The planar tensor C_n in S^n(R^2) has the n + 1 entries of the
// multi-indices (n - k, k), which are the entries (n - k, k, 0, 0) of the
// volume tensor; all other volume entries vanish for such rotations.  A stack
// of B images is a volume [B][n1][n2] correlated with a depth-1 template, so
// the planes never mix.
#include "ttm_internal.h"

namespace ttm {

// quats[j] = (a_j, b_j, 0, 0)
__global__ void k_planar_quats(const float* __restrict__ z, int nrot, float* __restrict__ quats) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nrot) return;
  quats[4 * j] = z[2 * j];
  quats[4 * j + 1] = z[2 * j + 1];
  quats[4 * j + 2] = 0.0f;
  quats[4 * j + 3] = 0.0f;
}

// mu_k = C(n, k), the multiplicity of the multi-index (n - k, k)
__global__ void k_planar_mu(int order_n, float* __restrict__ mu) {
  const int k = threadIdx.x;
  if (k > order_n) return;
  double c = 1.0;
  for (int i = 1; i <= k; ++i) c = c * (order_n - k + i) / i;
  mu[k] = (float)c;
}

// planar components out of the volume components, or the volume components
// (zero except the planar entries) out of the planar ones
__global__ void k_planar_gather(const float* __restrict__ comps3, PlanarIdx idx, int np, long A,
                                float* __restrict__ comps2) {
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (e >= (long)np * A) return;
  const int k = (int)(e / A);
  comps2[e] = comps3[(long)idx.k3[k] * A + e % A];
}

__global__ void k_planar_embed(const float* __restrict__ comps2, PlanarIdx idx, int np, int K3, long A,
                               float* __restrict__ comps3) {
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (e >= (long)K3 * A) return;
  const int c = (int)(e / A);
  float v = 0.0f;
  for (int k = 0; k < np; ++k)
    if (idx.k3[k] == c) v = comps2[(long)k * A + e % A];
  comps3[e] = v;
}

// one list of the stack's candidates: an exclusive scan of the per-plane
// counts (B <= 512) in LDS, then each entry copied with its plane index; one
// block
__global__ void __launch_bounds__(1024) k_planar_compact(int B, int P, const int* __restrict__ counts,
                                                         const int* __restrict__ cand, int* __restrict__ list,
                                                         int* __restrict__ idx, int* __restrict__ total) {
  __shared__ int off[513];
  if (threadIdx.x == 0) {
    int t = 0;
    for (int b = 0; b < B; ++b) {
      off[b] = t;
      t += min(max(counts[2 * b], 0), P);
    }
    off[B] = t;
    total[0] = t;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < B * P; e += blockDim.x) {
    const int b = e / P, p = e % P;
    if (p >= off[b + 1] - off[b]) continue;
    const int o = off[b] + p;
    list[3 * o] = b;
    list[3 * o + 1] = cand[3 * e + 1];
    list[3 * o + 2] = cand[3 * e + 2];
    idx[o] = e;
  }
}

__global__ void k_planar_scatter(int cap, const int* __restrict__ total, const int* __restrict__ idx,
                                 const int* __restrict__ pos3, const float* __restrict__ quat3,
                                 const double* __restrict__ lam3, const float* __restrict__ score3,
                                 const int* __restrict__ flags3, int* __restrict__ pos2, float* __restrict__ z2,
                                 double* __restrict__ lam, float* __restrict__ score, int* __restrict__ flags) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= cap || o >= total[0]) return;
  const int e = idx[o];
  pos2[2 * e] = pos3[3 * o + 1];
  pos2[2 * e + 1] = pos3[3 * o + 2];
  const float a = quat3[4 * o], bb = quat3[4 * o + 1];
  const float r = sqrtf(a * a + bb * bb);
  z2[2 * e] = r > 0.0f ? a / r : 1.0f;
  z2[2 * e + 1] = r > 0.0f ? bb / r : 0.0f;
  lam[e] = lam3[o];
  score[e] = score3[o];
  flags[e] = flags3[o];
}

hipError_t launch_planar_quats(const float* z, int nrot, float* quats, hipStream_t s) {
  hipLaunchKernelGGL(k_planar_quats, dim3((nrot + 255) / 256), dim3(256), 0, s, z, nrot, quats);
  return hipGetLastError();
}

hipError_t launch_planar_mu(int order_n, float* mu, hipStream_t s) {
  hipLaunchKernelGGL(k_planar_mu, dim3(1), dim3(64), 0, s, order_n, mu);
  return hipGetLastError();
}

hipError_t launch_planar_gather(const float* comps3, const PlanarIdx& idx, int np, long A, float* comps2,
                                hipStream_t s) {
  const long n = (long)np * A;
  hipLaunchKernelGGL(k_planar_gather, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, comps3, idx, np, A,
                     comps2);
  return hipGetLastError();
}

hipError_t launch_planar_embed(const float* comps2, const PlanarIdx& idx, int np, int K3, long A, float* comps3,
                               hipStream_t s) {
  const long n = (long)K3 * A;
  hipLaunchKernelGGL(k_planar_embed, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, comps2, idx, np, K3, A,
                     comps3);
  return hipGetLastError();
}

hipError_t launch_planar_compact(int B, int P, const int* counts, const int* cand, int* list, int* idx, int* total,
                                 hipStream_t s) {
  if (B < 1 || B > 512) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_planar_compact, dim3(1), dim3(1024), 0, s, B, P, counts, cand, list, idx, total);
  return hipGetLastError();
}

hipError_t launch_planar_scatter(int cap, const int* total, const int* idx, const int* pos3, const float* quat3,
                                 const double* lam3, const float* score3, const int* flags3, int* pos2, float* z2,
                                 double* lam, float* score, int* flags, hipStream_t s) {
  hipLaunchKernelGGL(k_planar_scatter, dim3((cap + 255) / 256), dim3(256), 0, s, cap, total, idx, pos3, quat3, lam3,
                     score3, flags3, pos2, z2, lam, score, flags);
  return hipGetLastError();
}

}  // namespace ttm
