// All-voxel rotation map (Section 3.4 with Theorem "main"): at every voxel x
// of the valid region, the dominant Z-eigenpair of the correlated tensor
// C_n(x), i.e. the maximiser over S^3 of phi(x, Q) = C_n(x) Q^n.
//
// 1. Seed scan, a dense contraction on the matrix cores: for J seed points
//    Q_j, phi(x, Q_j) = sum_alpha [mu_alpha Q_j^alpha] C_alpha(x) is the
//    product of the seed table A[J][K] with the field B[K][V].  It runs as
//    32 x 32 x 16 fp16 MFMA tiles with float32 accumulation: seeds are the
//    rows (A operand), voxels the columns (B operand).  Each lane holds 16
//    seeds of one voxel in its accumulators, so the running maximum over
//    the seeds is a per-lane reduction; only the winning group of 16 seeds
//    (tile, lane half) is kept per voxel.  Each voxel's column is scaled by
//    1 / max_alpha |C_alpha(x)| before rounding to fp16 (the argmax is
//    invariant to a positive scale).
// 2. Polish in float64, one lane per voxel: lambda at the 16 seeds of the
//    winning group, then the safeguarded Newton / shifted power iteration
//    from the best of them.
#include <cfloat>

#include "ttm_device.h"
#include "ttm_eig.h"
#include "ttm_internal.h"

namespace ttm {

typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// table entry (tile t, group g, row r) = 8 halves mu_alpha Q^alpha for
// alpha = 8 g .. 8 g + 7 (zero beyond K) of seed 32 t + r; one uint4 each,
// at ((t * KG + g) * 32 + r)
template <int N>
__global__ void __launch_bounds__(256) k_rmap_table(const float* __restrict__ seeds, int n_seeds,
                                                    uint4* __restrict__ table) {
  constexpr int K = (N + 1) * (N + 2) * (N + 3) / 6;
  constexpr int KG = 2 * ((K + 15) / 16);
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n_seeds) return;
  double q[4] = {seeds[4 * j], seeds[4 * j + 1], seeds[4 * j + 2], seeds[4 * j + 3]};
  const double nq = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
#pragma unroll
  for (int d = 0; d < 4; ++d) q[d] = nq > 0.0 ? q[d] / nq : (d == 0 ? 1.0 : 0.0);
  double pw[4][N + 1];
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    pw[d][0] = 1.0;
#pragma unroll
    for (int e = 1; e <= N; ++e) pw[d][e] = pw[d][e - 1] * q[d];
  }
  _Float16 v[KG * 8];
#pragma unroll
  for (int k = 0; k < KG * 8; ++k) v[k] = (_Float16)0.0f;
  static_for<0, K>([&](auto kk) {
    constexpr Alpha A = alpha_c(N, decltype(kk)::value);
    constexpr double mu = mult_c(N, A);
    v[decltype(kk)::value] =
        (_Float16)(mu * ((pw[0][A.a[0]] * pw[1][A.a[1]]) * (pw[2][A.a[2]] * pw[3][A.a[3]])));
  });
  const int t = j >> 5, r = j & 31;
#pragma unroll
  for (int g = 0; g < KG; ++g) {
    f16x8 e;
#pragma unroll
    for (int i = 0; i < 8; ++i) e[i] = v[8 * g + i];
    table[((long)t * KG + g) * 32 + r] = *reinterpret_cast<const uint4*>(&e);
  }
}

// Seed scan.  A block of 4 waves; wave w holds VT tiles of 32 voxels as B
// operands in registers for the whole scan.  The seed table streams through
// two LDS chunks of CT tiles (global loads of the next chunk are in flight
// while the current one is multiplied).  Output per voxel: the winning group
// 2 t + h (tile t, lane half h).
template <int KS>
struct ScanCfg {
  static constexpr int KG = 2 * KS;                 // 8-element groups per seed row
  static constexpr int TILE16 = KG * 32;            // uint4 entries per seed tile
  static constexpr int CT = 768 / TILE16 > 0 ? 768 / TILE16 : 1;   // tiles per chunk (<= 12 KiB)
  static constexpr int CH16 = CT * TILE16;          // uint4 entries per chunk
  static constexpr int PFN = (CH16 + 255) / 256;    // uint4 per thread per chunk
  static constexpr int VT = KS <= 3 ? 4 : (KS <= 6 ? 2 : 1);
  static constexpr int VOX = 4 * VT * 32;           // voxels per block
};

template <int KS>
__global__ void __launch_bounds__(256) k_rmap_scan(const float* __restrict__ planes, long Vv, int K,
                                                   const uint4* __restrict__ table, int ntiles, int tbits,
                                                   int* __restrict__ group_out) {
  using S = ScanCfg<KS>;
  constexpr int VT = S::VT, TILE16 = S::TILE16, CT = S::CT, CH16 = S::CH16, PFN = S::PFN;
  __shared__ uint4 buf[2][CH16];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int j = lane & 31, h = lane >> 5;
  const long vbase = ((long)blockIdx.x * 4 + wave) * (VT * 32);

  // B operands: lane (j, h) holds C[16 s + 8 h + e][voxel j], e = 0..7
  // (the loads use clamped, always valid indices and are masked afterwards,
  // so that all of them are in flight at once)
  f16x8 b[VT][KS];
#pragma unroll
  for (int v = 0; v < VT; ++v) {
    const long vox = vbase + v * 32 + j;
    const long vc = vox < Vv ? vox : Vv - 1;
    float cv[KS][8];
#pragma unroll
    for (int s = 0; s < KS; ++s)
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int k = 16 * s + 8 * h + e;
        cv[s][e] = planes[(long)(k < K ? k : K - 1) * Vv + vc];
      }
    float mx = 0.0f;
#pragma unroll
    for (int s = 0; s < KS; ++s)
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int k = 16 * s + 8 * h + e;
        if (!(k < K && vox < Vv)) cv[s][e] = 0.0f;
        mx = fmaxf(mx, fabsf(cv[s][e]));
      }
    mx = fmaxf(mx, __shfl_xor(mx, 32));
    const float sc = mx > 0.0f ? 1.0f / mx : 0.0f;
#pragma unroll
    for (int s = 0; s < KS; ++s)
#pragma unroll
      for (int e = 0; e < 8; ++e) b[v][s][e] = (_Float16)(cv[s][e] * sc);
  }

  // running best per voxel tile as a key: the tile's maximum with its low
  // tbits mantissa bits replaced by the tile index, so that one maximum keeps
  // both (the keys order as the maxima do up to 2^(tbits - 24) relative, far
  // below the fp16 rounding of the products)
  const unsigned tmask = (1u << tbits) - 1u;
  float best[VT];
#pragma unroll
  for (int v = 0; v < VT; ++v) best[v] = -FLT_MAX;
  const int nch = (ntiles + CT - 1) / CT;
  const long tab16 = (long)ntiles * TILE16;
  uint4 pf[PFN];
#pragma unroll
  for (int i = 0; i < PFN; ++i) {
    const int e = tid + 256 * i;
    pf[i] = (e < CH16 && e < tab16) ? table[e] : make_uint4(0u, 0u, 0u, 0u);
  }
#pragma unroll 1
  for (int c = 0; c < nch; ++c) {
    uint4* __restrict__ cur = buf[c & 1];
#pragma unroll
    for (int i = 0; i < PFN; ++i) {
      const int e = tid + 256 * i;
      if (e < CH16) cur[e] = pf[i];
    }
    __syncthreads();
    if (c + 1 < nch) {
      const long base = (long)(c + 1) * CH16;
#pragma unroll
      for (int i = 0; i < PFN; ++i) {
        const int e = tid + 256 * i;
        pf[i] = (e < CH16 && base + e < tab16) ? table[base + e] : make_uint4(0u, 0u, 0u, 0u);
      }
    }
    const int tc = min(CT, ntiles - c * CT);
#pragma unroll 1
    for (int t = 0; t < tc; ++t) {
      f16x8 a[KS];
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        const uint4 u = cur[t * TILE16 + (2 * s + h) * 32 + j];
        a[s] = *reinterpret_cast<const f16x8*>(&u);
      }
      const int tile = c * CT + t;
#pragma unroll
      for (int v = 0; v < VT; ++v) {
        f32x16 acc = {};
#pragma unroll
        for (int s = 0; s < KS; ++s) acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(a[s], b[v][s], acc, 0, 0, 0);
        float m = __builtin_elementwise_maximum(__builtin_elementwise_maximum(acc[0], acc[1]), acc[2]);
#pragma unroll
        for (int r = 3; r < 15; r += 2)
          m = __builtin_elementwise_maximum(__builtin_elementwise_maximum(m, acc[r]), acc[r + 1]);
        m = __builtin_elementwise_maximum(m, acc[15]);
        const float key = __uint_as_float((__float_as_uint(m) & ~tmask) | (unsigned)tile);
        best[v] = __builtin_elementwise_maximum(best[v], key);
      }
    }
  }
  // merge the two lane halves of each voxel: the larger key, half 0 on equal
  // keys (the tile index is clamped in case a non-finite input made the key
  // NaN)
#pragma unroll
  for (int v = 0; v < VT; ++v) {
    const float ob = __shfl_xor(best[v], 32);
    const long vox = vbase + v * 32 + j;
    if (h == 0 && vox < Vv) {
      const bool mine = !(ob > best[v]);
      const int t = (int)(__float_as_uint(mine ? best[v] : ob) & tmask);
      group_out[vox] = 2 * (t < ntiles ? t : ntiles - 1) + (mine ? 0 : 1);
    }
  }
}

struct RmapGeo {
  int n1, n2;
  int lo0, lo1, lo2;
  int W1, W2;
};

// column of one lane's tensor in the LDS table [K][64]
struct ColAcc {
  const float* p;
  __device__ double operator[](int k) const { return (double)p[k * 64]; }
};

// Polish: one lane per voxel.  The score F(x) = |C_n(x)|_F = (sum_alpha
// mu_alpha C_alpha^2)^(1/2) in float64 (Section 3.4); lambda at the 16 seeds
// of the voxel's winning group in float64 (the lowest seed on ties), then
// eig_polish from the best.  Where C_n(x) = 0 (w(x) = 0) the map holds
// lambda = 0 and the identity.
template <int N>
__global__ void __launch_bounds__(64) k_rmap_polish(RmapGeo g, const float* __restrict__ planes, long Vv,
                                                    const float* __restrict__ seeds, const int* __restrict__ group,
                                                    int max_iter, double tol, float* __restrict__ out_score,
                                                    float* __restrict__ out_quat, float* __restrict__ out_lambda,
                                                    int* __restrict__ unconv) {
  constexpr int K = (N + 1) * (N + 2) * (N + 3) / 6;
  __shared__ float cs[K * 64];
  __shared__ double mu[K];
  const int lane = threadIdx.x;
  for (int k = lane; k < K; k += 64) {
    int al[4];
    alpha_of_dev(N, k, al);
    mu[k] = fact_d(N) / (fact_d(al[0]) * fact_d(al[1]) * fact_d(al[2]) * fact_d(al[3]));
  }
  __syncthreads();
  const long vox = (long)blockIdx.x * 64 + lane;
  const bool live = vox < Vv;
  bool zero = true;
  double f2 = 0.0;
#pragma unroll 4
  for (int k = 0; k < K; ++k) {
    const float c = live ? planes[(long)k * Vv + vox] : 0.0f;
    cs[k * 64 + lane] = c;
    zero = zero && c == 0.0f;
    f2 += mu[k] * ((double)c * (double)c);
  }
  // each lane reads only its own column of cs: no barrier needed
  if (!live) return;
  const long yz = (long)g.W1 * g.W2;
  const int x0 = g.lo0 + (int)(vox / yz);
  const int x1 = g.lo1 + (int)((vox / g.W2) % g.W1);
  const int x2 = g.lo2 + (int)(vox % g.W2);
  const long o = ((long)x0 * g.n1 + x1) * g.n2 + x2;
  out_score[o] = (float)sqrt(f2);
  if (zero) {
    out_quat[4 * o] = 1.0f;
    out_quat[4 * o + 1] = 0.0f;
    out_quat[4 * o + 2] = 0.0f;
    out_quat[4 * o + 3] = 0.0f;
    out_lambda[o] = 0.0f;
    return;
  }
  const ColAcc C{cs + lane};
  const int gr = group[vox];
  const int t = gr >> 1, hh = gr & 1;
  double x[4] = {1.0, 0.0, 0.0, 0.0};
  double lam = -INFINITY;
  for (int r = 0; r < 16; ++r) {
    const int sd = 32 * t + 8 * (r >> 2) + 4 * hh + (r & 3);
    double q[4] = {seeds[4 * sd], seeds[4 * sd + 1], seeds[4 * sd + 2], seeds[4 * sd + 3]};
    const double nq = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    if (!(nq > 0.0)) continue;
#pragma unroll
    for (int d = 0; d < 4; ++d) q[d] /= nq;
    const double l = lambda_at<N>(C, q);
    if (l > lam) {
      lam = l;
#pragma unroll
      for (int d = 0; d < 4; ++d) x[d] = q[d];
    }
  }
  const bool conv = eig_polish<N>(C, x, lam, max_iter, tol);
  const double nx = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2] + x[3] * x[3]);
  double sgn = 1.0;
  for (int d = 0; d < 4; ++d)
    if (x[d] != 0.0) {
      sgn = x[d] > 0.0 ? 1.0 : -1.0;
      break;
    }
#pragma unroll
  for (int d = 0; d < 4; ++d) out_quat[4 * o + d] = (float)(sgn * x[d] / nx);
  out_lambda[o] = (float)lam;
  if (!conv && unconv) atomicAdd(unconv, 1);
}

long rmap_table_uint4(int order_n, int n_seeds) {
  const int K = num_components(order_n);
  return (long)(n_seeds / 32) * 2 * ((K + 15) / 16) * 32;
}

static RmapGeo make_rmapgeo(const Geo& gg, long& Vv) {
  RmapGeo g;
  g.n1 = gg.n1; g.n2 = gg.n2;
  g.lo0 = gg.lo0(); g.lo1 = gg.lo1(); g.lo2 = gg.c2;
  g.W1 = gg.hi1() - gg.lo1() + 1;
  g.W2 = gg.n2 - gg.L2 + 1;
  Vv = (long)(gg.hi0() - gg.lo0() + 1) * g.W1 * g.W2;
  return g;
}

hipError_t launch_rmap_table(int order_n, const float* seeds, int n_seeds, uint4* table, hipStream_t s) {
  const dim3 tg((unsigned)((n_seeds + 255) / 256));
  switch (order_n) {
    case 2: hipLaunchKernelGGL(k_rmap_table<2>, tg, dim3(256), 0, s, seeds, n_seeds, table); break;
    case 4: hipLaunchKernelGGL(k_rmap_table<4>, tg, dim3(256), 0, s, seeds, n_seeds, table); break;
    case 6: hipLaunchKernelGGL(k_rmap_table<6>, tg, dim3(256), 0, s, seeds, n_seeds, table); break;
    case 8: hipLaunchKernelGGL(k_rmap_table<8>, tg, dim3(256), 0, s, seeds, n_seeds, table); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int KS>
static void scan_ks(long Vv, int K, const float* planes, const uint4* table, int ntiles, int* group,
                    hipStream_t s) {
  const dim3 sg((unsigned)((Vv + ScanCfg<KS>::VOX - 1) / ScanCfg<KS>::VOX));
  int tbits = 1;
  while ((1 << tbits) < ntiles) ++tbits;
  hipLaunchKernelGGL(k_rmap_scan<KS>, sg, dim3(256), 0, s, planes, Vv, K, table, ntiles, tbits, group);
}

hipError_t launch_rmap_scan(const Geo& gg, int order_n, const float* planes, const uint4* table, int n_seeds,
                            int* group, hipStream_t s) {
  long Vv;
  make_rmapgeo(gg, Vv);
  const int K = num_components(order_n);
  const int ntiles = n_seeds / 32;
  switch (order_n) {
    case 2: scan_ks<1>(Vv, K, planes, table, ntiles, group, s); break;
    case 4: scan_ks<3>(Vv, K, planes, table, ntiles, group, s); break;
    case 6: scan_ks<6>(Vv, K, planes, table, ntiles, group, s); break;
    case 8: scan_ks<11>(Vv, K, planes, table, ntiles, group, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_rmap_polish(const Geo& gg, int order_n, const float* planes, const float* seeds,
                              const int* group, int max_iter, double tol, float* out_score, float* out_quat,
                              float* out_lambda, int* unconv, hipStream_t s) {
  long Vv;
  const RmapGeo g = make_rmapgeo(gg, Vv);
  const dim3 pg((unsigned)((Vv + 63) / 64));
  switch (order_n) {
    case 2:
      hipLaunchKernelGGL(k_rmap_polish<2>, pg, dim3(64), 0, s, g, planes, Vv, seeds, group, max_iter, tol,
                         out_score, out_quat, out_lambda, unconv);
      break;
    case 4:
      hipLaunchKernelGGL(k_rmap_polish<4>, pg, dim3(64), 0, s, g, planes, Vv, seeds, group, max_iter, tol,
                         out_score, out_quat, out_lambda, unconv);
      break;
    case 6:
      hipLaunchKernelGGL(k_rmap_polish<6>, pg, dim3(64), 0, s, g, planes, Vv, seeds, group, max_iter, tol,
                         out_score, out_quat, out_lambda, unconv);
      break;
    case 8:
      hipLaunchKernelGGL(k_rmap_polish<8>, pg, dim3(64), 0, s, g, planes, Vv, seeds, group, max_iter, tol,
                         out_score, out_quat, out_lambda, unconv);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace ttm
