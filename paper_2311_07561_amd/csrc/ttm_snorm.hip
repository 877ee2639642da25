// S'-consistent normalisation of peak scores (Section 3.4, the discussion of
// false positives; S_2 and S' = S_2 S from the proof of Theorem 1).
//
// The tensor correlation lambda(x) = w(x) <tau_x f, t_Q>_{S'} is normalised
// under S, not S'.  Per candidate window h (and once for the template) this
// computes the squared S'-norm of its S-normalised form,
//
//   D(h) = sum_j omega_j a_j^n <h~, N_m(I_{R_j} h~)>,
//   h~ = (h - <h,m>/m_sum) / ||h - <h,m>/m_sum||_S,
//
// with the tensor template's rotation quadrature (Q_j = (a_j, ...), omega_j),
// I_R the trilinear rotation about the box centre and N_m the masked
// normalisation, and rho' = lambda / sqrt(D(window) D(template)).
//
// Per rotation j the three masked sums of r = I_{R_j} h~ give N_m:
//   <h~, N_m(r)> = (sum m h~ r - mu_r sum m h~) / sqrt(sum m r^2 - mu_r sum m r),
//   mu_r = sum m r / m_sum.
// Kernels:
//   k_snorm_table  the rotation table: R_j (float, 12-float stride) and
//                  kappa_j = omega_j a_j^n (double); entries past n_rot are the
//                  identity with kappa 0
//   k_snorm_prep   one block per window: the two-pass masked mean and
//                  variance, then h~ over the whole box into a contiguous slab
//   k_snorm_rot    one block per (window, chunk of rotations): h~ in LDS, each
//                  wave takes groups of 8 rotations and streams the mask
//                  voxels once per group; the group's rotation matrices are
//                  wave-uniform (scalar registers).  Per-lane float sums, the
//                  wave reduction and everything after it in double.
//   k_snorm_final  per window: the chunk partials summed in a fixed order,
//                  rho' and the flags
#include <algorithm>

#include "ttm_internal.h"
#include "ttm_rotate.h"

namespace ttm {

constexpr int kSnormGroup = 8;      // rotations per wave pass over the mask voxels
constexpr int kSnormRotStride = 12; // floats per rotation-table entry

__global__ void k_snorm_table(const float* __restrict__ quats, const double* __restrict__ weights, int n_rot,
                              int n_pad, int order_n, float* __restrict__ rtab, double* __restrict__ kap) {
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n_pad; j += gridDim.x * blockDim.x) {
    float* r = rtab + (long)j * kSnormRotStride;
    if (j < n_rot) {
      const Rot R = quat_rot(quats + 4 * (long)j);
#pragma unroll
      for (int i = 0; i < 9; ++i) r[i] = R.r[i];
      const double a = quats[4 * j], b = quats[4 * j + 1], c = quats[4 * j + 2], d = quats[4 * j + 3];
      const double an = a / sqrt(a * a + b * b + c * c + d * d);
      double p = 1.0;
      for (int e = 0; e < order_n; ++e) p *= an;
      kap[j] = weights[j] * p;
    } else {
#pragma unroll
      for (int i = 0; i < 9; ++i) r[i] = (i % 4 == 0) ? 1.0f : 0.0f;
      kap[j] = 0.0;
    }
#pragma unroll
    for (int i = 9; i < kSnormRotStride; ++i) r[i] = 0.0f;
  }
}

__device__ __forceinline__ double block_sum_1024(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();                 // red may still be read by a previous call
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double t = 0.0;
  for (int w = 0; w < 16; ++w) t += red[w];
  return t;
}

// window p < max_pos: the image box at pos[p] - c (count from count_dev);
// window max_pos: the template.  stat[p] = {m_sum, sum m h~, flat, outside}.
__global__ void __launch_bounds__(1024) k_snorm_prep(SnormGeo g, const float* __restrict__ image,
                                                     const float* __restrict__ tmpl,
                                                     const unsigned* __restrict__ mlist,
                                                     const float* __restrict__ mval, const int* __restrict__ mcount,
                                                     const int* __restrict__ pos, const int* __restrict__ count_dev,
                                                     float* __restrict__ slabs, double* __restrict__ stat) {
  __shared__ double red[16];
  const int p = blockIdx.x;
  const int count = count_dev ? min(max(count_dev[0], 0), g.max_pos) : g.max_pos;
  if (p < g.max_pos && p >= count) return;
  const int L0 = g.L0, L1 = g.L1, L2 = g.L2;
  const long nL = (long)L0 * L1 * L2;
  const float* __restrict__ src;
  long s0, s1;
  double* st = stat + 4 * (long)p;
  if (p == g.max_pos) {
    src = tmpl;
    s0 = (long)L1 * L2;
    s1 = L2;
  } else {
    const int y0 = pos[3 * p] - L0 / 2, y1 = pos[3 * p + 1] - L1 / 2, y2 = pos[3 * p + 2] - L2 / 2;
    if (y0 < 0 || y1 < 0 || y2 < 0 || y0 + L0 > g.n0 || y1 + L1 > g.n1 || y2 + L2 > g.n2) {
      if (threadIdx.x == 0) {
        st[0] = 0.0; st[1] = 0.0; st[2] = 0.0; st[3] = 1.0;
      }
      return;
    }
    s1 = g.n2;
    s0 = (long)g.n1 * g.n2;
    src = image + y0 * s0 + y1 * s1 + y2;
  }
  const int nm = mcount[0];
  // pass 1: m_sum, sum m h
  float a0 = 0.0f, a1 = 0.0f;
  for (int i = threadIdx.x; i < nm; i += 1024) {
    const unsigned pk = mlist[i];
    const int u0 = (int)(pk & 1023u), u1 = (int)((pk >> 10) & 1023u), u2 = (int)(pk >> 20);
    const float mv = mval[i];
    a0 += mv;
    a1 += mv * src[u0 * s0 + u1 * s1 + u2];
  }
  const double msum = block_sum_1024(a0, red);
  const double mh = block_sum_1024(a1, red);
  const double mu = mh / msum;
  // pass 2: sum m (h - mu)^2 and sum m h^2 (for the flatness test)
  float b0 = 0.0f, b1 = 0.0f;
  const float muf = (float)mu;
  for (int i = threadIdx.x; i < nm; i += 1024) {
    const unsigned pk = mlist[i];
    const int u0 = (int)(pk & 1023u), u1 = (int)((pk >> 10) & 1023u), u2 = (int)(pk >> 20);
    const float mv = mval[i];
    const float h = src[u0 * s0 + u1 * s1 + u2];
    const float d = h - muf;
    b0 += mv * d * d;
    b1 += mv * h * h;
  }
  const double v = block_sum_1024(b0, red);
  const double hh = block_sum_1024(b1, red);
  const bool flat = !(v > kSnormFlatRel * hh);
  const float sc = flat ? 0.0f : (float)(1.0 / sqrt(v));
  float* __restrict__ dst = slabs + (long)p * nL;
  for (long e = threadIdx.x; e < nL; e += 1024) {
    const int u2 = (int)(e % L2);
    const long r = e / L2;
    const int u1 = (int)(r % L1), u0 = (int)(r / L1);
    dst[e] = (src[u0 * s0 + u1 * s1 + u2] - muf) * sc;
  }
  // sum m h~ of the stored values (about 0; kept for the N_m identity)
  float c0 = 0.0f;
  for (int i = threadIdx.x; i < nm; i += 1024) {
    const unsigned pk = mlist[i];
    const int u0 = (int)(pk & 1023u), u1 = (int)((pk >> 10) & 1023u), u2 = (int)(pk >> 20);
    c0 += mval[i] * ((src[u0 * s0 + u1 * s1 + u2] - muf) * sc);
  }
  const double mht = block_sum_1024(c0, red);
  if (threadIdx.x == 0) {
    st[0] = msum; st[1] = mht; st[2] = flat ? 1.0 : 0.0; st[3] = 0.0;
  }
}

template <bool LDS>
__global__ void __launch_bounds__(1024) k_snorm_rot(SnormGeo g, int nchunk, int groups_per_chunk,
                                                    const float* __restrict__ slabs,
                                                    const unsigned* __restrict__ mlist,
                                                    const float* __restrict__ mval, const int* __restrict__ mcount,
                                                    const int* __restrict__ count_dev,
                                                    const float* __restrict__ rtab, const double* __restrict__ kap,
                                                    const double* __restrict__ stat, double* __restrict__ partial) {
  __shared__ float tl[LDS ? kNccLdsCap : 1];
  __shared__ double red[16];
  const int p = blockIdx.x / nchunk, chunk = blockIdx.x % nchunk;
  const int count = count_dev ? min(max(count_dev[0], 0), g.max_pos) : g.max_pos;
  if (p < g.max_pos && p >= count) return;
  const double* st = stat + 4 * (long)p;
  if (st[2] != 0.0 || st[3] != 0.0) {          // flat or outside: block-uniform
    if (threadIdx.x == 0) partial[(long)p * nchunk + chunk] = 0.0;
    return;
  }
  const int L0 = g.L0, L1 = g.L1, L2 = g.L2;
  const int P2 = ncc_lds_p2(L2), P01 = ncc_lds_p01(L1, L2);
  const float* __restrict__ slab = slabs + (long)p * L0 * L1 * L2;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  if (LDS) {
    fill_lds_box(tl, slab, L0, L1, L2, P2, P01, tid, 1024);
    __syncthreads();
  }
  const double msum = st[0], mht = st[1];
  const int nm = mcount[0];
  // mcount[1]: the largest squared distance of a mask voxel from the centre;
  // below the squared inscribed radius every rotated sample point lies in
  // [0, L) on every axis
  const int cmin = min(L0 / 2, min(L1 / 2, L2 / 2));
  const bool inner = mcount[1] < cmin * cmin;
  const int g_lo = chunk * groups_per_chunk;
  const int g_hi = min(g.n_pad / kSnormGroup, g_lo + groups_per_chunk);
  double acc = 0.0;
  for (int grp = g_lo + wave; grp < g_hi; grp += 16) {
    Rot R[kSnormGroup];
    const float* rt = rtab + (long)grp * kSnormGroup * kSnormRotStride;
#pragma unroll
    for (int k = 0; k < kSnormGroup; ++k)
#pragma unroll
      for (int i = 0; i < 9; ++i) R[k].r[i] = rt[k * kSnormRotStride + i];
    float s1[kSnormGroup], s2[kSnormGroup], s3[kSnormGroup];
#pragma unroll
    for (int k = 0; k < kSnormGroup; ++k) s1[k] = s2[k] = s3[k] = 0.0f;
    // INNER: every mask voxel lies in the box's inscribed ball, so every
    // sample takes the LDS sampler's fast path and its test is left out
    auto pass = [&](auto inner_tag) {
      constexpr bool INNER = decltype(inner_tag)::value;
      for (int i = lane; i < nm; i += 64) {
        const unsigned pk = mlist[i];
        const int u0 = (int)(pk & 1023u), u1 = (int)((pk >> 10) & 1023u), u2 = (int)(pk >> 20);
        const float mv = mval[i];
        const float hv = LDS ? tl[u0 * P01 + u1 * P2 + u2] : slab[((long)u0 * L1 + u1) * L2 + u2];
        const float mh = mv * hv;
#pragma unroll
        for (int k = 0; k < kSnormGroup; ++k) {
          const float r = !LDS ? sample_rotated(slab, L0, L1, L2, R[k], u0, u1, u2)
                               : INNER ? sample_rotated_lds_inner(tl, L0, L1, L2, P2, P01, R[k], u0, u1, u2)
                                       : sample_rotated_lds(tl, L0, L1, L2, P2, P01, R[k], u0, u1, u2);
          const float mr = mv * r;
          s1[k] += mr;
          s2[k] += mr * r;
          s3[k] += mh * r;
        }
      }
    };
    if (LDS && inner)
      pass(std::true_type{});
    else
      pass(std::false_type{});
#pragma unroll
    for (int k = 0; k < kSnormGroup; ++k) {
      double t1 = s1[k], t2 = s2[k], t3 = s3[k];
      for (int off = 32; off > 0; off >>= 1) {
        t1 += __shfl_xor(t1, off);
        t2 += __shfl_xor(t2, off);
        t3 += __shfl_xor(t3, off);
      }
      const double mu = t1 / msum;
      const double var = t2 - mu * t1;
      if (var > kSnormFlatRel * t2) acc += kap[grp * kSnormGroup + k] * (t3 - mu * mht) / sqrt(var);
    }
  }
  // waves without a group hold acc = 0
  if (lane == 0) red[wave] = acc;
  __syncthreads();
  if (tid == 0) {
    double t = 0.0;
    for (int w = 0; w < 16; ++w) t += red[w];
    partial[(long)p * nchunk + chunk] = t;
  }
}

__global__ void k_snorm_final(SnormGeo g, int nchunk, const int* __restrict__ count_dev,
                              const double* __restrict__ stat, const double* __restrict__ partial,
                              const double* __restrict__ lambda, float* __restrict__ out_rho,
                              double* __restrict__ out_D, int* __restrict__ out_flags) {
  const int count = count_dev ? min(max(count_dev[0], 0), g.max_pos) : g.max_pos;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  auto window_D = [&](int q, int& fl) {
    const double* st = stat + 4 * (long)q;
    fl = 0;
    if (st[3] != 0.0) fl |= TTM_SNORM_OUTSIDE;
    if (st[2] != 0.0) fl |= TTM_SNORM_FLAT;
    if (fl) return (double)NAN;
    double D = 0.0;
    for (int c = 0; c < nchunk; ++c) D += partial[(long)q * nchunk + c];
    return D;
  };
  if (p == g.max_pos) {
    int fl;
    out_D[p] = window_D(p, fl);
    return;
  }
  if (p >= count) return;
  int ft, fl;
  const double Dt = window_D(g.max_pos, ft);
  const double D = window_D(p, fl);
  out_D[p] = D;
  if (!fl && !(D > 0.0)) fl |= TTM_SNORM_NONPOS;
  if (!(Dt > 0.0)) fl |= TTM_SNORM_TEMPLATE;
  out_rho[p] = fl ? 0.0f : (float)(lambda[p] / sqrt(D * Dt));
  out_flags[p] = fl;
}

int snorm_chunks(int n_win, int n_pad) {
  const int groups = n_pad / kSnormGroup;
  int nchunk = (512 + n_win - 1) / n_win;               // about two blocks per CU in all
  nchunk = std::min(nchunk, std::max(1, (groups + 15) / 16));   // at least one group per wave
  return std::max(1, nchunk);
}

int snorm_pad(int n_rot) { return (n_rot + kSnormGroup - 1) / kSnormGroup * kSnormGroup; }

hipError_t launch_snorm(const SnormGeo& g, const float* image, const float* tmpl, const float* mask,
                        const float* quats, const double* weights, int n_rot, int order_n, const int* pos,
                        const int* count_dev, const double* lambda, const SnormWs& w, float* out_rho, double* out_D,
                        int* out_flags, hipStream_t s) {
  const int n_win = g.max_pos + 1;
  const int nchunk = snorm_chunks(n_win, g.n_pad);
  const int groups = g.n_pad / kSnormGroup;
  const int gpc = (groups + nchunk - 1) / nchunk;
  hipLaunchKernelGGL(k_snorm_table, dim3((g.n_pad + 255) / 256), dim3(256), 0, s, quats, weights, n_rot, g.n_pad,
                     order_n, w.rtab, w.kap);
  hipError_t e = launch_mask_list(mask, g.L0, g.L1, g.L2, w.mlist, w.mval, w.mcount, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_snorm_prep, dim3(n_win), dim3(1024), 0, s, g, image, tmpl, w.mlist, w.mval, w.mcount, pos,
                     count_dev, w.slabs, w.stat);
  if (ncc_lds_floats(g.L0, g.L1, g.L2) <= kNccLdsCap)
    hipLaunchKernelGGL(k_snorm_rot<true>, dim3((unsigned)(n_win * nchunk)), dim3(1024), 0, s, g, nchunk, gpc,
                       w.slabs, w.mlist, w.mval, w.mcount, count_dev, w.rtab, w.kap, w.stat, w.partial);
  else
    hipLaunchKernelGGL(k_snorm_rot<false>, dim3((unsigned)(n_win * nchunk)), dim3(1024), 0, s, g, nchunk, gpc,
                       w.slabs, w.mlist, w.mval, w.mcount, count_dev, w.rtab, w.kap, w.stat, w.partial);
  hipLaunchKernelGGL(k_snorm_final, dim3((n_win + 255) / 256), dim3(256), 0, s, g, nchunk, count_dev, w.stat,
                     w.partial, lambda, out_rho, out_D, out_flags);
  return hipGetLastError();
}

}  // namespace ttm
