// FFT passes of the correlation path (Section 2, FFT inner products; Algorithm
// 1; Section 3.2).  Transforms are unnormalised; the 1/(n0 n1 n2) factor is
// applied once, in the last inverse pass.
//
// Layout of a half spectrum: [n0][n1][h2] complex float, h2 = n2/2 + 1.
// Forward path of the image: axis-2 R2C (rows), then axis 1 (pencils, in
// place); the axis-0 forward transform is done on the fly inside pass 1.
// Inverse path per (image spectrum, template entry) pair: pass 1 = axis 0
// (fused with the forward axis-0 transform of the pruned template block and
// the conjugate product), pass 2 = axis 1 (pencils, in place), pass 3 =
// axis-2 C2R fused with the per-voxel reduction.
#include "ttm_device.h"
#include "ttm_internal.h"

namespace ttm {

// ----------------------------------------------------------------------------
// image and mask moments (float64, deterministic two-level reduction)
// ----------------------------------------------------------------------------
constexpr int kStatBlocks = kStatPartials;

__device__ __forceinline__ void block_sum3(double& a, double& b, double& c, double* sh /* 768 */) {
  const int tid = threadIdx.x;
  sh[tid] = a;
  sh[tid + 256] = b;
  sh[tid + 512] = c;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) {
      sh[tid] += sh[tid + s];
      sh[tid + 256] += sh[tid + 256 + s];
      sh[tid + 512] += sh[tid + 512 + s];
    }
    __syncthreads();
  }
  a = sh[0];
  b = sh[256];
  c = sh[512];
}

// per block: sum f, sum f^2 over a grid-stride share of the image and, if
// mask is given, sum m over a share of the mask
__global__ void __launch_bounds__(256) k_stats_partial(const float* __restrict__ x, long n,
                                                       const float* __restrict__ mask, long nm,
                                                       double* __restrict__ partials) {
  __shared__ double sh[768];
  double s1 = 0.0, s2 = 0.0, s3 = 0.0;
  const long n4 = n / 4;
  const long gs = (long)gridDim.x * blockDim.x, t0 = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const float4* x4 = reinterpret_cast<const float4*>(x);
  for (long i = t0; i < n4; i += gs) {
    const float4 v = x4[i];
    s1 += (double)v.x + (double)v.y + (double)v.z + (double)v.w;
    s2 += (double)v.x * v.x + (double)v.y * v.y + (double)v.z * v.z + (double)v.w * v.w;
  }
  for (long i = n4 * 4 + t0; i < n; i += gs) {
    const double v = x[i];
    s1 += v;
    s2 += v * v;
  }
  if (mask)
    for (long i = t0; i < nm; i += gs) s3 += (double)mask[i];
  block_sum3(s1, s2, s3, sh);
  if (threadIdx.x == 0) {
    partials[3 * blockIdx.x] = s1;
    partials[3 * blockIdx.x + 1] = s2;
    partials[3 * blockIdx.x + 2] = s3;
  }
}

__global__ void __launch_bounds__(256) k_stats_final(const double* __restrict__ partials, int nb, long n,
                                                     int with_mask, double* __restrict__ stats, int mu_order,
                                                     float* __restrict__ mu) {
  __shared__ double sh[768];
  // the multiplicities n! / (a1! a2! a3! a4!) of the packed multi-indices
  if (mu) {
    const int K = (mu_order + 1) * (mu_order + 2) * (mu_order + 3) / 6;
    for (int k = threadIdx.x; k < K; k += blockDim.x) {
      int al[4];
      alpha_of_dev(mu_order, k, al);
      double f = 1.0;
      for (int i = 2; i <= mu_order; ++i) f *= i;
      for (int d = 0; d < 4; ++d)
        for (int i = 2; i <= al[d]; ++i) f /= i;
      mu[k] = (float)f;
    }
  }
  double s1 = 0.0, s2 = 0.0, s3 = 0.0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) {
    s1 += partials[3 * i];
    s2 += partials[3 * i + 1];
    s3 += partials[3 * i + 2];
  }
  block_sum3(s1, s2, s3, sh);
  if (threadIdx.x == 0) {
    const double mean = s1 / (double)n;
    double var = s2 / (double)n - mean * mean;
    stats[0] = mean;
    stats[1] = var > 0.0 ? var : 0.0;
    if (with_mask) stats[2] = s3;
  }
}

hipError_t launch_image_stats(const float* img, long n, const float* mask, long nm, double* partials,
                              double* stats, hipStream_t s, int mu_order, float* mu) {
  hipLaunchKernelGGL(k_stats_partial, dim3(kStatBlocks), dim3(256), 0, s, img, n, mask, nm, partials);
  hipLaunchKernelGGL(k_stats_final, dim3(1), dim3(256), 0, s, partials, kStatBlocks, n, mask ? 1 : 0, stats,
                     mu_order, mu);
  return hipGetLastError();
}

// ----------------------------------------------------------------------------
// axis-2 R2C of real rows through a half-length complex FFT:
// z(m) = x(2m) + i x(2m+1), Z = FFT_M(z),
// X(k) = (Z(k) + conj Z(M-k))/2 - (i/2) W_N^k (Z(k) - conj Z(M-k)), k = 0..M
// ----------------------------------------------------------------------------
template <int M>
struct RowCfg {
  static constexpr int R1 = Plan<M>::R1, R2 = Plan<M>::R2;
  static constexpr int RW = 256 / R1;          // rows per block
  static constexpr int SP = M + 1;             // stage pitch (complex)
};

template <int M, int MODE>
__global__ void __launch_bounds__(256) k_r2c_rows(const float* __restrict__ src, long src_stride,
                                                  int len_valid, long nrows, float2* __restrict__ dst0,
                                                  float2* __restrict__ dst1, long grp, long grp_stride,
                                                  const double* __restrict__ stats) {
  using C = RowCfg<M>;
  constexpr int R1 = C::R1, R2 = C::R2, RW = C::RW, SP = C::SP;
  constexpr int N2 = 2 * M, H2 = M + 1, P2 = row_pitch(N2);
  __shared__ float2 stage[RW * SP];
  __shared__ float2 twM[M];
  __shared__ float2 tw2[N2];
  const int tid = threadIdx.x;
  fill_twiddles(twM, M, tid, 256);
  fill_twiddles(tw2, N2, tid, 256);
  const long r0 = (long)blockIdx.x * RW;
  const int p = tid % RW, a = tid / RW;
  const float mean = MODE == 1 ? (float)stats[0] : 0.0f;

#pragma unroll 1
  for (int sq = 0; sq < (MODE == 1 ? 2 : 1); ++sq) {
    float2* dst = sq ? dst1 : dst0;
    __syncthreads();
    for (int e = tid; e < RW * M; e += 256) {
      const int rr = e / M, m = e % M;
      const long r = r0 + rr;
      float v0 = 0.0f, v1 = 0.0f;
      if (r < nrows) {
        const float* row = src + r * src_stride;
        if (2 * m < len_valid) v0 = row[2 * m];
        if (2 * m + 1 < len_valid) v1 = row[2 * m + 1];
        if (MODE == 1) {
          v0 -= mean;
          v1 -= mean;
          if (sq) {
            v0 *= v0;
            v1 *= v1;
          }
        }
      }
      stage[rr * SP + m] = make_float2(v0, v1);
    }
    __syncthreads();
    float2 x[R2], o[R2];
#pragma unroll
    for (int b = 0; b < R2; ++b) x[b] = stage[p * SP + a + R1 * b];
    // the engine's exchange buffer aliases the stage: all stage reads above
    // complete before the engine's first barrier
    engineA<M, RW, false>(x, o, stage, twM, p, a);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < R2 / R1; ++k)
#pragma unroll
      for (int d = 0; d < R1; ++d) stage[p * SP + (a + R1 * k) + R2 * d] = o[k * R1 + d];
    __syncthreads();
    for (int e = tid; e < RW * H2; e += 256) {
      const int rr = e / H2, k = e % H2;
      const long r = r0 + rr;
      if (r >= nrows) continue;
      const float2 zk = stage[rr * SP + (k % M)];
      const float2 zm = cconj(stage[rr * SP + ((M - k) % M)]);
      const float2 ev = cscale(cadd(zk, zm), 0.5f);
      const float2 pw = cmul(tw2[k], csub(zk, zm));
      const float2 X = make_float2(ev.x + 0.5f * pw.y, ev.y - 0.5f * pw.x);
      const long drow = (r / grp) * grp_stride + (r % grp);
      dst[drow * P2 + k] = X;
    }
  }
}

template <int M>
static hipError_t r2c_rows_m(const float* src, long src_stride, int len_valid, long nrows,
                             float2* dst0, float2* dst1, long grp, long grp_stride, int mode,
                             const double* stats, hipStream_t s) {
  constexpr int RW = RowCfg<M>::RW;
  dim3 grid((unsigned)((nrows + RW - 1) / RW));
  if (mode == 1)
    hipLaunchKernelGGL((k_r2c_rows<M, 1>), grid, dim3(256), 0, s, src, src_stride, len_valid, nrows,
                       dst0, dst1, grp, grp_stride, stats);
  else
    hipLaunchKernelGGL((k_r2c_rows<M, 0>), grid, dim3(256), 0, s, src, src_stride, len_valid, nrows,
                       dst0, dst1, grp, grp_stride, stats);
  return hipGetLastError();
}

hipError_t launch_r2c_rows(int n2, const float* src, long src_stride, int len_valid, long nrows,
                           float2* dst0, float2* dst1, long grp, long grp_stride, int mode,
                           const double* stats, hipStream_t s) {
  switch (n2) {
    case 16: return r2c_rows_m<8>(src, src_stride, len_valid, nrows, dst0, dst1, grp, grp_stride, mode, stats, s);
    case 32: return r2c_rows_m<16>(src, src_stride, len_valid, nrows, dst0, dst1, grp, grp_stride, mode, stats, s);
    case 64: return r2c_rows_m<32>(src, src_stride, len_valid, nrows, dst0, dst1, grp, grp_stride, mode, stats, s);
    case 128: return r2c_rows_m<64>(src, src_stride, len_valid, nrows, dst0, dst1, grp, grp_stride, mode, stats, s);
    case 256: return r2c_rows_m<128>(src, src_stride, len_valid, nrows, dst0, dst1, grp, grp_stride, mode, stats, s);
    case 512: return r2c_rows_m<256>(src, src_stride, len_valid, nrows, dst0, dst1, grp, grp_stride, mode, stats, s);
    default: return hipErrorInvalidValue;
  }
}

// ----------------------------------------------------------------------------
// strided pencils along one axis (in place)
// ----------------------------------------------------------------------------
template <int N>
struct PenCfg {
  static constexpr int R1 = Plan<N>::R1, R2 = Plan<N>::R2;
  static constexpr int PW = 256 / R1;    // pencils per block
};

// One block transforms PW pencils.  Element offsets are 32-bit from the
// block's array base (one array holds < 2^31 elements).
template <int N, bool INV, bool PRUNED>
__global__ void __launch_bounds__(256) k_pencils(float2* __restrict__ data, int npencils, int Q, long S_outer,
                                                 int S_axis, int nin, int shift, int slo, int shi,
                                                 long batch_stride) {
  using C = PenCfg<N>;
  constexpr int R1 = C::R1, R2 = C::R2, PW = C::PW;
  __shared__ float2 lds[PW * N];
  __shared__ float2 tw[N];
  const int tid = threadIdx.x;
  fill_twiddles(tw, N, tid, 256);
  // the table is written by several waves and read (by the engine's first
  // twiddle step) before any other barrier
  __syncthreads();
  const int pl = tid % PW, a = tid / PW;
  const int p = xcd_tile(blockIdx.x, gridDim.x) * PW + pl;
  const bool valid = p < npencils;
  float2* __restrict__ arr = data + (long)blockIdx.y * batch_stride;
  const unsigned toff = valid ? (unsigned)((long)(p / Q) * S_outer + (p % Q)) + (unsigned)(a * S_axis) : 0u;
  const unsigned step = (unsigned)(R1 * S_axis);
  float2 x[R2], o[R2];
#pragma unroll
  for (int b = 0; b < R2; ++b) {
    if (PRUNED)
      x[b] = (valid && a + R1 * b < nin) ? arr[toff + b * step] : make_float2(0.0f, 0.0f);
    else
      x[b] = arr[toff + b * step];
  }
  engineA<N, PW, INV>(x, o, lds, tw, pl, a);
  if (!valid) return;
  const unsigned base = toff - (unsigned)(a * S_axis);
#pragma unroll
  for (int k = 0; k < R2 / R1; ++k)
#pragma unroll
    for (int d = 0; d < R1; ++d) {
      const int j = (a + R1 * k) + R2 * d;
      const int x = (j + shift) & (N - 1);
      if ((unsigned)(x - slo) <= (unsigned)(shi - slo)) arr[base + (unsigned)(x * S_axis)] = o[k * R1 + d];
    }
}

template <int N>
static hipError_t pencils_n(bool inverse, float2* data, long npencils, long Q, long S_outer, long S_axis, int nin,
                            int shift, int slo, int shi, int nbatch, long batch_stride, hipStream_t s) {
  constexpr int PW = PenCfg<N>::PW;
  if (npencils <= 0 || nbatch <= 0) return hipSuccess;
  dim3 grid((unsigned)((npencils + PW - 1) / PW), (unsigned)nbatch);
  const bool pruned = nin < N;
#define TTM_PENCILS(I, PR)                                                                                  \
  hipLaunchKernelGGL((k_pencils<N, I, PR>), grid, dim3(256), 0, s, data, (int)npencils, (int)Q, S_outer, \
                     (int)S_axis, nin, shift, slo, shi, batch_stride)
  if (inverse) {
    if (pruned) TTM_PENCILS(true, true);
    else TTM_PENCILS(true, false);
  } else {
    if (pruned) TTM_PENCILS(false, true);
    else TTM_PENCILS(false, false);
  }
#undef TTM_PENCILS
  return hipGetLastError();
}

hipError_t launch_pencils(int N, bool inverse, float2* data, long npencils, long Q, long S_outer, long S_axis,
                          int nin, int shift, int slo, int shi, int nbatch, long batch_stride, hipStream_t s) {
  switch (N) {
#define TTM_CASE(n) \
  case n: return pencils_n<n>(inverse, data, npencils, Q, S_outer, S_axis, nin, shift, slo, shi, nbatch, batch_stride, s)
    TTM_CASE(16); TTM_CASE(32); TTM_CASE(64); TTM_CASE(128); TTM_CASE(256); TTM_CASE(512);
#undef TTM_CASE
    default: return hipErrorInvalidValue;
  }
}

// ----------------------------------------------------------------------------
// pass 1: axis 0, fused fan-out (Section 2: <f,g> = F^-1(F(f) conj F(g)))
// ----------------------------------------------------------------------------
// BM: the template block's L0 rows occupy the first BM of each thread's R2
// elements (BM = R2: no pruning)
template <int N0, int BM>
__global__ void __launch_bounds__(256) k_pass1(Pass1Args A, long P, int p2, int h2, int L0, int shift0, int lo0,
                                               int hi0) {
  using C = PenCfg<N0>;
  constexpr int R1 = C::R1, R2 = C::R2, PW = C::PW;
  __shared__ float2 lds[PW * N0];
  __shared__ float2 tw[N0];
  const int tid = threadIdx.x;
  fill_twiddles(tw, N0, tid, 256);
  __syncthreads();   // the table is read by the first engine call before its first barrier
  const int pl = tid % PW, a = tid / PW;
  const int p = xcd_tile(blockIdx.x, gridDim.x) * PW + pl;
  // pencils past the last tile's end are transformed as zeros and not stored
  const bool valid = p < P && (p % p2) < h2;
  const unsigned pu = valid ? (unsigned)p : 0u;
  const unsigned P32 = (unsigned)P;
  const unsigned step = (unsigned)R1 * P32;
  const unsigned off = (unsigned)a * P32 + pu;
  float2 x[R2], F[R2], T[R2], y[R2];
  const int nt = A.nt0 + A.nt1;
  // the template rows of entry i, loaded one entry ahead so that their
  // latency overlaps the previous entry's transforms; each load is
  // unconditional (element 0 of the entry where the row is absent, the value
  // then discarded), and only the BM rows the template can occupy are loaded
  float2 nx[R2];
  auto load_rows = [&](int i, float2* dst) {
    const float2* __restrict__ tb = i < A.nt0 ? A.tmpl0 + (long)i * A.tmpl_stride
                                              : A.tmpl1 + (long)(i - A.nt0) * A.tmpl_stride;
#pragma unroll
    for (int b = 0; b < R2; ++b) {
      if (b < BM) {
        const bool ok = valid && a + R1 * b < L0;
        const float2 v = tb[ok ? off + b * step : 0u];
        dst[b] = ok ? v : make_float2(0.0f, 0.0f);
      } else {
        dst[b] = make_float2(0.0f, 0.0f);
      }
    }
  };
  load_rows(0, nx);
#pragma unroll 1
  for (int i = 0; i < nt; ++i) {
    if (i == 0 || i == A.nt0) {
      // forward axis-0 transform of the image tile of this group of entries
      const float2* __restrict__ src = i == 0 ? A.src0 : A.src1;
#pragma unroll
      for (int b = 0; b < R2; ++b) x[b] = src[off + b * step];
      if (!valid) {
#pragma unroll
        for (int b = 0; b < R2; ++b) x[b] = make_float2(0.0f, 0.0f);
      }
      engineA<N0, PW, false>(x, F, lds, tw, pl, a);
    }
#pragma unroll
    for (int b = 0; b < R2; ++b) x[b] = nx[b];
    if (i + 1 < nt) load_rows(i + 1, nx);
    engineA<N0, PW, false, BM>(x, T, lds, tw, pl, a);
#pragma unroll
    for (int j = 0; j < R2; ++j) T[j] = cmulc(F[j], T[j]);
    engineB<N0, PW, true>(T, y, lds, tw, pl, a);
    if (valid) {
      float2* __restrict__ ob = A.out + (long)i * A.out_stride;
#pragma unroll
      for (int g = 0; g < R2; ++g) {
        const int j = (a + R1 * g + shift0) & (N0 - 1);
        if ((unsigned)(j - lo0) <= (unsigned)(hi0 - lo0)) ob[(unsigned)j * P32 + pu] = y[g];
      }
    }
  }
}

template <int N0>
static hipError_t pass1_n(const Geo& g, const Pass1Args& a, hipStream_t s) {
  constexpr int PW = PenCfg<N0>::PW, R1 = PenCfg<N0>::R1, R2 = PenCfg<N0>::R2;
  const long P = (long)g.n1 * g.p2;
  dim3 grid((unsigned)((P + PW - 1) / PW));
  const int bm = (g.L0 + R1 - 1) / R1;
  if (bm == 1)
    hipLaunchKernelGGL((k_pass1<N0, 1>), grid, dim3(256), 0, s, a, P, g.p2, g.h2, g.L0, g.c0, g.lo0(), g.hi0());
  else if (bm == 2)
    hipLaunchKernelGGL((k_pass1<N0, 2>), grid, dim3(256), 0, s, a, P, g.p2, g.h2, g.L0, g.c0, g.lo0(), g.hi0());
  else if (bm <= 4 && R2 > 4)
    hipLaunchKernelGGL((k_pass1<N0, (R2 > 4 ? 4 : R2)>), grid, dim3(256), 0, s, a, P, g.p2, g.h2, g.L0, g.c0,
                       g.lo0(), g.hi0());
  else
    hipLaunchKernelGGL((k_pass1<N0, R2>), grid, dim3(256), 0, s, a, P, g.p2, g.h2, g.L0, g.c0, g.lo0(), g.hi0());
  return hipGetLastError();
}

hipError_t launch_pass1(const Geo& g, const Pass1Args& a, hipStream_t s) {
  if (a.nt0 < 1 || a.nt1 < 0) return hipErrorInvalidValue;
  switch (g.n0) {
    case 16: return pass1_n<16>(g, a, s);
    case 32: return pass1_n<32>(g, a, s);
    case 64: return pass1_n<64>(g, a, s);
    case 128: return pass1_n<128>(g, a, s);
    case 256: return pass1_n<256>(g, a, s);
    case 512: return pass1_n<512>(g, a, s);
    default: return hipErrorInvalidValue;
  }
}

// ----------------------------------------------------------------------------
// pass 3: axis-2 C2R fused with the reduction over pair arrays.
// 2 Z(k) = (X(k) + conj X(M-k)) + i (X(k) - conj X(M-k)) e^{+2 pi i k/N},
// IDFT_M(2Z)(m) = N (x(2m) + i x(2m+1)).
// ----------------------------------------------------------------------------
struct P3Geo {
  int n0, n1, n2, h2, p2;
  int lo0, hi0, lo1, hi1, lo2, hi2;   // valid region, inclusive bounds
  int c2;
  int l1;                             // log2(n1)
  double inv_vol;
  __device__ bool row_valid(long r) const {
    const int x0 = (int)(r >> l1), x1 = (int)(r & (n1 - 1));
    return (unsigned)(x0 - lo0) <= (unsigned)(hi0 - lo0) && (unsigned)(x1 - lo1) <= (unsigned)(hi1 - lo1);
  }
};

template <int M, int MODE>
__global__ void __launch_bounds__(256) k_pass3(P3Geo g, Pass3Args A) {
  constexpr bool SC = MODE == P3_SCORE;                        // score (and optional w) outputs
  constexpr bool MOM = SC || MODE == P3_FIELD;                  // moment pairs first, then components
  using C = RowCfg<M>;
  constexpr int R1 = C::R1, R2 = C::R2, RW = C::RW, SP = C::SP;
  constexpr int N2 = 2 * M, H2 = M + 1;
  __shared__ float2 stage[RW * SP];
  // output stage (pitch N2 + 1: rows on distinct banks), aliasing the input
  // stage, which is free once the last pair has been transformed
  constexpr int OP = N2 + 1;
  static_assert(RW * OP <= 2 * RW * SP, "output stage exceeds the input stage");
  float* const ostage = reinterpret_cast<float*>(stage);
  __shared__ float2 twM[M];
  __shared__ float2 tw2[N2];
  const int tid = threadIdx.x;
  fill_twiddles(twM, M, tid, 256);
  fill_twiddles(tw2, N2, tid, 256);
  const long nrows = (long)g.n0 * g.n1;
  const long r0 = (long)blockIdx.x * RW;
  const int p = tid % RW, a = tid / RW;
  const long myrow = r0 + p;
  const bool myrow_ok = myrow < nrows && g.row_valid(myrow);

  // per-thread element values: e[k*R1+d] holds (x(2n), x(2n+1)), n = (a + R1 k) + R2 d
  float2 wv[R2];     // w (P3_SCORE) or running best (P3_MAX)
  float2 acc[R2];    // sum mu G^2 (P3_SCORE)
  int2 bidx[R2];     // running argmax (P3_MAX)
  double msum = 0.0, floor_v = 0.0, inv_msum = 0.0;
  if (MODE != P3_MAX) {
    msum = A.stats[2];
    inv_msum = 1.0 / msum;
    floor_v = (double)A.eps_v * msum * A.stats[1];
  }
#pragma unroll
  for (int j = 0; j < R2; ++j) {
    wv[j] = make_float2(0.0f, 0.0f);
    acc[j] = make_float2(0.0f, 0.0f);
    bidx[j] = make_int2(0, 0);
  }
  if (MODE == P3_MAX) {
#pragma unroll
    for (int k = 0; k < R2 / R1; ++k)
#pragma unroll
      for (int d = 0; d < R1; ++d) {
        const int n = (a + R1 * k) + R2 * d;
        const int j = k * R1 + d;
        if (A.init || !myrow_ok) {
          wv[j] = make_float2(-INFINITY, -INFINITY);
          bidx[j] = make_int2(0, 0);
        } else {
          const long o0 = myrow * g.n2 + ((2 * n + g.c2) & (N2 - 1));
          const long o1 = myrow * g.n2 + ((2 * n + 1 + g.c2) & (N2 - 1));
          wv[j] = make_float2(A.best[o0], A.best[o1]);
          bidx[j] = make_int2(A.best_idx[o0], A.best_idx[o1]);
        }
      }
  }

  // a tile with no row in the valid region reads nothing: its outputs are zero
  if (!__syncthreads_or(tid < RW && r0 + tid < nrows && g.row_valid(r0 + tid))) {
    if (MODE == P3_MAX) return;
    for (int e = tid; e < RW * N2; e += 256) {
      const long r = r0 + e / N2;
      if (r >= nrows) continue;
      if (SC) {
        A.out_score[r * g.n2 + e % N2] = 0.0f;
        if (A.out_w) A.out_w[r * g.n2 + e % N2] = 0.0f;
      } else {
        A.out_w[r * g.n2 + e % N2] = 0.0f;
      }
    }
    return;
  }

  const int npass = MOM ? A.npairs + 2 : (MODE == P3_W ? 2 : A.npairs);
  // pair order: P3_SCORE and P3_FIELD do M1 (index npairs), M2 (npairs+1),
  // then the components
  auto pair_of = [&](int it) { return MOM ? (it < 2 ? A.npairs + it : it - 2) : it; };
  // software pipeline: the rows of the next pair are fetched into registers
  // while the current pair is transformed (each thread owns a fixed slice of
  // the block's contiguous RW x H2 tile)
  constexpr int PF = (RW * H2 + 255) / 256;
  constexpr int P2 = row_pitch(N2);             // row pitch of the arrays
  // rows are unpadded in memory and in the stage: element e of the block's
  // tile sits at offset e in both
  static_assert(P2 == H2 && SP == H2, "the tile is contiguous in memory and in LDS");
  const long nvalid = (nrows - r0 < RW ? nrows - r0 : RW) * (long)H2;
  // rows outside the valid region are not read (transformed as zeros)
  bool ld_ok[PF];
#pragma unroll
  for (int i = 0; i < PF; ++i) {
    const int e = tid + 256 * i;
    ld_ok[i] = e < nvalid && g.row_valid(r0 + e / H2);
  }
  // unconditional loads (element 0 of the tile in place of a skipped one, the
  // value then discarded), so that no branch sits between them
  float2 pf[PF];
  {
    const float2* Hn = A.H + (long)pair_of(0) * A.pstride + r0 * P2;
#pragma unroll
    for (int i = 0; i < PF; ++i) {
      const int e = tid + 256 * i;
      const float2 v = Hn[ld_ok[i] ? e : 0];
      pf[i] = ld_ok[i] ? v : make_float2(0.0f, 0.0f);
    }
  }
#pragma unroll 1
  for (int it = 0; it < npass; ++it) {
    const int pair = pair_of(it);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < PF; ++i) {
      const int e = tid + 256 * i;
      if (e < RW * H2) stage[e] = pf[i];
    }
    __syncthreads();
    if (it + 1 < npass) {
      const float2* Hn = A.H + (long)pair_of(it + 1) * A.pstride + r0 * P2;
#pragma unroll
      for (int i = 0; i < PF; ++i) {
        const int e = tid + 256 * i;
        const float2 v = Hn[ld_ok[i] ? e : 0];
        pf[i] = ld_ok[i] ? v : make_float2(0.0f, 0.0f);
      }
    }
    float2 z[R2], o[R2];
#pragma unroll
    for (int b = 0; b < R2; ++b) {
      const int k = a + R1 * b;
      const float2 xk = stage[p * SP + k];
      const float2 xm = cconj(stage[p * SP + (M - k)]);
      const float2 s = cadd(xk, xm);
      const float2 q = cmul(csub(xk, xm), cconj(tw2[k]));
      z[b] = make_float2(s.x - q.y, s.y + q.x);
    }
    engineA<M, RW, true>(z, o, stage, twM, p, a);
    if (MOM || MODE == P3_W) {
      if (it == 0) {
#pragma unroll
        for (int j = 0; j < R2; ++j) wv[j] = o[j];               // M1 (unscaled)
      } else if (it == 1) {
#pragma unroll
        for (int j = 0; j < R2; ++j) {
          const double m1x = (double)wv[j].x * g.inv_vol, m1y = (double)wv[j].y * g.inv_vol;
          const double m2x = (double)o[j].x * g.inv_vol, m2y = (double)o[j].y * g.inv_vol;
          // the cancelling subtraction in float64, the reciprocal root in float32
          const double vx = m2x - m1x * m1x * inv_msum, vy = m2y - m1y * m1y * inv_msum;
          wv[j] = make_float2(vx > floor_v ? rsqrtf((float)vx) : 0.0f,
                              vy > floor_v ? rsqrtf((float)vy) : 0.0f);
        }
      } else {
        if (SC) {
          const float mu = A.mu[pair];
#pragma unroll
          for (int j = 0; j < R2; ++j) {
            acc[j].x += mu * o[j].x * o[j].x;
            acc[j].y += mu * o[j].y * o[j].y;
          }
        }
        if (MODE == P3_FIELD) {
          // C_alpha = w G_alpha staged with the axis-2 centre shift, then the
          // valid part of each row stored contiguously in the plane of alpha
          const float fs = (float)g.inv_vol;
          __syncthreads();
#pragma unroll
          for (int k = 0; k < R2 / R1; ++k)
#pragma unroll
            for (int d = 0; d < R1; ++d) {
              const int n = (a + R1 * k) + R2 * d;
              const int j = k * R1 + d;
              ostage[p * OP + ((2 * n + g.c2) & (N2 - 1))] = wv[j].x * o[j].x * fs;
              ostage[p * OP + ((2 * n + 1 + g.c2) & (N2 - 1))] = wv[j].y * o[j].y * fs;
            }
          __syncthreads();
          const int W1 = g.hi1 - g.lo1 + 1, W2 = g.hi2 - g.lo2 + 1;
          float* __restrict__ plane = A.out_C + (long)pair * A.c_plane;
          // row by row (uniform validity), each thread a strided set of columns
#pragma unroll 1
          for (int rr = 0; rr < RW; ++rr) {
            const long r = r0 + rr;
            if (r >= nrows || !g.row_valid(r)) continue;
            const int x0 = (int)(r >> g.l1), x1 = (int)(r & (g.n1 - 1));
            float* __restrict__ prow = plane + ((long)(x0 - g.lo0) * W1 + (x1 - g.lo1)) * W2 - g.lo2;
            for (int x2 = g.lo2 + tid; x2 <= g.hi2; x2 += 256) prow[x2] = ostage[rr * OP + x2];
          }
        }
      }
    } else {
      const int idx = A.first_index + pair;
#pragma unroll
      for (int j = 0; j < R2; ++j) {
        if (o[j].x > wv[j].x) { wv[j].x = o[j].x; bidx[j].x = idx; }
        if (o[j].y > wv[j].y) { wv[j].y = o[j].y; bidx[j].y = idx; }
      }
    }
  }

  if (MODE == P3_MAX) {
    if (myrow_ok) {
#pragma unroll
      for (int k = 0; k < R2 / R1; ++k)
#pragma unroll
        for (int d = 0; d < R1; ++d) {
          const int n = (a + R1 * k) + R2 * d;
          const int j = k * R1 + d;
          const long o0 = myrow * g.n2 + ((2 * n + g.c2) & (N2 - 1));
          const long o1 = myrow * g.n2 + ((2 * n + 1 + g.c2) & (N2 - 1));
          A.best[o0] = wv[j].x;
          A.best[o1] = wv[j].y;
          A.best_idx[o0] = bidx[j].x;
          A.best_idx[o1] = bidx[j].y;
        }
    }
    return;
  }

  // stage the outputs in LDS with the axis-2 centre shift, then store rows
  const float fscale = (float)g.inv_vol;
#pragma unroll 1
  for (int outk = 0; outk < 2; ++outk) {
    float* dst = outk == 0 ? (SC ? A.out_score : A.out_w) : (SC ? A.out_w : nullptr);
    if (dst == nullptr) break;
    const bool is_w = !SC || outk == 1;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < R2 / R1; ++k)
#pragma unroll
      for (int d = 0; d < R1; ++d) {
        const int n = (a + R1 * k) + R2 * d;
        const int j = k * R1 + d;
        float v0, v1;
        if (is_w) {
          v0 = wv[j].x;
          v1 = wv[j].y;
        } else {
          v0 = wv[j].x * sqrtf(acc[j].x) * fscale;
          v1 = wv[j].y * sqrtf(acc[j].y) * fscale;
        }
        ostage[p * OP + ((2 * n + g.c2) & (N2 - 1))] = v0;
        ostage[p * OP + ((2 * n + 1 + g.c2) & (N2 - 1))] = v1;
      }
    __syncthreads();
    for (int e = tid; e < RW * N2; e += 256) {
      const int rr = e / N2, x2 = e % N2;
      const long r = r0 + rr;
      if (r >= nrows) continue;
      const int x0 = (int)(r / g.n1), x1 = (int)(r % g.n1);
      const bool ok = x0 >= g.lo0 && x0 <= g.hi0 && x1 >= g.lo1 && x1 <= g.hi1 && x2 >= g.lo2 && x2 <= g.hi2;
      dst[r * g.n2 + x2] = ok ? ostage[rr * OP + x2] : 0.0f;
    }
  }
}

static P3Geo make_p3geo(const Geo& g) {
  P3Geo q;
  q.n0 = g.n0; q.n1 = g.n1; q.n2 = g.n2; q.h2 = g.h2; q.p2 = g.p2;
  q.lo0 = g.c0; q.hi0 = g.n0 - g.L0 + g.c0;
  q.lo1 = g.c1; q.hi1 = g.n1 - g.L1 + g.c1;
  q.lo2 = g.c2; q.hi2 = g.n2 - g.L2 + g.c2;
  q.c2 = g.c2;
  q.l1 = 0;
  while ((1 << q.l1) < g.n1) ++q.l1;
  q.inv_vol = 1.0 / (double)g.vol();
  return q;
}

template <int M>
static hipError_t pass3_m(const Geo& g, const Pass3Args& a, hipStream_t s) {
  constexpr int RW = RowCfg<M>::RW;
  const long nrows = (long)g.n0 * g.n1;
  dim3 grid((unsigned)((nrows + RW - 1) / RW));
  const P3Geo q = make_p3geo(g);
  switch (a.mode) {
    case P3_SCORE: hipLaunchKernelGGL((k_pass3<M, P3_SCORE>), grid, dim3(256), 0, s, q, a); break;
    case P3_W: hipLaunchKernelGGL((k_pass3<M, P3_W>), grid, dim3(256), 0, s, q, a); break;
    case P3_MAX: hipLaunchKernelGGL((k_pass3<M, P3_MAX>), grid, dim3(256), 0, s, q, a); break;
    case P3_FIELD: hipLaunchKernelGGL((k_pass3<M, P3_FIELD>), grid, dim3(256), 0, s, q, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_pass3(const Geo& g, const Pass3Args& a, hipStream_t s) {
  switch (g.n2) {
    case 16: return pass3_m<8>(g, a, s);
    case 32: return pass3_m<16>(g, a, s);
    case 64: return pass3_m<32>(g, a, s);
    case 128: return pass3_m<64>(g, a, s);
    case 256: return pass3_m<128>(g, a, s);
    case 512: return pass3_m<256>(g, a, s);
    default: return hipErrorInvalidValue;
  }
}

// ----------------------------------------------------------------------------
// the correlated tensor field at candidate voxels, read from the K arrays
// after their axis-0 and axis-1 inverse passes: for the row (x0, x1) of array
// alpha, G(y) = Re Y(0) + (-1)^y Re Y(M) + 2 sum_{k=1}^{M-1} Re(Y(k) e^{2 pi i k y / n2})
// (unnormalised inverse real DFT at one point), y = x2 - c2 mod n2;
// C_alpha(x) = w(x) G / (n0 n1 n2).  One block per (candidate, neighbour row).
// ----------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_field_at(P3Geo g, const float2* __restrict__ H, long pstride, int K,
                                                  const float* __restrict__ wmap, int refine,
                                                  const int* __restrict__ pos, const int* __restrict__ count_dev,
                                                  int count_host, double* __restrict__ Cbuf,
                                                  double* __restrict__ wbuf, int* __restrict__ okbuf,
                                                  const int* __restrict__ active) {
  extern __shared__ float2 twf[];            // n2 entries: (cos, sin)(2 pi j / n2)
  const int rows = refine ? 9 : 1;
  const int NB = refine ? 27 : 1;
  const int b = blockIdx.x;
  const int p = b / rows, r = b % rows;
  const int count = count_dev ? count_dev[0] : count_host;
  if (p >= count || (active && !active[p])) return;
  const int tid = threadIdx.x;
  for (int j = tid; j < g.n2; j += 256) {
    float sn, cs;
    sincospif(2.0f * (float)j / (float)g.n2, &sn, &cs);
    twf[j] = make_float2(cs, sn);
  }
  __syncthreads();
  const int o0 = refine ? r / 3 - 1 : 0, o1 = refine ? r % 3 - 1 : 0;
  const int x0 = pos[3 * p] + o0, x1 = pos[3 * p + 1] + o1;
  const int npt = refine ? 3 : 1;
  const int M = g.n2 / 2;
  const bool row_ok = x0 >= g.lo0 && x0 <= g.hi0 && x1 >= g.lo1 && x1 <= g.hi1;
  for (int pr = tid; pr < K * npt; pr += 256) {
    const int alpha = pr / npt, pt = pr % npt;
    const int o2 = refine ? pt - 1 : 0;
    const int x2 = pos[3 * p + 2] + o2;
    const int k = refine ? (o0 + 1) * 9 + (o1 + 1) * 3 + (o2 + 1) : 0;
    const long cb = (long)p * NB + k;
    const bool ok = row_ok && x2 >= g.lo2 && x2 <= g.hi2;
    if (!ok) {
      Cbuf[cb * K + alpha] = 0.0;
      if (alpha == 0) {
        okbuf[cb] = 0;
        wbuf[cb] = 0.0;
      }
      continue;
    }
    const int y = ((x2 - g.c2) % g.n2 + g.n2) % g.n2;
    const float2* row = H + (long)alpha * pstride + ((long)x0 * g.n1 + x1) * g.p2;
    double acc = (double)row[0].x + ((y & 1) ? -(double)row[M].x : (double)row[M].x);
    double s2 = 0.0;
    int ph = y;
    for (int kk = 1; kk < M; ++kk, ph += y) {
      const float2 v = row[kk];
      const float2 w = twf[ph & (g.n2 - 1)];
      s2 += (double)v.x * w.x - (double)v.y * w.y;
    }
    acc += 2.0 * s2;
    const double wv = (double)wmap[((long)x0 * g.n1 + x1) * g.n2 + x2];
    Cbuf[cb * K + alpha] = wv * acc * g.inv_vol;
    if (alpha == 0) {
      okbuf[cb] = 1;
      wbuf[cb] = wv;
    }
  }
}

hipError_t launch_field_at(const Geo& gg, const float2* H, long pstride, int K, const float* wmap,
                           int max_peaks, int refine, const int* pos_in, const int* count_dev, int count_host,
                           const PoseScratch& ps, hipStream_t s) {
  const P3Geo q = make_p3geo(gg);
  const unsigned nblk = (unsigned)(max_peaks * (refine ? 9 : 1));
  hipLaunchKernelGGL(k_field_at, dim3(nblk), dim3(256), sizeof(float2) * gg.n2, s, q, H, pstride, K, wmap,
                     refine, pos_in, count_dev, count_host, ps.C, ps.w, ps.ok, ps.active);
  return hipGetLastError();
}

// ----------------------------------------------------------------------------
// classical epilogue and fills
// ----------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_classical_final(P3Geo g, const float* __restrict__ w,
                                                         float* __restrict__ best, int* __restrict__ idx) {
  const long n = (long)g.n0 * g.n1 * g.n2;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const int x2 = (int)(i % g.n2);
    const long r = i / g.n2;
    const int x1 = (int)(r % g.n1), x0 = (int)(r / g.n1);
    const bool ok = x0 >= g.lo0 && x0 <= g.hi0 && x1 >= g.lo1 && x1 <= g.hi1 && x2 >= g.lo2 && x2 <= g.hi2;
    if (!ok) {
      best[i] = 0.0f;
      idx[i] = -1;
    } else {
      const float wi = w[i];
      if (wi > 0.0f) {
        best[i] = (float)((double)best[i] * (double)wi * g.inv_vol);
      } else {
        best[i] = 0.0f;
        idx[i] = 0;
      }
    }
  }
}

hipError_t launch_classical_final(const Geo& g, const float* w, float* best, int* idx,
                                  hipStream_t s) {
  const P3Geo q = make_p3geo(g);
  hipLaunchKernelGGL(k_classical_final, dim3(2048), dim3(256), 0, s, q, w, best, idx);
  return hipGetLastError();
}

__global__ void k_fill_f32(float* p, long n, float v) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) p[i] = v;
}
__global__ void k_fill_i32(int* p, long n, int v) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) p[i] = v;
}
hipError_t launch_fill_f32(float* p, long n, float v, hipStream_t s) {
  const unsigned nb = (unsigned)std::min<long>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_fill_f32, dim3(nb > 0 ? nb : 1), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}
hipError_t launch_fill_i32(int* p, long n, int v, hipStream_t s) {
  const unsigned nb = (unsigned)std::min<long>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_fill_i32, dim3(nb > 0 ? nb : 1), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

}  // namespace ttm
