// The inverse half of the correlation in two passes over HBM (Section 2, FFT
// inner products <f, g> = F^-1(F(f) conj F(g)); Algorithm 1), for images
// whose axes 1 and 2 are 256 long.
//
// The inverse transform along axis 1 (length n1 = 4 Q) is split into two
// digits, k1 = kb + Q ka and j1 = ja + 4 jb:
//   y(ja + 4 jb) = sum_kb e^{2 pi i jb kb / Q} [ e^{2 pi i ja kb / n1}
//                  sum_ka X(kb + Q ka) e^{2 pi i ja ka / 4} ].
// Pass A (k_pass1x) transforms axis 0 and the 4-point digit: a block holds
// 8 neighbouring columns q = kb h2 + k2 of the four planes ka (32 pencils of
// axis 0), so every global access moves runs of 8 complex values (64 bytes);
// after the axis-0 inverse the four ka pencils of a column sit in lanes that
// differ in bits 3 and 4 and are combined by cross-lane exchanges.  It writes
// Z[x0][ja][kb][k2] (the valid planes x0 only).
// Pass B (k_pass3x) reads one contiguous [Q][h2] tile Z[x0][ja] per array,
// finishes axis 1 (a Q-point transform of each column, the columns k2 = 0
// and n2/2 packed into one: both are real once axes 0 and 1 are inverted),
// then axis 2 (C2R rows), and reduces the arrays into the local norm w and
// the score F = w sqrt(sum mu G^2) / V of Section 3.4 for the Q rows
// x1 = ja + 4 jb (+ the centre shift) of plane x0.
//
// Against the three-pass path (axis 0, then axis 1 in place, then axis 2)
// this removes one read and one write of every array.
#include "ttm_device.h"
#include "ttm_internal.h"

namespace ttm {

namespace {

// v from the lane whose index is this lane's xor X (X = 4, 8 or 16): a
// rotation by 8 within each row of 16 lanes for X = 8 (DPP), else a
// bit-mask swizzle within each group of 32 lanes
template <int X>
__device__ __forceinline__ float2 lane_xor(float2 v) {
  if constexpr (X == 8) {
    constexpr int kRor8 = 0x128;   // DPP row_ror:8
    return make_float2(__int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v.x), kRor8, 0xF, 0xF, false)),
                       __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v.y), kRor8, 0xF, 0xF, false)));
  } else {
    static_assert(X == 4 || X == 16, "xor partner within 32 lanes");
    constexpr int kPat = (X << 10) | 0x1F;   // and 0x1F, or 0, xor X
    return make_float2(__int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v.x), kPat)),
                       __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v.y), kPat)));
  }
}
// engineA (ttm_device.h) with its outputs handed to `use(k, z)` one task of
// R1 values at a time (z[d] = X(c + R2 d), c = a + R1 k) instead of being
// collected, so that only R1 outputs are live at once
template <int N, int PW, bool INV, class Use>
__device__ __forceinline__ void engineA_each(float2 (&x)[Plan<N>::R2], float2* lds, const float2* tw, int p, int a,
                                             Use&& use) {
  constexpr int R1 = Plan<N>::R1, R2 = Plan<N>::R2;
  fft_reg<R2, INV>(x);
#pragma unroll
  for (int c = 1; c < R2; ++c) x[c] = twiddle<INV>(x[c], tw, (a * c) & (N - 1));
  __syncthreads();
#pragma unroll
  for (int c = 0; c < R2; ++c) lds[(c * R1 + a) * PW + p] = x[c];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < R2 / R1; ++k) {
    const int c = a + R1 * k;
    float2 z[R1];
#pragma unroll
    for (int j = 0; j < R1; ++j) z[j] = lds[(c * R1 + j) * PW + p];
    fft_reg<R1, INV>(z);
    use(k, z);
  }
}

}  // namespace

// ----------------------------------------------------------------------------
// pass A: axis 0 (fused forward transform of the pruned template rows, the
// product with the conjugate, the inverse) and the 4-point digit of axis 1
// ----------------------------------------------------------------------------
// CW columns per block, 4 CW pencils (the four planes ka of each column)
constexpr int kColsA = 8;

template <int N0, int BM, int CW>
__global__ void __launch_bounds__(4 * CW * Plan<N0>::R1)
    k_pass1x(Pass1Args A, int QH, int h2, int n1, int L0, int shift0, int lo0, int hi0) {
  constexpr int R1 = Plan<N0>::R1, R2 = Plan<N0>::R2, PW = 4 * CW;
  constexpr int kColsA = CW;
  __shared__ float2 lds[PW * N0];
  __shared__ float2 tw[N0];
  const int tid = threadIdx.x;
  fill_twiddles(tw, N0, tid, PW * R1);
  __syncthreads();   // the table is read by the first engine call before its first barrier
  const int pl = tid % PW, a = tid / PW;
  const int c = pl % kColsA, ka = pl / kColsA;
  const int q = xcd_tile(blockIdx.x, gridDim.x) * kColsA + c;
  // columns past the end are transformed as zeros and not stored
  const bool valid = q < QH;
  const unsigned qu = valid ? (unsigned)q : 0u;
  const unsigned P32 = (unsigned)n1 * (unsigned)h2;       // elements between axis-0 rows
  const unsigned step = (unsigned)R1 * P32;
  const unsigned off = (unsigned)a * P32 + qu + (unsigned)ka * (unsigned)QH;
  // the 4-point digit: X = (x0, x1, x2, x3) over ka = 2 h + l, first
  // A(h', l) = X(l) + (-1)^h' X(2 + l) across bit h (lanes xor 2 CW), held by
  // the lane (h = h', l); then Y(h' + 2 l') = A(h', 0) + i^(h' + 2 l') A(h', 1)
  // across bit l (lanes xor CW), held by the lane (h = h', l = l').  So the
  // lane ends with ja = h + 2 l, and each step is s y + p or a y + b p with
  // per-lane constants (the second scaled by e^{2 pi i ja kb / n1}).
  const int h = ka >> 1, l = ka & 1;
  const int ja = h + 2 * l;
  const int kb = (int)(qu / (unsigned)h2);
  float ts, tc;
  sincospif(2.0f * (float)(ja * kb) / (float)n1, &ts, &tc);
  const float2 twz = make_float2(tc, ts);
  const float sA = h == 0 ? 1.0f : -1.0f;
  // l = 0: Y = A0 + i^h A1 (own A0, partner A1); l = 1: Y = A0 - i^h A1
  // (own A1, partner A0)
  const float2 ih = h ? make_float2(0.0f, 1.0f) : make_float2(1.0f, 0.0f);
  const float2 cOwn = cmul(l == 0 ? make_float2(1.0f, 0.0f) : make_float2(-ih.x, -ih.y), twz);
  const float2 cPar = cmul(l == 0 ? ih : make_float2(1.0f, 0.0f), twz);
  float2 x[R2], F[R2], T[R2], y[R2];
  const int nt = A.nt0 + A.nt1;
  // the template rows of entry i, loaded one entry ahead (unconditional
  // loads from a clamped index, the value discarded where absent)
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
    // the 4-point inverse DFT across the planes ka
#pragma unroll
    for (int g = 0; g < R2; ++g) {
      const float2 p = lane_xor<2 * CW>(y[g]);
      y[g] = make_float2(sA * y[g].x + p.x, sA * y[g].y + p.y);
    }
#pragma unroll
    for (int g = 0; g < R2; ++g) {
      const float2 p = lane_xor<CW>(y[g]);
      y[g] = cadd(cmul(y[g], cOwn), cmul(p, cPar));
    }
    if (valid) {
      float2* __restrict__ ob = A.out + (long)i * A.out_stride + (unsigned)ja * (unsigned)QH + qu;
#pragma unroll
      for (int g = 0; g < R2; ++g) {
        const int j = (a + R1 * g + shift0) & (N0 - 1);
        if ((unsigned)(j - lo0) <= (unsigned)(hi0 - lo0)) ob[(unsigned)j * 4u * (unsigned)QH] = y[g];
      }
    }
  }
}

template <int N0>
static hipError_t pass1x_n(const Geo& g, const Pass1Args& a, hipStream_t s) {
  constexpr int R1 = Plan<N0>::R1, R2 = Plan<N0>::R2, CW = kColsA;
  const int Q = g.n1 / 4;
  const int QH = Q * g.h2;
  dim3 grid((unsigned)((QH + CW - 1) / CW));
  dim3 block(4 * CW * R1);
  const int bm = (g.L0 + R1 - 1) / R1;
  if (bm == 1)
    hipLaunchKernelGGL((k_pass1x<N0, 1, CW>), grid, block, 0, s, a, QH, g.h2, g.n1, g.L0, g.c0, g.lo0(), g.hi0());
  else if (bm == 2)
    hipLaunchKernelGGL((k_pass1x<N0, 2, CW>), grid, block, 0, s, a, QH, g.h2, g.n1, g.L0, g.c0, g.lo0(), g.hi0());
  else if (bm <= 4 && R2 > 4)
    hipLaunchKernelGGL((k_pass1x<N0, (R2 > 4 ? 4 : R2), CW>), grid, block, 0, s, a, QH, g.h2, g.n1, g.L0, g.c0,
                       g.lo0(), g.hi0());
  else
    hipLaunchKernelGGL((k_pass1x<N0, R2, CW>), grid, block, 0, s, a, QH, g.h2, g.n1, g.L0, g.c0, g.lo0(), g.hi0());
  return hipGetLastError();
}

// ----------------------------------------------------------------------------
// pass B: the Q-point digit of axis 1, axis-2 C2R, local norm and score
// ----------------------------------------------------------------------------
constexpr int kQ = 64;                    // Q = n1 / 4
constexpr int kM = 128;                   // M = n2 / 2
constexpr int kThreadsB = 512;
constexpr int kColP = kM;                 // pitch of the column stage (complex)
constexpr int kRowP = kM + 1;             // pitch of the row stage (complex)
constexpr int kOutP = 2 * kM + 1;         // pitch of the output stage (floats)
constexpr int kStageB = kQ * kRowP > 16 * 4 * kColP ? kQ * kRowP : 16 * 4 * kColP;
static_assert(kOutP * kQ <= 2 * kStageB, "output stage exceeds the shared stage");
static_assert(kQ * kM == 16 * kThreadsB, "one column element per thread and digit");

struct P3xGeo {
  int n0, n1, n2, h2;
  int lo0, hi0, lo1, hi1, lo2, hi2;
  int c1, c2;
  long tile;          // complex elements of one [Q][h2] tile
  double inv_vol;
};

// A.out_w is required here: w is written once the moments are transformed
// and read back for the score at the end (no registers held across arrays)
__global__ void __launch_bounds__(kThreadsB) __attribute__((amdgpu_waves_per_eu(4, 4)))
    k_pass3x(P3xGeo g, Pass3Args A) {
  constexpr int N2 = 2 * kM;
  constexpr int R1 = Plan<kM>::R1, R2 = Plan<kM>::R2;   // row transforms: 8 x 16
  static_assert(kThreadsB / R1 == kQ, "one row per lane of a wave");
  __shared__ float2 stage[kStageB];
  __shared__ float2 twM[kM];
  __shared__ float2 tw2[N2];
  __shared__ float2 twQ[kQ];
  float* const ostage = reinterpret_cast<float*>(stage);
  const int tid = threadIdx.x;
  fill_twiddles(twM, kM, tid, kThreadsB);
  fill_twiddles(tw2, N2, tid, kThreadsB);
  fill_twiddles(twQ, kQ, tid, kThreadsB);
  const int x0 = blockIdx.x >> 2, ja = blockIdx.x & 3;
  // rows of this block: x1 = (ja + 4 jb + c1) mod n1, jb < Q
  const bool plane_ok = x0 >= g.lo0 && x0 <= g.hi0;
  if (!plane_ok) {
    // no array holds this plane: its outputs are zero
    for (int e = tid; e < kQ * N2; e += kThreadsB) {
      const int jb = e / N2, x2 = e % N2;
      const int x1 = (ja + 4 * jb + g.c1) & (g.n1 - 1);
      const long o = ((long)x0 * g.n1 + x1) * g.n2 + x2;
      A.out_score[o] = 0.0f;
      if (A.out_w) A.out_w[o] = 0.0f;
    }
    return;
  }
  // column phase: thread (k2, kq) holds the elements kb = kq + 4 b of column k2
  int k2 = tid & (kM - 1), kq = tid >> 7;
  // row phase: thread (p = row jb, a)
  int p = tid & (kQ - 1), a = tid >> 6;
  const double msum = A.stats[2];
  const double inv_msum = 1.0 / msum;
  const double floor_v = (double)A.eps_v * msum * A.stats[1];
  const long tile_off = ((long)x0 * 4 + ja) * g.tile;
  const int npass = A.npairs + 2;
  auto pair_of = [&](int it) { return it < 2 ? A.npairs + it : it - 2; };
  // the column elements of an array, with column 0 carrying column M in its
  // imaginary part (both real after the inverse transforms of axes 0 and 1)
  constexpr unsigned kH2 = kM + 1;          // the tile's row pitch (complex)
  auto load = [&](int it, float2* v) {
    const unsigned eoff = (unsigned)kq * kH2 + (unsigned)k2;
    const float2* __restrict__ Z = A.H + (long)pair_of(it) * A.pstride + tile_off;
#pragma unroll
    for (int b = 0; b < 16; ++b) v[b] = Z[eoff + (unsigned)b * 4u * kH2];
    if (k2 == 0) {
#pragma unroll
      for (int b = 0; b < 16; ++b) {
        const float2 zm = Z[eoff + (unsigned)b * 4u * kH2 + kM];
        v[b] = make_float2(v[b].x - zm.y, v[b].y + zm.x);
      }
    }
  };
  float2 acc[R2];
#pragma unroll
  for (int j = 0; j < R2; ++j) acc[j] = make_float2(0.0f, 0.0f);
  // stores whole rows of a staged [Q][N2] float block (in transform order:
  // the axis-2 centre shift is applied as the rows are read), zero outside
  // the valid region
  auto store_rows = [&](float* dst) {
    for (int e = tid; e < kQ * N2; e += kThreadsB) {
      const int jb = e / N2, x2 = e % N2;
      const int x1 = (ja + 4 * jb + g.c1) & (g.n1 - 1);
      const bool ok = x1 >= g.lo1 && x1 <= g.hi1 && x2 >= g.lo2 && x2 <= g.hi2;
      dst[((long)x0 * g.n1 + x1) * g.n2 + x2] = ok ? ostage[jb * kOutP + ((x2 - g.c2) & (N2 - 1))] : 0.0f;
    }
  };
  auto stage_values = [&](const float2* val) {
#pragma unroll
    for (int k = 0; k < R2 / R1; ++k)
#pragma unroll
      for (int d = 0; d < R1; ++d) {
        const int n = (a + R1 * k) + R2 * d;
        const int j = k * R1 + d;
        ostage[p * kOutP + 2 * n] = val[j].x;
        ostage[p * kOutP + 2 * n + 1] = val[j].y;
      }
  };
  __syncthreads();   // twiddle tables
#pragma unroll 1
  for (int it = 0; it < npass; ++it) {
    // the lane coordinates are made opaque here, so that the LDS and global
    // addresses derived from them are recomputed in each iteration instead
    // of being hoisted out of the loop and held in registers
    asm volatile("" : "+v"(k2), "+v"(kq), "+v"(p), "+v"(a));
    float2 v[16];
    load(it, v);
    // 16-point inverse transform over b, then e^{2 pi i s kq / Q}
    fft_reg<16, true>(v);
#pragma unroll
    for (int s = 1; s < 16; ++s) v[s] = twiddle<true>(v[s], twQ, s * kq);
    __syncthreads();
#pragma unroll
    for (int s = 0; s < 16; ++s) stage[(kq * 16 + s) * kColP + k2] = v[s];
    __syncthreads();
    // 4-point transforms over kq for s = 4 kq' + t: outputs jb = s + 16 r
    float2 yv[16];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int s = 4 * kq + t;
      float2 z[4];
#pragma unroll
      for (int m = 0; m < 4; ++m) z[m] = stage[(m * 16 + s) * kColP + k2];
      fft_reg<4, true>(z);
#pragma unroll
      for (int r = 0; r < 4; ++r) yv[4 * t + r] = z[r];
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) stage[(4 * kq + t + 16 * r) * kRowP + k2] = yv[4 * t + r];
    __syncthreads();
    // row p: C2R through the half-length complex transform
    // 2 Z(k) = (X(k) + conj X(M-k)) + i (X(k) - conj X(M-k)) e^{+2 pi i k / N2}
    float2 z[R2];
#pragma unroll
    for (int b = 0; b < R2; ++b) {
      const int k = a + R1 * b;
      float2 xk, xm;
      if (k == 0) {
        const float2 pk = stage[p * kRowP];
        xk = make_float2(pk.x, 0.0f);     // X(0), real
        xm = make_float2(pk.y, 0.0f);     // conj X(M), real
      } else {
        xk = stage[p * kRowP + k];
        xm = cconj(stage[p * kRowP + (kM - k)]);
      }
      const float2 s = cadd(xk, xm);
      const float2 qd = cmul(csub(xk, xm), cconj(tw2[k]));
      z[b] = make_float2(s.x - qd.y, s.y + qd.x);
    }
    if (it == 0) {
      // M1 (unscaled)
      engineA_each<kM, kQ, true>(z, stage, twM, p, a, [&](int k, const float2* o) {
#pragma unroll
        for (int d = 0; d < R1; ++d) acc[k * R1 + d] = o[d];
      });
    } else if (it == 1) {
      // w from M1 and M2: the cancelling subtraction in float64, the
      // reciprocal root in float32
      engineA_each<kM, kQ, true>(z, stage, twM, p, a, [&](int k, const float2* o) {
#pragma unroll
        for (int d = 0; d < R1; ++d) {
          const int j = k * R1 + d;
          const double m1x = (double)acc[j].x * g.inv_vol, m1y = (double)acc[j].y * g.inv_vol;
          const double m2x = (double)o[d].x * g.inv_vol, m2y = (double)o[d].y * g.inv_vol;
          const double vx = m2x - m1x * m1x * inv_msum, vy = m2y - m1y * m1y * inv_msum;
          acc[j] = make_float2(vx > floor_v ? rsqrtf((float)vx) : 0.0f, vy > floor_v ? rsqrtf((float)vy) : 0.0f);
        }
      });
      // w out now, read back for the score at the end
      __syncthreads();
      stage_values(acc);
      __syncthreads();
      store_rows(A.out_w);
#pragma unroll
      for (int j = 0; j < R2; ++j) acc[j] = make_float2(0.0f, 0.0f);
    } else {
      const float mu = A.mu[pair_of(it)];
      engineA_each<kM, kQ, true>(z, stage, twM, p, a, [&](int k, const float2* o) {
#pragma unroll
        for (int d = 0; d < R1; ++d) {
          acc[k * R1 + d].x += mu * o[d].x * o[d].x;
          acc[k * R1 + d].y += mu * o[d].y * o[d].y;
        }
      });
    }
  }
  // F = w sqrt(sum mu G^2) / V, with w read back from this block's own rows
  const float fscale = (float)g.inv_vol;
#pragma unroll
  for (int j = 0; j < R2; ++j) acc[j] = make_float2(sqrtf(acc[j].x) * fscale, sqrtf(acc[j].y) * fscale);
  __syncthreads();
  stage_values(acc);
  __syncthreads();
  for (int e = tid; e < kQ * N2; e += kThreadsB) {
    const int jb = e / N2, x2 = e % N2;
    const int x1 = (ja + 4 * jb + g.c1) & (g.n1 - 1);
    const bool ok = x1 >= g.lo1 && x1 <= g.hi1 && x2 >= g.lo2 && x2 <= g.hi2;
    const long o = ((long)x0 * g.n1 + x1) * g.n2 + x2;
    A.out_score[o] = ok ? A.out_w[o] * ostage[jb * kOutP + ((x2 - g.c2) & (N2 - 1))] : 0.0f;
  }
}

bool two_pass_supported(const Geo& g) {
  return g.n1 == 4 * kQ && g.n2 == 2 * kM && supported_len(g.n0) && g.n0 <= 256 && g.planar == 0;
}

hipError_t launch_pass1x(const Geo& g, const Pass1Args& a, hipStream_t s) {
  if (!two_pass_supported(g) || a.nt0 < 1 || a.nt1 < 0) return hipErrorInvalidValue;
  switch (g.n0) {
    case 16: return pass1x_n<16>(g, a, s);
    case 32: return pass1x_n<32>(g, a, s);
    case 64: return pass1x_n<64>(g, a, s);
    case 128: return pass1x_n<128>(g, a, s);
    case 256: return pass1x_n<256>(g, a, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_pass3x(const Geo& g, const Pass3Args& a, hipStream_t s) {
  if (!two_pass_supported(g) || a.mode != P3_SCORE || !a.out_w) return hipErrorInvalidValue;
  P3xGeo q;
  q.n0 = g.n0; q.n1 = g.n1; q.n2 = g.n2; q.h2 = g.h2;
  q.lo0 = g.lo0(); q.hi0 = g.hi0();
  q.lo1 = g.lo1(); q.hi1 = g.hi1();
  q.lo2 = g.c2; q.hi2 = g.n2 - g.L2 + g.c2;
  q.c1 = g.c1; q.c2 = g.c2;
  q.tile = (long)kQ * g.h2;
  q.inv_vol = 1.0 / (double)g.vol();
  hipLaunchKernelGGL(k_pass3x, dim3((unsigned)(g.n0 * 4)), dim3(kThreadsB), 0, s, q, a);
  return hipGetLastError();
}

}  // namespace ttm
