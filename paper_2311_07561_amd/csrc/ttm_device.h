// Device building blocks for libttm (gfx950, wave64): complex arithmetic,
// in-register power-of-two DFTs with compile-time twiddles, and two-stage
// LDS-exchanged FFT engines for lengths N = R1 * R2.
//
// Two-stage decomposition used by every FFT here (Cooley-Tukey with
// n = a + R1 b and k = c + R2 d):
//   X(c + R2 d) = sum_a W_R1^{a d} W_N^{a c} sum_b x(a + R1 b) W_R2^{b c}
// "Engine A" takes thread a holding x(a + R1 b), b < R2 (natural layout), and
// leaves the thread owning tasks c = a + R1 k holding X(c + R2 d), d < R1
// (task layout).  "Engine B" is the transpose: task layout in, natural
// layout out.  Both run in either direction.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <type_traits>

namespace ttm {

// ----------------------------------------------------------------------------
// complex float helpers
// ----------------------------------------------------------------------------
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {
  return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }

// ----------------------------------------------------------------------------
// compile-time loops
// ----------------------------------------------------------------------------
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

constexpr int ilog2(int v) { return v <= 1 ? 0 : 1 + ilog2(v >> 1); }
constexpr int bitrev(int v, int bits) {
  int r = 0;
  for (int i = 0; i < bits; ++i) r |= ((v >> i) & 1) << (bits - 1 - i);
  return r;
}

// cos(2 pi k / 32) for k in [0, 8] (first quarter wave)
constexpr float kCosQ[9] = {
    1.0f, 0.980785280403230449126f, 0.923879532511286756128f,
    0.831469612302545237079f, 0.707106781186547524401f,
    0.555570233019602224743f, 0.382683432365089771728f,
    0.195090322016128267848f, 0.0f};

constexpr float cos32(int k) {
  k &= 31;
  return k <= 8 ? kCosQ[k] : k <= 16 ? -kCosQ[16 - k] : k <= 24 ? -kCosQ[k - 16] : kCosQ[32 - k];
}
constexpr float sin32(int k) { return cos32(k - 8); }

// v * W_32^k with W = exp(-2 pi i / 32) (forward) or exp(+2 pi i / 32) (inverse)
template <int K, bool INV>
__device__ __forceinline__ float2 twmul32(float2 v) {
  constexpr int k = K & 31;
  if constexpr (k == 0) {
    return v;
  } else if constexpr (k == 16) {
    return make_float2(-v.x, -v.y);
  } else if constexpr (k == 8) {
    return INV ? make_float2(-v.y, v.x) : make_float2(v.y, -v.x);
  } else if constexpr (k == 24) {
    return INV ? make_float2(v.y, -v.x) : make_float2(-v.y, v.x);
  } else {
    constexpr float c = cos32(k);
    constexpr float s = sin32(k);
    if constexpr (INV)
      return make_float2(v.x * c - v.y * s, v.y * c + v.x * s);
    else
      return make_float2(v.x * c + v.y * s, v.y * c - v.x * s);
  }
}

// In-register DFT of length R (power of two, 2..32), natural order in and out.
// Unnormalised: forward sum x(n) e^{-2 pi i n k / R}, inverse with +.
template <int R, bool INV>
__device__ __forceinline__ void fft_reg(float2 (&x)[R]) {
  static_assert(R >= 1 && R <= 32 && (R & (R - 1)) == 0, "radix must be a power of two <= 32");
  if constexpr (R > 1) {
    constexpr int LG = ilog2(R);
    // radix-2 decimation in frequency
    static_for<0, LG>([&](auto s) {
      constexpr int span = R >> (s + 1);
      static_for<0, R / 2>([&](auto b) {
        constexpr int grp = b / span;
        constexpr int j = b % span;
        constexpr int i0 = grp * 2 * span + j;
        constexpr int i1 = i0 + span;
        const float2 u = x[i0];
        const float2 v = x[i1];
        x[i0] = cadd(u, v);
        x[i1] = twmul32<j * (32 / (2 * span)), INV>(csub(u, v));
      });
    });
    float2 y[R];
    static_for<0, R>([&](auto k) { y[k] = x[bitrev(k, LG)]; });
    static_for<0, R>([&](auto k) { x[k] = y[k]; });
  }
}

// fft_reg for an input whose entries b >= BM are zero: y(k) = sum_{b < BM}
// x(b) W_R^{bk}, evaluated directly for BM <= 2 (the first stage of a
// zero-padded transform), else the full transform.
template <int R, int BM, bool INV>
__device__ __forceinline__ void fft_reg_pruned(float2 (&x)[R]) {
  if constexpr (BM == 1) {
    static_for<1, R>([&](auto k) { x[k] = x[0]; });
  } else if constexpr (BM == 2 && R >= 2) {
    const float2 x0 = x[0], x1 = x[1];
    static_for<0, R>([&](auto k) { x[k] = cadd(x0, twmul32<decltype(k)::value * (32 / R), INV>(x1)); });
  } else {
    fft_reg<R, INV>(x);
  }
}

// ----------------------------------------------------------------------------
// FFT plans: N = R1 * R2 with R1 <= R2, R2 % R1 == 0
// ----------------------------------------------------------------------------
template <int N> struct Plan;
template <> struct Plan<4>   { static constexpr int R1 = 2,  R2 = 2;  };
template <> struct Plan<8>   { static constexpr int R1 = 2,  R2 = 4;  };
template <> struct Plan<16>  { static constexpr int R1 = 4,  R2 = 4;  };
template <> struct Plan<32>  { static constexpr int R1 = 4,  R2 = 8;  };
template <> struct Plan<64>  { static constexpr int R1 = 8,  R2 = 8;  };
template <> struct Plan<128> { static constexpr int R1 = 8,  R2 = 16; };
template <> struct Plan<256> { static constexpr int R1 = 16, R2 = 16; };
template <> struct Plan<512> { static constexpr int R1 = 16, R2 = 32; };

// Fill tw[k] = exp(-2 pi i k / N), k < N, cooperatively (caller syncs).
__device__ __forceinline__ void fill_twiddles(float2* tw, int N, int tid, int nthreads) {
  for (int k = tid; k < N; k += nthreads) {
    float s, c;
    sincospif(2.0f * (float)k / (float)N, &s, &c);
    tw[k] = make_float2(c, -s);
  }
}

template <bool INV>
__device__ __forceinline__ float2 twiddle(float2 v, const float2* tw, int idx) {
  const float2 w = tw[idx];
  return INV ? cmulc(v, w) : cmul(v, w);
}

// LDS exchange buffer layout: element (slot, j) of pencil p at (slot*J + j)*PW + p
// Engine A.  in: x[b] = x(a + R1 b), b < R2.  out: o[k*R1 + d] = X(c + R2 d),
// c = a + R1 k, k < R2/R1, d < R1.  tw: the length-N table.  Starts with a
// barrier (protects lds from earlier readers).
// BM < R2: x[b] is zero for b >= BM (a zero-padded input of at most BM * R1
// leading entries).
template <int N, int PW, bool INV, int BM = Plan<N>::R2>
__device__ __forceinline__ void engineA(float2 (&x)[Plan<N>::R2], float2 (&o)[Plan<N>::R2],
                                        float2* lds, const float2* tw, int p, int a) {
  constexpr int R1 = Plan<N>::R1, R2 = Plan<N>::R2;
  fft_reg_pruned<R2, (BM < R2 ? BM : R2), INV>(x);
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
#pragma unroll
    for (int d = 0; d < R1; ++d) o[k * R1 + d] = z[d];
  }
}

// Engine B.  in: o[k*R1 + d] = X(c + R2 d) (task layout).  out: y[g] = y(a + R1 g).
template <int N, int PW, bool INV>
__device__ __forceinline__ void engineB(float2 (&o)[Plan<N>::R2], float2 (&y)[Plan<N>::R2],
                                        float2* lds, const float2* tw, int p, int a) {
  constexpr int R1 = Plan<N>::R1, R2 = Plan<N>::R2;
  __syncthreads();
#pragma unroll
  for (int k = 0; k < R2 / R1; ++k) {
    const int c = a + R1 * k;
    float2 z[R1];
#pragma unroll
    for (int d = 0; d < R1; ++d) z[d] = o[k * R1 + d];
    fft_reg<R1, INV>(z);
#pragma unroll
    for (int e = 1; e < R1; ++e) z[e] = twiddle<INV>(z[e], tw, (c * e) & (N - 1));
#pragma unroll
    for (int e = 0; e < R1; ++e) lds[(e * R2 + c) * PW + p] = z[e];
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < R2; ++c) y[c] = lds[(a * R2 + c) * PW + p];
  fft_reg<R2, INV>(y);
}

// Workgroups of a launch are dealt to the 8 XCDs round-robin (block b runs on
// XCD b mod 8).  This maps block b to a tile index so that each XCD receives
// one contiguous range of tiles: neighbouring tiles that share cache lines
// then share one L2.  A bijection on [0, nb).
__device__ __forceinline__ int xcd_tile(int b, int nb) {
  const int q = nb >> 3, rem = nb & 7, x = b & 7, slot = b >> 3;
  return (x < rem ? x * (q + 1) : rem * (q + 1) + (x - rem) * q) + slot;
}

// number of packed components of S^n(R^4): C(n+3, 3)
__device__ __forceinline__ int num_components_dev(int n) { return (n + 1) * (n + 2) * (n + 3) / 6; }

// packed multi-index alpha of position k for order n (alpha1 from n down to
// 0, then alpha2, then alpha3; alpha4 is the remainder)
__device__ __forceinline__ void alpha_of_dev(int n, int k, int* al) {
  int idx = 0;
  for (int a1 = n; a1 >= 0; --a1)
    for (int a2 = n - a1; a2 >= 0; --a2)
      for (int a3 = n - a1 - a2; a3 >= 0; --a3) {
        if (idx == k) {
          al[0] = a1; al[1] = a2; al[2] = a3; al[3] = n - a1 - a2 - a3;
          return;
        }
        ++idx;
      }
}

}  // namespace ttm
