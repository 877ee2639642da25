// Rotation of a template box by a unit quaternion (device side), shared by the
// tensor build, classical matching and the NCC check of the pose recovery.
//
// R(Q) of Q = (a,b,c,d): the active Hamilton rotation v -> Q v Q*, vector part
// on axes (0,1,2).  The rotated template is t_R(u) = t(c + R^-1 (u - c)) with
// c = L / 2 per axis, sampled trilinearly with zero outside the box.
#pragma once

#include <hip/hip_runtime.h>

namespace ttm {

struct Rot {
  float r[9];   // row-major R
};

__device__ __forceinline__ Rot quat_rot(const float* q4) {
  double a = q4[0], b = q4[1], c = q4[2], d = q4[3];
  const double nrm = sqrt(a * a + b * b + c * c + d * d);
  a /= nrm; b /= nrm; c /= nrm; d /= nrm;
  Rot R;
  R.r[0] = (float)(a * a + b * b - c * c - d * d);
  R.r[1] = (float)(2.0 * (b * c - a * d));
  R.r[2] = (float)(2.0 * (b * d + a * c));
  R.r[3] = (float)(2.0 * (b * c + a * d));
  R.r[4] = (float)(a * a - b * b + c * c - d * d);
  R.r[5] = (float)(2.0 * (c * d - a * b));
  R.r[6] = (float)(2.0 * (b * d - a * c));
  R.r[7] = (float)(2.0 * (c * d + a * b));
  R.r[8] = (float)(a * a - b * b - c * c + d * d);
  return R;
}

// t(c + R^-1 (u - c)) with R^-1 = R^T, trilinear, zero outside [0, L)
__device__ __forceinline__ float sample_rotated(const float* __restrict__ t, int L0, int L1, int L2,
                                                const Rot& R, int u0, int u1, int u2) {
  const int c0 = L0 / 2, c1 = L1 / 2, c2 = L2 / 2;
  const float v0 = (float)(u0 - c0), v1 = (float)(u1 - c1), v2 = (float)(u2 - c2);
  const float p0 = c0 + R.r[0] * v0 + R.r[3] * v1 + R.r[6] * v2;
  const float p1 = c1 + R.r[1] * v0 + R.r[4] * v1 + R.r[7] * v2;
  const float p2 = c2 + R.r[2] * v0 + R.r[5] * v1 + R.r[8] * v2;
  const float f0 = floorf(p0), f1 = floorf(p1), f2 = floorf(p2);
  const int i0 = (int)f0, i1 = (int)f1, i2 = (int)f2;
  const float w0 = p0 - f0, w1 = p1 - f1, w2 = p2 - f2;
  float acc = 0.0f;
#pragma unroll
  for (int d0 = 0; d0 < 2; ++d0) {
    const int j0 = i0 + d0;
    if (j0 < 0 || j0 >= L0) continue;
    const float a0 = d0 ? w0 : 1.0f - w0;
#pragma unroll
    for (int d1 = 0; d1 < 2; ++d1) {
      const int j1 = i1 + d1;
      if (j1 < 0 || j1 >= L1) continue;
      const float a1 = a0 * (d1 ? w1 : 1.0f - w1);
#pragma unroll
      for (int d2 = 0; d2 < 2; ++d2) {
        const int j2 = i2 + d2;
        if (j2 < 0 || j2 >= L2) continue;
        acc += a1 * (d2 ? w2 : 1.0f - w2) * t[((long)j0 * L1 + j1) * L2 + j2];
      }
    }
  }
  return acc;
}

// The same sampling from a box held in LDS with padded pitches and a zero
// guard one past the box's upper edge on every axis: row pitch P2 = L2 + 3
// (columns L2..L2+2 zero), L1 + 1 rows per plane (row L1 zero) and plane
// pitch P01 = (L1 + 1) P2 + 5, L0 + 1 planes (plane L0 zero).  Every cell
// whose lower corner lies in the box then reads its eight corners without a
// test: the corners on the guard are zero, as outside the box.  Only points
// below the box or past its last cell take the branch-free general path,
// where corners outside the box get weight 0 and read element 0.  For
// L = 32 the banks see j2 + 35 j1 + 8 j0 mod 64.  The layout must fit
// kNccLdsCap floats (fill it with fill_lds_box).
constexpr int kNccLdsCap = 38400;
__host__ __device__ constexpr int ncc_lds_p2(int L2) { return L2 + 3; }
__host__ __device__ constexpr int ncc_lds_p01(int L1, int L2) { return (L1 + 1) * (L2 + 3) + 5; }
__host__ __device__ constexpr long ncc_lds_floats(int L0, int L1, int L2) {
  return (long)(L0 + 1) * ncc_lds_p01(L1, L2);
}
// the layout offset of cell (i0, i1, i2), every index non-negative and every
// product below 2^24 (the layout fits in LDS): 24-bit multiplies, which run
// at full rate where a 32-bit multiply takes four passes
__device__ __forceinline__ int lds_cell(int i0, int i1, int i2, int P2, int P01) {
  return (int)(__umul24((unsigned)i0, (unsigned)P01) + __umul24((unsigned)i1, (unsigned)P2)) + i2;
}

// the trilinear interpolation in the cell whose lower corner q points at
__device__ __forceinline__ float lerp_cell(const float* q, int P2, int P01, float w0, float w1, float w2) {
  const float c00 = q[0] + w2 * (q[1] - q[0]);
  const float c01 = q[P2] + w2 * (q[P2 + 1] - q[P2]);
  const float c10 = q[P01] + w2 * (q[P01 + 1] - q[P01]);
  const float c11 = q[P01 + P2] + w2 * (q[P01 + P2 + 1] - q[P01 + P2]);
  const float c0 = c00 + w1 * (c01 - c00), c1 = c10 + w1 * (c11 - c10);
  return c0 + w0 * (c1 - c0);
}

// The guarded sampler without its test, for a caller that has shown that
// every sample point lies in [0, L) on every axis (the sampled voxels within
// a ball about the centre that rotations keep inside the box): the same
// arithmetic as the test's fast path, so the same values.
__device__ __forceinline__ float sample_rotated_lds_inner(const float* t, int L0, int L1, int L2, int P2, int P01,
                                                          const Rot& R, int u0, int u1, int u2) {
  const int c0 = L0 / 2, c1 = L1 / 2, c2 = L2 / 2;
  const float v0 = (float)(u0 - c0), v1 = (float)(u1 - c1), v2 = (float)(u2 - c2);
  const float p0 = c0 + R.r[0] * v0 + R.r[3] * v1 + R.r[6] * v2;
  const float p1 = c1 + R.r[1] * v0 + R.r[4] * v1 + R.r[7] * v2;
  const float p2 = c2 + R.r[2] * v0 + R.r[5] * v1 + R.r[8] * v2;
  const float f0 = floorf(p0), f1 = floorf(p1), f2 = floorf(p2);
  const int i0 = (int)f0, i1 = (int)f1, i2 = (int)f2;
  return lerp_cell(t + lds_cell(i0, i1, i2, P2, P01), P2, P01, p0 - f0, p1 - f1, p2 - f2);
}

// GUARD = false keeps the test of a box without the guard (the fast path for
// cells whose upper corners are in the box too), so that its sums round as
// they did before the guard existed (the tensor build: its components are
// compared with tolerances that its float32 rounding nearly fills).
template <bool GUARD = true>
__device__ __forceinline__ float sample_rotated_lds(const float* t, int L0, int L1, int L2, int P2, int P01,
                                                    const Rot& R, int u0, int u1, int u2) {
  const int c0 = L0 / 2, c1 = L1 / 2, c2 = L2 / 2;
  const float v0 = (float)(u0 - c0), v1 = (float)(u1 - c1), v2 = (float)(u2 - c2);
  const float p0 = c0 + R.r[0] * v0 + R.r[3] * v1 + R.r[6] * v2;
  const float p1 = c1 + R.r[1] * v0 + R.r[4] * v1 + R.r[7] * v2;
  const float p2 = c2 + R.r[2] * v0 + R.r[5] * v1 + R.r[8] * v2;
  const float f0 = floorf(p0), f1 = floorf(p1), f2 = floorf(p2);
  const int i0 = (int)f0, i1 = (int)f1, i2 = (int)f2;
  const float w0 = p0 - f0, w1 = p1 - f1, w2 = p2 - f2;
  const int e = GUARD ? 0 : 1;
  if ((unsigned)i0 < (unsigned)(L0 - e) && (unsigned)i1 < (unsigned)(L1 - e) && (unsigned)i2 < (unsigned)(L2 - e)) {
    // the lower corner in the box (the common case): the upper corners are
    // in the box or on its zero guard
    return lerp_cell(t + lds_cell(i0, i1, i2, P2, P01), P2, P01, w0, w1, w2);
  }
  float a[2], b[2], c[2];
  int j0[2], j1[2], j2[2];
#pragma unroll
  for (int d = 0; d < 2; ++d) {
    const bool ok0 = (unsigned)(i0 + d) < (unsigned)L0, ok1 = (unsigned)(i1 + d) < (unsigned)L1,
               ok2 = (unsigned)(i2 + d) < (unsigned)L2;
    a[d] = ok0 ? (d ? w0 : 1.0f - w0) : 0.0f;
    b[d] = ok1 ? (d ? w1 : 1.0f - w1) : 0.0f;
    c[d] = ok2 ? (d ? w2 : 1.0f - w2) : 0.0f;
    j0[d] = ok0 ? (int)__umul24((unsigned)(i0 + d), (unsigned)P01) : 0;
    j1[d] = ok1 ? (int)__umul24((unsigned)(i1 + d), (unsigned)P2) : 0;
    j2[d] = ok2 ? i2 + d : 0;
  }
  float acc = 0.0f;
#pragma unroll
  for (int d0 = 0; d0 < 2; ++d0)
#pragma unroll
    for (int d1 = 0; d1 < 2; ++d1) {
      const float ab = a[d0] * b[d1];
      const int r = j0[d0] + j1[d1];
      acc += ab * (c[0] * t[r + j2[0]] + c[1] * t[r + j2[1]]);
    }
  return acc;
}


// Copies the L0 x L1 x L2 box src (C order) into the padded LDS layout above.
// Each of the block's nthreads threads keeps eight loads in flight before
// its stores, so the copy is not a chain of dependent load-store steps.  The
// caller synchronises before the box is read.
// the box into the padded layout of sample_rotated_lds, the guard rows,
// columns and plane zero: every float of the layout is written, eight loads
// in flight per thread.  A layout index e is split into plane, row and column
// by multiply-high with the reciprocals m = ceil(2^32 / d) of the pitches,
// exact here: e < 2^17 and d < 2^11, so e (m d - 2^32) < e d < 2^32.
__device__ __forceinline__ void fill_lds_box(float* tl, const float* __restrict__ src, int L0, int L1, int L2,
                                             int P2, int P01, int tid, int nthreads) {
  const int total = (L0 + 1) * P01;
  const unsigned m01 = (unsigned)((0x100000000ull + (unsigned)P01 - 1) / (unsigned)P01);
  const unsigned m2 = (unsigned)((0x100000000ull + (unsigned)P2 - 1) / (unsigned)P2);
  constexpr int U = 8;
  for (int e0 = tid; e0 < total; e0 += nthreads * U) {
    float v[U];
#pragma unroll
    for (int j = 0; j < U; ++j) {
      const unsigned e = (unsigned)(e0 + j * nthreads);
      const unsigned j0 = __umulhi(e, m01), rem = e - __umul24(j0, (unsigned)P01);
      const unsigned j1 = __umulhi(rem, m2), j2 = rem - __umul24(j1, (unsigned)P2);
      const bool in = (int)e < total && j0 < (unsigned)L0 && j1 < (unsigned)L1 && j2 < (unsigned)L2;
      // an unconditional load (of element 0 outside the box), so that the
      // group's loads issue before any wait
      const float x = src[in ? ((int)j0 * L1 + (int)j1) * L2 + (int)j2 : 0];
      v[j] = in ? x : 0.0f;
    }
#pragma unroll
    for (int j = 0; j < U; ++j) {
      const int e = e0 + j * nthreads;
      if (e < total) tl[e] = v[j];
    }
  }
}

}  // namespace ttm
