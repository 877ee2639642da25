// Candidate positions and rotations (Sections 3.3, 3.4).
//
// Peaks: valid-region voxels with F > threshold that are strictly above all
// 26 neighbours, ordered by (F descending, linear index ascending), greedily
// suppressed within min_dist of accepted peaks.  Candidates are bounded by a
// histogram of the float bit patterns of F (F >= 0, so the order of the bit
// patterns is the order of the values): the top candidates, at most
// kCandCap, are compacted, sorted with a bitonic network in LDS, and
// suppressed by one wavefront.
//
// Pose: at each peak C_n(x) is recomputed directly (float64) from the image
// window and the components, then the dominant Z-eigenpair max C Q^n, |Q| = 1
// (eq. "Zeigen"; Theorem "main") is found from a scan of S^3 seed points and
// a shifted power iteration (SS-HOPM) accelerated by safeguarded Newton steps
// on the sphere, from the 4 best mutually distant seeds.
#include "ttm_device.h"
#include "ttm_internal.h"

namespace ttm {

struct PeakGeo {
  int n0, n1, n2;
  int lo0, hi0, lo1, hi1, lo2, hi2;
};

__device__ __forceinline__ bool strict_local_max(const float* __restrict__ F, const PeakGeo& g, int x0,
                                                 int x1, int x2, float v) {
  for (int d0 = -1; d0 <= 1; ++d0) {
    const int y0 = x0 + d0;
    if (y0 < 0 || y0 >= g.n0) continue;
    for (int d1 = -1; d1 <= 1; ++d1) {
      const int y1 = x1 + d1;
      if (y1 < 0 || y1 >= g.n1) continue;
      const float* row = F + ((long)y0 * g.n1 + y1) * g.n2;
      for (int d2 = -1; d2 <= 1; ++d2) {
        const int y2 = x2 + d2;
        if (y2 < 0 || y2 >= g.n2) continue;
        if (d0 == 0 && d1 == 0 && d2 == 0) continue;
        if (!(v > row[y2])) return false;
      }
    }
  }
  return true;
}

// pass 0: histogram of candidate keys; pass 1: compaction of keys >= ctrl[1]
template <int PASS>
__global__ void __launch_bounds__(256) k_peaks_scan(const float* __restrict__ F, PeakGeo g, float threshold,
                                                    unsigned* __restrict__ hist, unsigned* __restrict__ ctrl,
                                                    unsigned long long* __restrict__ cand) {
  const int e0 = g.hi0 - g.lo0 + 1, e1 = g.hi1 - g.lo1 + 1, e2 = g.hi2 - g.lo2 + 1;
  const long nvalid = (long)e0 * e1 * e2;
  const unsigned kmin = PASS == 1 ? ctrl[1] : 0u;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < nvalid; i += (long)gridDim.x * blockDim.x) {
    const int x2 = g.lo2 + (int)(i % e2);
    const long r = i / e2;
    const int x1 = g.lo1 + (int)(r % e1);
    const int x0 = g.lo0 + (int)(r / e1);
    const long lin = ((long)x0 * g.n1 + x1) * g.n2 + x2;
    const float v = F[lin];
    if (!(v > threshold)) continue;
    if (!strict_local_max(F, g, x0, x1, x2, v)) continue;
    const unsigned key = __float_as_uint(v) >> 16;
    if (PASS == 0) {
      atomicAdd(&hist[key], 1u);
    } else if (key >= kmin) {
      const unsigned slot = atomicAdd(&ctrl[0], 1u);
      if (slot < (unsigned)kCandCap)
        cand[slot] = ((unsigned long long)(0xFFFFFFFFu - __float_as_uint(v)) << 32) | (unsigned long long)lin;
    }
  }
}

// smallest key b with sum_{k >= b} hist[k] <= kCandCap
__global__ void __launch_bounds__(1024) k_peaks_select(const unsigned* __restrict__ hist,
                                                       unsigned* __restrict__ ctrl) {
  __shared__ unsigned part[1024];
  constexpr int per = kHistBins / 1024;
  const int tid = threadIdx.x;
  unsigned s = 0;
  for (int i = 0; i < per; ++i) s += hist[tid * per + i];
  part[tid] = s;
  __syncthreads();
  // inclusive suffix sums over threads (Hillis-Steele)
  for (int off = 1; off < 1024; off <<= 1) {
    const unsigned v = (tid + off < 1024) ? part[tid + off] : 0u;
    __syncthreads();
    part[tid] += v;
    __syncthreads();
  }
  // part[tid] = sum of bins from tid*per to the end
  const unsigned above = (tid + 1 < 1024) ? part[tid + 1] : 0u;   // bins after this chunk
  if (part[tid] > (unsigned)kCandCap && above <= (unsigned)kCandCap) {
    unsigned run = above;
    int b = tid * per + per;
    for (int i = per - 1; i >= 0; --i) {
      const unsigned h = hist[tid * per + i];
      if (run + h > (unsigned)kCandCap) break;
      run += h;
      b = tid * per + i;
    }
    ctrl[1] = (unsigned)b;
    ctrl[2] = 1u;   // the total exceeds the capacity: candidates below b exist
  }
  if (tid == 0 && part[0] <= (unsigned)kCandCap) {
    ctrl[1] = 0u;
    ctrl[2] = 0u;
  }
}

__device__ __forceinline__ void decode_lin(unsigned long long key, int n1, int n2, int& x0, int& x1, int& x2) {
  const long lin = (long)(key & 0xFFFFFFFFull);
  x2 = (int)(lin % n2);
  const long r = lin / n2;
  x1 = (int)(r % n1);
  x0 = (int)(r / n1);
}

// one block: bitonic sort of the candidate keys (ascending key = F descending,
// then linear index ascending), written back in place
__global__ void __launch_bounds__(1024) k_peaks_sort(const unsigned* __restrict__ ctrl,
                                                     unsigned long long* __restrict__ cand) {
  __shared__ unsigned long long keys[kCandCap];
  const int tid = threadIdx.x;
  const unsigned nc = min(ctrl[0], (unsigned)kCandCap);
  int np2 = 1;
  while (np2 < (int)nc) np2 <<= 1;
  for (int i = tid; i < np2; i += 1024) keys[i] = (i < (int)nc) ? cand[i] : ~0ull;
  __syncthreads();
  for (int k = 2; k <= np2; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = tid; i < np2; i += 1024) {
        const int ixj = i ^ j;
        if (ixj > i) {
          const unsigned long long a = keys[i], b = keys[ixj];
          const bool up = (i & k) == 0;
          if ((a > b) == up) {
            keys[i] = b;
            keys[ixj] = a;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int i = tid; i < (int)nc; i += 1024) cand[i] = keys[i];
}

// one wavefront: greedy suppression over the sorted candidates, 64 at a time.
// Each lane tests its candidate against the accepted list; conflicts inside
// the chunk are resolved in candidate order with lane broadcasts.
__global__ void __launch_bounds__(64) k_peaks_nms(PeakGeo g, const unsigned* __restrict__ ctrl,
                                                  const unsigned long long* __restrict__ cand,
                                                  float min_dist, int max_peaks, int* __restrict__ out_pos,
                                                  float* __restrict__ out_score, int* __restrict__ out_count) {
  __shared__ int acc_pos[3 * 4096];
  const int lane = threadIdx.x;
  const unsigned nc = min(ctrl[0], (unsigned)kCandCap);
  const float d2min = min_dist * min_dist;
  int nacc = 0;
  bool exhausted = true;
  for (int base = 0; base < (int)nc; base += 64) {
    if (nacc >= max_peaks) {
      exhausted = false;
      break;
    }
    const int i = base + lane;
    const bool have = i < (int)nc;
    unsigned long long key = have ? cand[i] : ~0ull;
    int x0 = 0, x1 = 0, x2 = 0;
    if (have) decode_lin(key, g.n1, g.n2, x0, x1, x2);
    bool sup = !have;
    for (int q = 0; q < nacc && !sup; ++q) {
      const float d0 = (float)(x0 - acc_pos[3 * q]), d1 = (float)(x1 - acc_pos[3 * q + 1]),
                  d2 = (float)(x2 - acc_pos[3 * q + 2]);
      if (d0 * d0 + d1 * d1 + d2 * d2 < d2min) sup = true;
    }
    unsigned long long conf = 0ull;
    for (int m2 = 0; m2 < 64; ++m2) {
      const int y0 = __shfl(x0, m2), y1 = __shfl(x1, m2), y2 = __shfl(x2, m2);
      if (m2 < lane) {
        const float d0 = (float)(x0 - y0), d1 = (float)(x1 - y1), d2 = (float)(x2 - y2);
        if (d0 * d0 + d1 * d1 + d2 * d2 < d2min) conf |= (1ull << m2);
      }
    }
    unsigned long long accepted = 0ull;
    const int nacc0 = nacc;
    for (int m2 = 0; m2 < 64; ++m2) {
      const int s_m = __shfl((int)sup, m2);
      const unsigned long long c_m = __shfl(conf, m2);
      if (nacc < max_peaks && !s_m && (c_m & accepted) == 0ull) {
        accepted |= (1ull << m2);
        ++nacc;
      }
    }
    // lane m writes its own accepted entry at its rank among the accepted lanes
    if ((accepted >> lane) & 1ull) {
      const int rank = nacc0 + __popcll(accepted & ((1ull << lane) - 1ull));
      acc_pos[3 * rank] = x0;
      acc_pos[3 * rank + 1] = x1;
      acc_pos[3 * rank + 2] = x2;
      out_pos[3 * rank] = x0;
      out_pos[3 * rank + 1] = x1;
      out_pos[3 * rank + 2] = x2;
      out_score[rank] = __uint_as_float(0xFFFFFFFFu - (unsigned)(key >> 32));
    }
    __syncthreads();
  }
  if (lane == 0) {
    out_count[0] = nacc;
    const bool more_below = ctrl[2] != 0u;
    out_count[1] = ((nacc < max_peaks && exhausted && more_below) || ctrl[0] > (unsigned)kCandCap)
                       ? TTM_PEAKS_TRUNCATED : 0;
  }
}

hipError_t launch_peaks(const Geo& gg, const float* score, float threshold, float min_dist,
                        int max_peaks, const PeakWs& w, int* out_pos, float* out_score,
                        int* out_count, hipStream_t s) {
  PeakGeo g;
  g.n0 = gg.n0; g.n1 = gg.n1; g.n2 = gg.n2;
  g.lo0 = gg.c0; g.hi0 = gg.n0 - gg.L0 + gg.c0;
  g.lo1 = gg.c1; g.hi1 = gg.n1 - gg.L1 + gg.c1;
  g.lo2 = gg.c2; g.hi2 = gg.n2 - gg.L2 + gg.c2;
  hipError_t e;
  if ((e = launch_fill_i32(reinterpret_cast<int*>(w.hist), kHistBins, 0, s)) != hipSuccess) return e;
  if ((e = launch_fill_i32(reinterpret_cast<int*>(w.ctrl), 4, 0, s)) != hipSuccess) return e;
  hipLaunchKernelGGL((k_peaks_scan<0>), dim3(2048), dim3(256), 0, s, score, g, threshold, w.hist, w.ctrl, w.cand);
  hipLaunchKernelGGL(k_peaks_select, dim3(1), dim3(1024), 0, s, w.hist, w.ctrl);
  hipLaunchKernelGGL((k_peaks_scan<1>), dim3(2048), dim3(256), 0, s, score, g, threshold, w.hist, w.ctrl, w.cand);
  hipLaunchKernelGGL(k_peaks_sort, dim3(1), dim3(1024), 0, s, w.ctrl, w.cand);
  hipLaunchKernelGGL(k_peaks_nms, dim3(1), dim3(64), 0, s, g, w.ctrl, w.cand, min_dist, max_peaks,
                     out_pos, out_score, out_count);
  return hipGetLastError();
}

// ----------------------------------------------------------------------------
// pose
// ----------------------------------------------------------------------------
struct PoseGeo {
  int n0, n1, n2, L0, L1, L2;
};

__device__ __forceinline__ double block_sum(double v, double* sh) {
  const int tid = threadIdx.x;
  __syncthreads();
  sh[tid] = v;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) sh[tid] += sh[tid + s];
    __syncthreads();
  }
  return sh[0];
}

// wavefront sum (64 lanes); the butterfly leaves each lane with a sum in a
// different association order, so lane 0's value is broadcast to keep every
// lane's control flow identical
__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return __shfl(v, 0);
}

constexpr int kPoseChunk = 8;
constexpr int kMaxTerms = kMaxK;

// Evaluate phi(Q) = sum_alpha mu_alpha A_alpha Q^alpha (A pre-multiplied by mu)
__device__ __forceinline__ double phi_eval(const double* muA, const int* al, int K, int n, const double* q) {
  double pw[4][kMaxOrder + 1];
  for (int d = 0; d < 4; ++d) {
    pw[d][0] = 1.0;
    for (int e = 1; e <= n; ++e) pw[d][e] = pw[d][e - 1] * q[d];
  }
  double s = 0.0;
  for (int k = 0; k < K; ++k) s += muA[k] * pw[0][al[4 * k]] * pw[1][al[4 * k + 1]] * pw[2][al[4 * k + 2]] * pw[3][al[4 * k + 3]];
  return s;
}

__device__ __forceinline__ void seed_point(int i, int n, double* q) {
  const double phi = 1.4142135623730950488;      // sqrt(2)
  const double psi = 1.533751168755204288118041; // real root of psi^4 = psi + 4
  const double s = i + 0.5;
  const double r = sqrt(s / n), R = sqrt(1.0 - s / n);
  const double al = 6.283185307179586477 * s / phi, be = 6.283185307179586477 * s / psi;
  q[0] = r * sin(al);
  q[1] = r * cos(al);
  q[2] = R * sin(be);
  q[3] = R * cos(be);
}

// Solve the 4x4 system H xi = rhs by Gaussian elimination with partial pivoting.
__device__ __forceinline__ bool solve4(double H[4][4], double* rhs) {
  for (int c = 0; c < 4; ++c) {
    int piv = c;
    for (int r = c + 1; r < 4; ++r)
      if (fabs(H[r][c]) > fabs(H[piv][c])) piv = r;
    if (fabs(H[piv][c]) < 1e-300) return false;
    if (piv != c) {
      for (int k = 0; k < 4; ++k) {
        const double t = H[c][k];
        H[c][k] = H[piv][k];
        H[piv][k] = t;
      }
      const double t = rhs[c];
      rhs[c] = rhs[piv];
      rhs[piv] = t;
    }
    for (int r = c + 1; r < 4; ++r) {
      const double f = H[r][c] / H[c][c];
      for (int k = c; k < 4; ++k) H[r][k] -= f * H[c][k];
      rhs[r] -= f * rhs[c];
    }
  }
  for (int c = 3; c >= 0; --c) {
    double s = rhs[c];
    for (int k = c + 1; k < 4; ++k) s -= H[c][k] * rhs[k];
    rhs[c] = s / H[c][c];
  }
  return true;
}

// lambda, gradient term A x^{n-1} and matrix A x^{n-2} (times n(n-1) later),
// accumulated across the wavefront: each lane owns components k = lane + 64 i.
__device__ __forceinline__ void tensor_terms(const double* muA, const int* al, int K, int n, const double* x,
                                             int lane, double& lam, double* g, double* Hm) {
  double pw[4][kMaxOrder + 1];
  for (int d = 0; d < 4; ++d) {
    pw[d][0] = 1.0;
    for (int e = 1; e <= n; ++e) pw[d][e] = pw[d][e - 1] * x[d];
  }
  double l = 0.0, gg[4] = {0, 0, 0, 0}, hh[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int k = lane; k < K; k += 64) {
    const int e[4] = {al[4 * k], al[4 * k + 1], al[4 * k + 2], al[4 * k + 3]};
    const double c = muA[k];
    l += c * pw[0][e[0]] * pw[1][e[1]] * pw[2][e[2]] * pw[3][e[3]];
    for (int i = 0; i < 4; ++i) {
      if (e[i] == 0) continue;
      double t = c * e[i];
      for (int d = 0; d < 4; ++d) t *= pw[d][d == i ? e[d] - 1 : e[d]];
      gg[i] += t;
    }
    int h = 0;
    for (int i = 0; i < 4; ++i)
      for (int j = i; j < 4; ++j, ++h) {
        const int ci = e[i] * (e[j] - (i == j ? 1 : 0));
        if (ci == 0) continue;
        double t = c * ci;
        for (int d = 0; d < 4; ++d) {
          int ex = e[d] - (d == i ? 1 : 0) - (d == j ? 1 : 0);
          t *= pw[d][ex];
        }
        hh[h] += t;
      }
  }
  lam = wave_sum(l);
  for (int i = 0; i < 4; ++i) g[i] = wave_sum(gg[i]) / n;                 // A x^{n-1}
  for (int h = 0; h < 10; ++h) Hm[h] = wave_sum(hh[h]) / (n * (n - 1));   // A x^{n-2}
}

__global__ void __launch_bounds__(256) k_pose(PoseGeo g, const float* __restrict__ image,
                                              const float* __restrict__ comps, const float* __restrict__ mask,
                                              int order_n, const double* __restrict__ img_stats, float eps_v,
                                              int n_seeds, int max_iter, double tol, const int* __restrict__ pos,
                                              const int* __restrict__ count, float* __restrict__ out_quat,
                                              double* __restrict__ out_lambda, int* __restrict__ out_flags,
                                              double* __restrict__ out_C) {
  __shared__ double sh[256];
  __shared__ double muA[kMaxTerms];
  __shared__ int al[4 * kMaxTerms];
  __shared__ double sel[4][4];
  __shared__ double wres[4][6];    // per wave: lambda, q0..q3, flags
  __shared__ int shi[256];
  const int peak = blockIdx.x;
  if (peak >= count[0]) return;
  const int tid = threadIdx.x;
  const int n = order_n;
  const int K = num_components_dev(n);
  const int L0 = g.L0, L1 = g.L1, L2 = g.L2, nL = L0 * L1 * L2;
  const int x0 = pos[3 * peak], x1 = pos[3 * peak + 1], x2 = pos[3 * peak + 2];
  const int c0 = L0 / 2, c1 = L1 / 2, c2 = L2 / 2;
  auto img_at = [&](int u) -> double {
    const int u2 = u % L2, u1 = (u / L2) % L1, u0 = u / (L1 * L2);
    int y0 = x0 + u0 - c0, y1 = x1 + u1 - c1, y2 = x2 + u2 - c2;
    y0 = ((y0 % g.n0) + g.n0) % g.n0;
    y1 = ((y1 % g.n1) + g.n1) % g.n1;
    y2 = ((y2 % g.n2) + g.n2) % g.n2;
    return (double)image[((long)y0 * g.n1 + y1) * g.n2 + y2];
  };
  // two-pass masked mean and variance of the window
  double s0 = 0.0, s1 = 0.0;
  for (int u = tid; u < nL; u += 256) {
    const double mv = mask[u];
    if (mv != 0.0) {
      s0 += mv;
      s1 += mv * img_at(u);
    }
  }
  const double msum = block_sum(s0, sh);
  const double mean = block_sum(s1, sh) / msum;
  double s2 = 0.0;
  for (int u = tid; u < nL; u += 256) {
    const double mv = mask[u];
    if (mv != 0.0) {
      const double d = img_at(u) - mean;
      s2 += mv * d * d;
    }
  }
  const double var = block_sum(s2, sh);
  const double floor_v = (double)eps_v * msum * img_stats[1];
  const double w = var > floor_v ? 1.0 / sqrt(var) : 0.0;

  // packed exponents and multiplicities
  if (tid < K) {
    int e[4];
    alpha_of_dev(n, tid, e);
    for (int d = 0; d < 4; ++d) al[4 * tid + d] = e[d];
  }
  __syncthreads();

  // C_alpha = w <tau_x f, T_alpha>, in chunks of kPoseChunk components
  for (int k0 = 0; k0 < K; k0 += kPoseChunk) {
    double acc[kPoseChunk];
    for (int i = 0; i < kPoseChunk; ++i) acc[i] = 0.0;
    for (int u = tid; u < nL; u += 256) {
      const double v = img_at(u);
      for (int i = 0; i < kPoseChunk; ++i)
        if (k0 + i < K) acc[i] += v * (double)comps[(long)(k0 + i) * nL + u];
    }
    for (int i = 0; i < kPoseChunk; ++i) {
      if (k0 + i >= K) break;
      const double c = block_sum(acc[i], sh) * w;
      if (tid == 0) {
        if (out_C) out_C[(long)peak * K + k0 + i] = c;
        const int* e = &al[4 * (k0 + i)];
        double mu = 1.0;
        for (int j = 2; j <= n; ++j) mu *= j;
        for (int d = 0; d < 4; ++d)
          for (int j = 2; j <= e[d]; ++j) mu /= j;
        muA[k0 + i] = mu * c;
      }
    }
  }
  __syncthreads();

  // seed scan: 4 rounds of block argmax, each excluding seeds within 10 degrees
  // (|<q, s>| > cos 5 deg) of the seeds already selected
  const double cosx = 0.99619469809174553;   // cos(5 deg)
  for (int r = 0; r < 4; ++r) {
    double best = -INFINITY;
    int bi = -1;
    for (int i = tid; i < n_seeds; i += 256) {
      double q[4];
      seed_point(i, n_seeds, q);
      bool skip = false;
      for (int t = 0; t < r; ++t) {
        const double dp = q[0] * sel[t][0] + q[1] * sel[t][1] + q[2] * sel[t][2] + q[3] * sel[t][3];
        if (fabs(dp) > cosx) skip = true;
      }
      if (skip) continue;
      const double v = phi_eval(muA, al, K, n, q);
      if (v > best) {
        best = v;
        bi = i;
      }
    }
    // block argmax (value, then lower index)
    __syncthreads();
    sh[tid] = best;
    shi[tid] = bi;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if (tid < s) {
        const double a = sh[tid], b = sh[tid + s];
        const int ia = shi[tid], ib = shi[tid + s];
        if (b > a || (b == a && ib >= 0 && (ia < 0 || ib < ia))) {
          sh[tid] = b;
          shi[tid] = ib;
        }
      }
      __syncthreads();
    }
    if (tid == 0) {
      double q[4] = {1.0, 0.0, 0.0, 0.0};
      if (shi[0] >= 0) seed_point(shi[0], n_seeds, q);
      for (int d = 0; d < 4; ++d) sel[r][d] = q[d];
    }
    __syncthreads();
  }

  // per wave: polish from sel[wave]
  const int wave = tid / 64, lane = tid % 64;
  double x[4] = {sel[wave][0], sel[wave][1], sel[wave][2], sel[wave][3]};
  double lam, gv[4], Hm[10];
  tensor_terms(muA, al, K, n, x, lane, lam, gv, Hm);
  int it = 0;
  bool conv = false;
  for (it = 1; it <= max_iter; ++it) {
    // Newton step on the sphere: (P M P - n lam P + x x^T) xi = -n (A x^{n-1} - lam x)
    double M[4][4];
    {
      int h = 0;
      for (int i = 0; i < 4; ++i)
        for (int j = i; j < 4; ++j, ++h) {
          M[i][j] = n * (n - 1) * Hm[h];
          M[j][i] = M[i][j];
        }
    }
    double grad[4];
    for (int i = 0; i < 4; ++i) grad[i] = n * (gv[i] - lam * x[i]);
    double PMP[4][4], Mx[4];
    double xMx = 0.0;
    for (int i = 0; i < 4; ++i) {
      Mx[i] = 0.0;
      for (int j = 0; j < 4; ++j) Mx[i] += M[i][j] * x[j];
      xMx += x[i] * Mx[i];
    }
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j)
        PMP[i][j] = M[i][j] - x[i] * Mx[j] - Mx[i] * x[j] + x[i] * x[j] * xMx
                    - n * lam * ((i == j ? 1.0 : 0.0) - x[i] * x[j]) + x[i] * x[j];
    double xi[4] = {-grad[0], -grad[1], -grad[2], -grad[3]};
    double y[4];
    bool newton_ok = solve4(PMP, xi);
    double ny = 0.0;
    if (newton_ok) {
      for (int i = 0; i < 4; ++i) { y[i] = x[i] + xi[i]; ny += y[i] * y[i]; }
      newton_ok = ny > 0.0;
    }
    double lam_new = -INFINITY, gv2[4], Hm2[10];
    if (newton_ok) {
      ny = sqrt(ny);
      for (int i = 0; i < 4; ++i) y[i] /= ny;
      tensor_terms(muA, al, K, n, y, lane, lam_new, gv2, Hm2);
    }
    if (!(lam_new >= lam)) {
      // shifted power step: y = A x^{n-1} + alpha x, alpha keeping the shifted
      // objective locally convex (Gershgorin bound on lambda_min(A x^{n-2}))
      double gmin = INFINITY;
      double Hf[4][4];
      int h = 0;
      for (int i = 0; i < 4; ++i)
        for (int j = i; j < 4; ++j, ++h) { Hf[i][j] = Hm[h]; Hf[j][i] = Hm[h]; }
      for (int i = 0; i < 4; ++i) {
        double r = Hf[i][i];
        for (int j = 0; j < 4; ++j)
          if (j != i) r -= fabs(Hf[i][j]);
        gmin = fmin(gmin, r);
      }
      const double alpha = fmax(0.0, 1e-6 - (n - 1) * gmin);
      ny = 0.0;
      for (int i = 0; i < 4; ++i) { y[i] = gv[i] + alpha * x[i]; ny += y[i] * y[i]; }
      ny = sqrt(ny);
      for (int i = 0; i < 4; ++i) y[i] /= ny;
      tensor_terms(muA, al, K, n, y, lane, lam_new, gv2, Hm2);
    }
    const double dl = fabs(lam_new - lam);
    double gnorm = 0.0;
    for (int i = 0; i < 4; ++i) gnorm += grad[i] * grad[i];
    for (int i = 0; i < 4; ++i) x[i] = y[i];
    for (int i = 0; i < 4; ++i) gv[i] = gv2[i];
    for (int hh = 0; hh < 10; ++hh) Hm[hh] = Hm2[hh];
    const double lam_prev = lam;
    lam = lam_new;
    if (dl <= tol * fmax(1.0, fabs(lam)) && sqrt(gnorm) <= 1e-6 * fmax(1.0, fabs(lam_prev))) {
      conv = true;
      break;
    }
  }
  if (lane == 0) {
    wres[wave][0] = lam;
    for (int d = 0; d < 4; ++d) wres[wave][1 + d] = x[d];
    wres[wave][5] = conv ? 0.0 : 1.0;
  }
  __syncthreads();
  if (tid == 0) {
    int b = 0;
    for (int wv = 1; wv < 4; ++wv)
      if (wres[wv][0] > wres[b][0]) b = wv;
    double q[4] = {wres[b][1], wres[b][2], wres[b][3], wres[b][4]};
    const double nq = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    double sgn = 1.0;
    for (int d = 0; d < 4; ++d) {
      if (q[d] != 0.0) {
        sgn = q[d] > 0.0 ? 1.0 : -1.0;
        break;
      }
    }
    for (int d = 0; d < 4; ++d) out_quat[4 * peak + d] = (float)(sgn * q[d] / nq);
    out_lambda[peak] = wres[b][0];
    int flags = 0;
    if (wres[b][5] != 0.0) flags |= TTM_POSE_NOT_CONVERGED;
    if (w == 0.0) flags |= TTM_POSE_ZERO_NORM;
    out_flags[peak] = flags;
  }
}

hipError_t launch_pose(const Geo& gg, const float* image, const float* comps, const float* mask,
                       int order_n, const double* img_stats, float eps_v, int n_seeds, int max_iter,
                       double tol, int max_peaks, const int* pos, const int* count, float* out_quat,
                       double* out_lambda, int* out_flags, double* out_C, double* /*Cbuf*/,
                       hipStream_t s) {
  PoseGeo g;
  g.n0 = gg.n0; g.n1 = gg.n1; g.n2 = gg.n2;
  g.L0 = gg.L0; g.L1 = gg.L1; g.L2 = gg.L2;
  hipLaunchKernelGGL(k_pose, dim3(max_peaks), dim3(256), 0, s, g, image, comps, mask, order_n, img_stats,
                     eps_v, n_seeds, max_iter, tol, pos, count, out_quat, out_lambda, out_flags, out_C);
  return hipGetLastError();
}

}  // namespace ttm
