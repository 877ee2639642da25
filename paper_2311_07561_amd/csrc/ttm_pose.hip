// Candidate positions and rotations (Sections 3.3, 3.4).
//
// Peaks: valid-region voxels with F > threshold that are strictly above all
// 26 neighbours, ordered by (F descending, linear index ascending), greedily
// suppressed within min_dist of accepted peaks.  The scan appends each
// block's maxima to one of kPeakSubs sub-lists (block b to sub-list b mod
// kPeakSubs, so no counter is shared by the whole grid); candidates are
// bounded by a histogram of the float bit patterns of F (F >= 0, so the
// order of the bit patterns is the order of the values): the top candidates,
// at most kCandCap, are compacted, sorted with a bitonic network in LDS, and
// suppressed by one wavefront.
//
// Pose: at each peak C_n(x) is recomputed directly (float64) from the image
// window and the components, then the dominant Z-eigenpair max C Q^n, |Q| = 1
// (eq. "Zeigen"; Theorem "main") is found from a scan of S^3 seed points and
// a shifted power iteration (SS-HOPM) accelerated by safeguarded Newton steps
// on the sphere, from the 4 best mutually distant seeds.
#include <algorithm>

#include "ttm_device.h"
#include "ttm_eig.h"
#include "ttm_internal.h"
#include "ttm_rotate.h"

namespace ttm {

struct PeakGeo {
  int n0, n1, n2;
  int lo0, hi0, lo1, hi1, lo2, hi2;
};

// candidates sorted in the first round (the second takes kCandCap)
constexpr unsigned kCandCap1 = 2048;

// control words of the peak search
enum PeakCtrl { PK_B1 = 1, PK_MORE1 = 2, PK_CNT1 = 3, PK_B2 = 4, PK_MORE2 = 5, PK_CNT2 = 6, PK_REDO = 7 };

__device__ __forceinline__ unsigned long long peak_key(float v, long lin) {
  // ascending key order = F descending, then linear index ascending
  return ((unsigned long long)(0xFFFFFFFFu - __float_as_uint(v)) << 32) | (unsigned long long)lin;
}

// One pass over the valid region in blocks of 8 rows x 32 columns and runs
// of up to 16 planes along axis 0, staged with a one-voxel halo in LDS:
// every strict local maximum above the threshold is appended to the full
// candidate list.  Each thread walks its column (x1, x2) through the run and
// reduces every plane it reads to the maximum of its 3 x 3 window with and
// without the centre, so a plane's window is read once and serves the test
// of its own voxel and of the voxels above and below: v is a strict maximum
// when it exceeds the window maximum without the centre in its own plane
// and the window maxima of both neighbouring planes.  The maxima propagate
// NaN, so a NaN anywhere among the 26 neighbours rejects v, as a comparison
// with each of them would.  Out-of-image neighbours hold -inf.  Maps of
// depth 1 (the planes of a stack) take runs of one plane (RUN = 1), so that
// their blocks reserve the LDS of three planes, not eighteen.
constexpr int QS1 = 8, QS2 = 32, QRUN = 16;
constexpr int QH1 = QS1 + 2, QH2 = QS2 + 2;

// The scan's output per map: block b appends its maxima (at most KEYS:
// strict maxima are never neighbours, so there is at most one per 2x2x2
// cell, or per 2x2 cell of a single plane) to sub-list b mod kPeakSubs of
// allc, which holds cap_sub keys (its blocks' KEYS each), counted by control
// word 16 + b mod kPeakSubs.
constexpr int kPeakSubCtl = 16;
__host__ __device__ constexpr int peak_region_keys(int run) { return run == 1 ? QS1 * QS2 / 4 : run * QS1 * QS2 / 8; }
// every key of the sub-lists, shared by the nwaves wavefronts of the grid
// (this one is number `wave`): with nwaves a multiple of kPeakSubs, the
// wavefronts of one sub-list take its keys in turns of 64; with fewer, each
// takes whole sub-lists
template <class Fn>
__device__ __forceinline__ void for_each_key(const unsigned long long* __restrict__ allc, long cap_sub,
                                             const unsigned* __restrict__ ctrl, int wave, int nwaves, Fn&& fn) {
  const int lane = threadIdx.x & 63;
  if (nwaves >= kPeakSubs) {
    const int nparts = nwaves / kPeakSubs;
    const int sub = wave % kPeakSubs, part = wave / kPeakSubs;
    if (part >= nparts) return;
    const int n = __builtin_amdgcn_readfirstlane((int)ctrl[kPeakSubCtl + sub]);
    const unsigned long long* list = allc + sub * cap_sub;
    for (int i = part * 64 + lane; i < n; i += nparts * 64) fn(list[i]);
  } else {
    for (int sub = wave; sub < kPeakSubs; sub += nwaves) {
      const int n = __builtin_amdgcn_readfirstlane((int)ctrl[kPeakSubCtl + sub]);
      const unsigned long long* list = allc + sub * cap_sub;
      for (int i = lane; i < n; i += 64) fn(list[i]);
    }
  }
}

// max(a, b), NaN when either is NaN
__device__ __forceinline__ float max_nan(float a, float b) { return (a >= b || a != a) ? a : b; }

template <int RUN>
__global__ void __launch_bounds__(256) k_peaks_scan(const float* __restrict__ F, PeakGeo g, float threshold,
                                                    unsigned* __restrict__ ctrl,
                                                    unsigned long long* __restrict__ allc, long bigcap,
                                                    long cap_sub, int ztiles, long fplane) {
  static_assert(QS1 * QS2 == 256, "one column per thread");
  constexpr int QH0 = RUN + 2;
  constexpr int KEYS = peak_region_keys(RUN);
  __shared__ float tile[QH0 * QH1 * QH2];
  __shared__ unsigned long long lkeys[KEYS];
  __shared__ unsigned lcount, lbase;
  const int tid = threadIdx.x;
  // several maps (planes of a stack) at once: blockIdx.z = plane * ztiles + run
  const int plane = blockIdx.z / ztiles, bz = blockIdx.z % ztiles;
  F += plane * fplane;
  ctrl += kPeakCtrlWords * plane;
  allc += bigcap * plane;
  const int sub = ((bz * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x) % kPeakSubs;
  const int b0 = g.lo0 + bz * RUN, b1 = g.lo1 + blockIdx.y * QS1, b2 = g.lo2 + blockIdx.x * QS2;
  // the run's planes that hold valid voxels and their two halo planes
  const int nv0 = min(RUN, g.hi0 - b0 + 1);
  const int NT = (nv0 + 2) * QH1 * QH2;
  // all of a thread's loads in flight at once: each load is unconditional (of
  // voxel 0 outside the map) so that the compiler issues them before it waits
  constexpr int U = (QH0 * QH1 * QH2 + 255) / 256;
  for (int e0 = tid; e0 < NT; e0 += 256 * U) {
    float v[U];
    bool in[U];
#pragma unroll
    for (int j = 0; j < U; ++j) {
      const int e = e0 + 256 * j;
      const int t2 = e % QH2, t1 = (e / QH2) % QH1, t0 = e / (QH1 * QH2);
      const int y0 = b0 - 1 + t0, y1 = b1 - 1 + t1, y2 = b2 - 1 + t2;
      in[j] = e < NT && y0 >= 0 && y0 < g.n0 && y1 >= 0 && y1 < g.n1 && y2 >= 0 && y2 < g.n2;
      v[j] = F[in[j] ? ((long)y0 * g.n1 + y1) * g.n2 + y2 : 0];
    }
#pragma unroll
    for (int j = 0; j < U; ++j) {
      const int e = e0 + 256 * j;
      if (e < NT) tile[e] = in[j] ? v[j] : -INFINITY;
    }
  }
  if (tid == 0) lcount = 0u;
  __syncthreads();
  const int t2 = tid % QS2, t1 = tid / QS2;
  const int x1 = b1 + t1, x2 = b2 + t2;
  const bool col_ok = x1 <= g.hi1 && x2 <= g.hi2;
  // window maxima of tile plane t at this column: pe without the centre,
  // pi with it; v the centre
  auto window = [&](int t, float& v, float& pe, float& pi) {
    const float* r = tile + (t * QH1 + t1) * QH2 + t2;
    const float a0 = max_nan(max_nan(r[0], r[1]), r[2]);
    const float a2 = max_nan(max_nan(r[2 * QH2], r[2 * QH2 + 1]), r[2 * QH2 + 2]);
    pe = max_nan(max_nan(a0, a2), max_nan(r[QH2], r[QH2 + 2]));
    v = r[QH2 + 1];
    pi = max_nan(pe, v);
  };
  float v_c, pe_c, pi_p, pi_c, tmp_v, tmp_e;
  window(0, tmp_v, tmp_e, pi_p);
  window(1, v_c, pe_c, pi_c);
  for (int t = 0; t < nv0; ++t) {
    float v_n, pe_n, pi_n;
    window(t + 2, v_n, pe_n, pi_n);
    // the centre plane t + 1 holds x0 = b0 + t
    if (col_ok && v_c > threshold && v_c > pe_c && v_c > pi_p && v_c > pi_n) {
      const long lin = ((long)(b0 + t) * g.n1 + x1) * g.n2 + x2;
      const unsigned ls = atomicAdd(&lcount, 1u);
      lkeys[ls] = peak_key(v_c, lin);
    }
    pi_p = pi_c;
    v_c = v_n;
    pe_c = pe_n;
    pi_c = pi_n;
  }
  __syncthreads();
  const unsigned nl = lcount;
  if (nl == 0u) return;
  if (tid == 0) lbase = atomicAdd(&ctrl[kPeakSubCtl + sub], nl);
  __syncthreads();
  unsigned long long* list = allc + sub * cap_sub + lbase;
  for (unsigned i = tid; i < nl; i += 256) list[i] = lkeys[i];
}

// Histogram of the candidates' key top bits (the float bits of F >> 16): each
// block counts its wavefronts' share of the scan's sub-lists in LDS, then adds
// its non-zero bins to the global histogram.
constexpr int kHistBlocks = 64;
__global__ void __launch_bounds__(1024) k_peaks_hist(const unsigned* __restrict__ ctrl,
                                                     const unsigned long long* __restrict__ allc, long bigcap,
                                                     long cap_sub, unsigned* __restrict__ hist) {
  __shared__ unsigned lh[kHistBins];
  const int tid = threadIdx.x;
  const int plane = blockIdx.y;
  ctrl += kPeakCtrlWords * plane;
  allc += bigcap * plane;
  hist += (long)kHistBins * plane;
  for (int i = tid; i < kHistBins; i += 1024) lh[i] = 0u;
  __syncthreads();
  for_each_key(allc, cap_sub, ctrl, blockIdx.x * 16 + (tid >> 6), gridDim.x * 16, [&](unsigned long long k) {
    const unsigned bits = 0xFFFFFFFFu - (unsigned)(k >> 32);
    atomicAdd(&lh[bits >> 16], 1u);
  });
  __syncthreads();
  for (int i = tid; i < kHistBins; i += 1024) {
    const unsigned v = lh[i];
    if (v) atomicAdd(&hist[i], v);
  }
}

// round r: the smallest bin b with sum_{k >= b} hist[k] <= cap (one block
// of 1024 threads; part: 1024 words of LDS); the outcome (bin, whether
// candidates below it exist) goes to the round's control words and, if
// out is given, to out[0], out[1] (exactly one thread writes it)
__device__ void select_bin(const unsigned* __restrict__ hist, unsigned* __restrict__ ctrl, int round,
                           unsigned cap, unsigned* part, unsigned* out = nullptr) {
  constexpr int per = kHistBins / 1024;
  const int tid = threadIdx.x;
  const int base = round == 1 ? PK_B1 : PK_B2;
  unsigned s = 0;
  for (int i = 0; i < per; ++i) s += hist[tid * per + i];
  part[tid] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const unsigned v = (tid + off < 1024) ? part[tid + off] : 0u;
    __syncthreads();
    part[tid] += v;
    __syncthreads();
  }
  const unsigned above = (tid + 1 < 1024) ? part[tid + 1] : 0u;
  if (part[tid] > cap && above <= cap) {
    unsigned run = above;
    int b = tid * per + per;
    for (int i = per - 1; i >= 0; --i) {
      const unsigned h = hist[tid * per + i];
      if (run + h > cap) break;
      run += h;
      b = tid * per + i;
    }
    ctrl[base] = (unsigned)b;
    ctrl[base + 1] = 1u;           // candidates below b exist
    if (out) {
      out[0] = (unsigned)b;
      out[1] = 1u;
    }
  }
  if (tid == 0 && part[0] <= cap) {
    ctrl[base] = 0u;
    ctrl[base + 1] = 0u;
    if (out) {
      out[0] = 0u;
      out[1] = 0u;
    }
  }
}

__global__ void __launch_bounds__(1024) k_peaks_select(const unsigned* __restrict__ hist,
                                                       unsigned* __restrict__ ctrl) {
  hist += (long)kHistBins * blockIdx.x;
  ctrl += kPeakCtrlWords * blockIdx.x;
  __shared__ unsigned part[1024];
  select_bin(hist, ctrl, 1, kCandCap1, part);
}

// the candidates whose key bin is >= bmin among the scan's sub-lists,
// appended to cand (at most cap; cnt counts them all); this wavefront is
// number `wave` of nwaves sharing the lists
__device__ void gather_keys(unsigned* __restrict__ cnt, unsigned bmin, const unsigned long long* __restrict__ allc,
                            long cap_sub, const unsigned* __restrict__ ctrl, unsigned long long* __restrict__ cand,
                            unsigned cap, int wave, int nwaves) {
  for_each_key(allc, cap_sub, ctrl, wave, nwaves, [&](unsigned long long k) {
    const unsigned bits = 0xFFFFFFFFu - (unsigned)(k >> 32);
    if ((bits >> 16) >= bmin) {
      const unsigned slot = atomicAdd(cnt, 1u);
      if (slot < cap) cand[slot] = k;
    }
  });
}

// round 1: the candidates above the round's bin
__global__ void __launch_bounds__(256) k_peaks_gather(unsigned* __restrict__ ctrl,
                                                      const unsigned long long* __restrict__ allc, long bigcap,
                                                      long cap_sub, unsigned long long* __restrict__ cand) {
  const int plane = blockIdx.y;
  ctrl += kPeakCtrlWords * plane;
  allc += bigcap * plane;
  cand += (long)kCandCap * plane;
  gather_keys(&ctrl[PK_CNT1], ctrl[PK_B1], allc, cap_sub, ctrl, cand, kCandCap1, blockIdx.x * 4 + (threadIdx.x >> 6),
              gridDim.x * 4);
}

__device__ __forceinline__ void decode_lin(unsigned long long key, int n1, int n2, int& x0, int& x1, int& x2) {
  const long lin = (long)(key & 0xFFFFFFFFull);
  x2 = (int)(lin % n2);
  const long r = lin / n2;
  x1 = (int)(r % n1);
  x0 = (int)(r / n1);
}

// one block: bitonic sort of the round's candidate keys (ascending), in
// place.  Round 1 (at most 2048 keys): thread t holds the keys t and t + 1024
// (missing keys are ~0, sorted to the end) in registers; a compare-exchange
// at distance j < 64 pairs lanes of one wavefront (cross-lane shuffles), at
// distance 1024 the two keys of one thread, and only distances 64..512 go
// through LDS.
__device__ __forceinline__ unsigned long long shfl_xor_u64(unsigned long long v, int j) {
  const unsigned lo = (unsigned)__shfl_xor((int)(unsigned)v, j);
  const unsigned hi = (unsigned)__shfl_xor((int)(unsigned)(v >> 32), j);
  return ((unsigned long long)hi << 32) | lo;
}
// the key that element i keeps after the compare-exchange with its partner
// i ^ j (holding y) in the merge of blocks of k
__device__ __forceinline__ unsigned long long bitonic_keep(unsigned long long x, unsigned long long y, int i, int j,
                                                           int k) {
  const bool up = (i & k) == 0, lower = (i & j) == 0;
  return (lower == up) ? (x < y ? x : y) : (x < y ? y : x);
}

__global__ void __launch_bounds__(1024) k_peaks_sort1(const unsigned* __restrict__ ctrl,
                                                      unsigned long long* __restrict__ cand) {
  ctrl += kPeakCtrlWords * blockIdx.x;
  cand += (long)kCandCap * blockIdx.x;
  __shared__ unsigned long long keys[kCandCap1];
  const unsigned nc = min(ctrl[PK_CNT1], kCandCap1);
  const int ia = threadIdx.x, ib = threadIdx.x + 1024;
  unsigned long long a = ia < (int)nc ? cand[ia] : ~0ull;
  unsigned long long b = ib < (int)nc ? cand[ib] : ~0ull;
#pragma unroll
  for (int k = 2; k <= (int)kCandCap1; k <<= 1) {
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
      unsigned long long pa, pb;
      if (j == 1024) {
        pa = b;
        pb = a;
      } else if (j >= 64) {
        keys[ia] = a;
        keys[ib] = b;
        __syncthreads();
        pa = keys[ia ^ j];
        pb = keys[ib ^ j];
        __syncthreads();
      } else {
        pa = shfl_xor_u64(a, j);
        pb = shfl_xor_u64(b, j);
      }
      a = bitonic_keep(a, pa, ia, j, k);
      b = bitonic_keep(b, pb, ib, j, k);
    }
  }
  if (ia < (int)nc) cand[ia] = a;
  if (ib < (int)nc) cand[ib] = b;
}

// the whole network in LDS over keys[0, np2) (np2 the power of two >= n,
// keys past n set to ~0), by a block of 1024 threads
__device__ void sort_keys_lds(unsigned long long* keys, int n) {
  const int tid = threadIdx.x;
  int np2 = 1;
  while (np2 < n) np2 <<= 1;
  for (int i = n + tid; i < np2; i += 1024) keys[i] = ~0ull;
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
}

// LDS writes of a wavefront made visible to its other lanes
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// one wavefront: greedy suppression over the nc sorted candidate keys, 64 at
// a time.  Each lane tests its candidate against the accepted list
// (acc_pos, 3 x max_peaks coordinates); conflicts inside the chunk are
// resolved in candidate order with lane broadcasts.  exhausted: the list ran
// out before max_peaks peaks were accepted.
template <class AccT>
__device__ void nms_wave(const PeakGeo& g, const unsigned long long* keys, unsigned nc, float min_dist,
                         int max_peaks, AccT* acc_pos, int* __restrict__ out_pos, float* __restrict__ out_score,
                         int& nacc_out, bool& exhausted_out) {
  const int lane = threadIdx.x & 63;
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
    const unsigned long long key = have ? keys[i] : ~0ull;
    int x0 = 0, x1 = 0, x2 = 0;
    if (have) decode_lin(key, g.n1, g.n2, x0, x1, x2);
    bool sup = !have;
    for (int q = 0; q < nacc && !sup; ++q) {
      const float d0 = (float)(x0 - (int)acc_pos[3 * q]), d1 = (float)(x1 - (int)acc_pos[3 * q + 1]),
                  d2 = (float)(x2 - (int)acc_pos[3 * q + 2]);
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
    if ((accepted >> lane) & 1ull) {
      const int rank = nacc0 + __popcll(accepted & ((1ull << lane) - 1ull));
      acc_pos[3 * rank] = (AccT)x0;
      acc_pos[3 * rank + 1] = (AccT)x1;
      acc_pos[3 * rank + 2] = (AccT)x2;
      out_pos[3 * rank] = x0;
      out_pos[3 * rank + 1] = x1;
      out_pos[3 * rank + 2] = x2;
      out_score[rank] = __uint_as_float(0xFFFFFFFFu - (unsigned)(key >> 32));
    }
    wave_sync();
  }
  nacc_out = nacc;
  exhausted_out = exhausted;
}

// round 1's suppression, one wavefront per map; asks for round 2 (a larger
// candidate list) when its list ran out before max_peaks peaks were
// accepted while lower candidates exist
__global__ void __launch_bounds__(64) k_peaks_nms(PeakGeo g, unsigned* __restrict__ ctrl,
                                                  const unsigned long long* __restrict__ cand, float min_dist,
                                                  int max_peaks, int* __restrict__ out_pos,
                                                  float* __restrict__ out_score, int* __restrict__ out_count) {
  const int plane = blockIdx.x;
  ctrl += kPeakCtrlWords * plane;
  cand += (long)kCandCap * plane;
  out_pos += 3L * max_peaks * plane;
  out_score += (long)max_peaks * plane;
  out_count += 2 * plane;
  __shared__ int acc_pos[3 * 4096];
  const unsigned ncount = ctrl[PK_CNT1];
  const bool more_below = ctrl[PK_MORE1] != 0u || ncount > kCandCap1;
  int nacc = 0;
  bool exhausted = true;
  nms_wave(g, cand, min(ncount, kCandCap1), min_dist, max_peaks, acc_pos, out_pos, out_score, nacc, exhausted);
  if (threadIdx.x == 0) {
    const bool short_list = nacc < max_peaks && exhausted && more_below;
    out_count[0] = nacc;
    out_count[1] = 0;
    if (short_list) ctrl[PK_REDO] = 1u;
  }
}

// round 2, only where round 1 asked for it, in one block per map: the bin
// for kCandCap candidates, their gather, a sort in LDS and the suppression
// by the first wavefront (its accepted coordinates as 16-bit values: every
// extent is at most 8192)
__global__ void __launch_bounds__(1024) k_peaks_round2(PeakGeo g, const unsigned* __restrict__ hist,
                                                       unsigned* __restrict__ ctrl,
                                                       const unsigned long long* __restrict__ allc, long bigcap,
                                                       long cap_sub,
                                                       unsigned long long* __restrict__ cand, float min_dist,
                                                       int max_peaks, int* __restrict__ out_pos,
                                                       float* __restrict__ out_score, int* __restrict__ out_count) {
  const int plane = blockIdx.x;
  hist += (long)kHistBins * plane;
  ctrl += kPeakCtrlWords * plane;
  allc += bigcap * plane;
  cand += (long)kCandCap * plane;
  out_pos += 3L * max_peaks * plane;
  out_score += (long)max_peaks * plane;
  out_count += 2 * plane;
  if (ctrl[PK_REDO] == 0u) return;
  __shared__ unsigned long long keys[kCandCap];   // the select's partial sums, then the keys
  __shared__ short acc_pos[3 * 4096];
  __shared__ unsigned sel[2], s_count;
  const int tid = threadIdx.x;
  select_bin(hist, ctrl, 2, kCandCap, reinterpret_cast<unsigned*>(keys), sel);
  __syncthreads();
  const unsigned bmin = sel[0];
  const bool more_flag = sel[1] != 0u;
  gather_keys(&ctrl[PK_CNT2], bmin, allc, cap_sub, ctrl, cand, kCandCap, tid >> 6, 16);
  __syncthreads();
  // the count from the atomic unit (the counter's cache line was read at the start)
  if (tid == 0) s_count = atomicAdd(&ctrl[PK_CNT2], 0u);
  __syncthreads();
  const unsigned ncount = s_count;
  const unsigned nc = min(ncount, (unsigned)kCandCap);
  for (int i = tid; i < (int)nc; i += 1024) keys[i] = cand[i];
  sort_keys_lds(keys, (int)nc);
  if (tid >= 64) return;
  int nacc = 0;
  bool exhausted = true;
  nms_wave(g, keys, nc, min_dist, max_peaks, acc_pos, out_pos, out_score, nacc, exhausted);
  if (tid == 0) {
    const bool short_list = nacc < max_peaks && exhausted && (more_flag || ncount > (unsigned)kCandCap);
    out_count[0] = nacc;
    out_count[1] = short_list ? TTM_PEAKS_TRUNCATED : 0;
  }
}

// the histogram and control words of every map cleared in one launch
__global__ void k_peaks_clear(unsigned* __restrict__ hist, long nh, unsigned* __restrict__ ctrl, int nc) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nh) hist[i] = 0u;
  else if (i < nh + nc) ctrl[i - nh] = 0u;
}

// the scan's grid over one map: runs of `run` planes (one for a single
// plane) and blocks of QS1 x QS2 columns over the valid region
struct PeakGrid {
  int run, ztiles, gy, gx;
  long nblk() const { return (long)ztiles * gy * gx; }
  // a sub-list's capacity: its blocks' keys
  long cap_sub() const { return (nblk() + kPeakSubs - 1) / kPeakSubs * peak_region_keys(run); }
};
static PeakGrid peak_grid(const Geo& gg) {
  const int e0 = gg.n0 - gg.L0 + 1, e1 = gg.n1 - gg.L1 + 1, e2 = gg.n2 - gg.L2 + 1;
  PeakGrid pg;
  pg.run = gg.n0 == 1 ? 1 : QRUN;
  pg.ztiles = (e0 + pg.run - 1) / pg.run;
  pg.gy = (e1 + QS1 - 1) / QS1;
  pg.gx = (e2 + QS2 - 1) / QS2;
  return pg;
}

// the scan's sub-lists
long peaks_bigcap(const Geo& g) { return kPeakSubs * peak_grid(g).cap_sub(); }

hipError_t launch_peaks(const Geo& gg, const float* score, float threshold, float min_dist,
                        int max_peaks, const PeakWs& w, int* out_pos, float* out_score,
                        int* out_count, hipStream_t s, int planes) {
  PeakGeo g;
  g.n0 = gg.n0; g.n1 = gg.n1; g.n2 = gg.n2;
  g.lo0 = gg.c0; g.hi0 = gg.n0 - gg.L0 + gg.c0;
  g.lo1 = gg.c1; g.hi1 = gg.n1 - gg.L1 + gg.c1;
  g.lo2 = gg.c2; g.hi2 = gg.n2 - gg.L2 + gg.c2;
  const long bigcap = peaks_bigcap(gg);
  const PeakGrid pg = peak_grid(gg);
  const long cap_sub = pg.cap_sub();
  const unsigned P = (unsigned)planes;
  const long nh = (long)kHistBins * planes;
  const int nctl = kPeakCtrlWords * planes;
  hipLaunchKernelGGL(k_peaks_clear, dim3((unsigned)((nh + nctl + 255) / 256)), dim3(256), 0, s, w.hist, nh, w.ctrl,
                     nctl);
  dim3 sgrid((unsigned)pg.gx, (unsigned)pg.gy, (unsigned)pg.ztiles * P);
  if (pg.run == 1)
    hipLaunchKernelGGL(k_peaks_scan<1>, sgrid, dim3(256), 0, s, score, g, threshold, w.ctrl, w.allc, bigcap,
                       cap_sub, pg.ztiles, gg.vol());
  else
    hipLaunchKernelGGL(k_peaks_scan<QRUN>, sgrid, dim3(256), 0, s, score, g, threshold, w.ctrl, w.allc, bigcap,
                       cap_sub, pg.ztiles, gg.vol());
  hipLaunchKernelGGL(k_peaks_hist, dim3(kHistBlocks, P), dim3(1024), 0, s, w.ctrl, w.allc, bigcap, cap_sub, w.hist);
  hipLaunchKernelGGL(k_peaks_select, dim3(P), dim3(1024), 0, s, w.hist, w.ctrl);
  hipLaunchKernelGGL(k_peaks_gather, dim3(256, P), dim3(256), 0, s, w.ctrl, w.allc, bigcap, cap_sub, w.cand);
  hipLaunchKernelGGL(k_peaks_sort1, dim3(P), dim3(1024), 0, s, w.ctrl, w.cand);
  hipLaunchKernelGGL(k_peaks_nms, dim3(P), dim3(64), 0, s, g, w.ctrl, w.cand, min_dist, max_peaks, out_pos,
                     out_score, out_count);
  hipLaunchKernelGGL(k_peaks_round2, dim3(P), dim3(1024), 0, s, g, w.hist, w.ctrl, w.allc, bigcap, cap_sub,
                     w.cand, min_dist, max_peaks, out_pos, out_score, out_count);
  return hipGetLastError();
}

// ----------------------------------------------------------------------------
// pose
// ----------------------------------------------------------------------------
struct PoseGeo {
  int n0, n1, n2, L0, L1, L2;
  int lo0, hi0, lo1, hi1, lo2, hi2;
  int planar;   // a stack of planes: neighbours in other planes are outside
};

constexpr int kTensorChunk = 36;

// point i of the n-point super-Fibonacci spiral on S^3 (Alexa, CVPR 2022):
// phi = sqrt(2), psi the real root of psi^4 = psi + 4
__device__ __forceinline__ void seed_point(int i, int n, double* q) {
  const double phi = 1.4142135623730950488;
  const double psi = 1.533751168755204288118041;
  const double s = i + 0.5;
  const double r = sqrt(s / n), R = sqrt(1.0 - s / n);
  const double al = 6.283185307179586477 * s / phi, be = 6.283185307179586477 * s / psi;
  q[0] = r * sin(al);
  q[1] = r * cos(al);
  q[2] = R * sin(be);
  q[3] = R * cos(be);
}

__global__ void k_seed_table(int n, double* __restrict__ seeds) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) seed_point(i, n, seeds + 4 * i);
}

// 256-thread sum of kTensorChunk values per thread (wave shuffles, then LDS)
__device__ __forceinline__ void block_sum_chunk(double* v, int kc, double* sh /* 4 * kTensorChunk */) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < kTensorChunk; ++i) {
    if (i < kc) {
      double t = v[i];
      for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off);
      if (lane == 0) sh[wave * kTensorChunk + i] = t;
    }
  }
  __syncthreads();
  if (threadIdx.x < kc)
    v[0] = sh[threadIdx.x] + sh[kTensorChunk + threadIdx.x] + sh[2 * kTensorChunk + threadIdx.x] +
           sh[3 * kTensorChunk + threadIdx.x];
  __syncthreads();
}

__device__ __forceinline__ double block_sum(double v, double* sh) {
  double a[kTensorChunk];
  a[0] = v;
  block_sum_chunk(a, 1, sh);
  if (threadIdx.x == 0) sh[0] = a[0];
  __syncthreads();
  const double r = sh[0];
  __syncthreads();
  return r;
}

__device__ __forceinline__ void neighbour_offset(int k, int NB, int& o0, int& o1, int& o2) {
  if (NB == 27) {
    o0 = k / 9 - 1;
    o1 = (k / 3) % 3 - 1;
    o2 = k % 3 - 1;
  } else {
    o0 = o1 = o2 = 0;
  }
}

// C_alpha(x) = w(x) <tau_x f, T_alpha> in float64 at x = pos[p] + offset(k), with
// w(x) from the two-pass masked mean and variance of the window (Section 2).
__global__ void __launch_bounds__(256) k_pose_tensor(PoseGeo g, const float* __restrict__ image,
                                                     const float* __restrict__ comps,
                                                     const float* __restrict__ mask, int K,
                                                     const double* __restrict__ img_stats, float eps_v,
                                                     const int* __restrict__ pos, const int* __restrict__ count_dev,
                                                     int count_host, int NB, double* __restrict__ Cbuf,
                                                     double* __restrict__ wbuf, int* __restrict__ okbuf,
                                                     const int* __restrict__ active) {
  __shared__ double sh[4 * kTensorChunk];
  const int b = blockIdx.x;
  const int p = b / NB, k = b % NB;
  const int count = count_dev ? count_dev[0] : count_host;
  if (p >= count || (active && !active[p])) return;
  const int tid = threadIdx.x;
  int o0, o1, o2;
  neighbour_offset(k, NB, o0, o1, o2);
  const int x0 = pos[3 * p] + o0, x1 = pos[3 * p + 1] + o1, x2 = pos[3 * p + 2] + o2;
  const bool inside = x0 >= g.lo0 && x0 <= g.hi0 && x1 >= g.lo1 && x1 <= g.hi1 && x2 >= g.lo2 && x2 <= g.hi2 &&
                      !(g.planar && o0 != 0);
  if (!inside) {
    if (tid == 0) {
      okbuf[b] = 0;
      wbuf[b] = 0.0;
    }
    return;
  }
  const int L0 = g.L0, L1 = g.L1, L2 = g.L2, nL = L0 * L1 * L2;
  const int c0 = L0 / 2, c1 = L1 / 2, c2 = L2 / 2;
  // the window lies inside the image (valid region), no wrap needed
  const float* base = image + ((long)(x0 - c0) * g.n1 + (x1 - c1)) * g.n2 + (x2 - c2);
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
  // a planar stack: only the entries (n - k, k, 0, 0), at packed index
  // C(k + 2, 3), can be non-zero; the others are written as zeros
  int Kc = K;
  if (g.planar) {
    Kc = 0;
    while ((Kc + 1) * (Kc + 2) * (Kc + 3) / 6 < K) ++Kc;
    ++Kc;
    for (int e = tid; e < K; e += 256) {
      bool on = false;
      for (int i = 0; i < Kc; ++i) on = on || e == i * (i + 1) * (i + 2) / 6;
      if (!on) Cbuf[(long)b * K + e] = 0.0;
    }
  }
  auto comp_of = [&](int i) { return g.planar ? i * (i + 1) * (i + 2) / 6 : i; };
  for (int k0 = 0; k0 < Kc; k0 += kTensorChunk) {
    const int kc = min(kTensorChunk, Kc - k0);
    double acc[kTensorChunk];
#pragma unroll
    for (int i = 0; i < kTensorChunk; ++i) acc[i] = 0.0;
    if (g.planar) {
      for (int u = tid; u < nL; u += 256) {
        const double v = img_at(u);
#pragma unroll
        for (int i = 0; i <= kPlanarMaxOrder; ++i)
          if (i < kc) acc[i] += v * (double)comps[(long)(i * (i + 1) * (i + 2) / 6) * nL + u];
      }
    } else {
      for (int u = tid; u < nL; u += 256) {
        const double v = img_at(u);
        const float* cu = comps + (long)k0 * nL + u;
#pragma unroll
        for (int i = 0; i < kTensorChunk; ++i)
          if (i < kc) acc[i] += v * (double)cu[(long)i * nL];
      }
    }
    block_sum_chunk(acc, kc, sh);
    if (tid < kc) Cbuf[(long)b * K + comp_of(k0 + tid)] = acc[0] * w;
  }
  if (tid == 0) {
    okbuf[b] = 1;
    wbuf[b] = w;
  }
}

// ---- the direct tensor at candidates, all neighbours of a candidate together ----
// G_alpha(y) = <tau_y f, T_alpha> in float64 for the voxels y = x + o of a
// candidate x: the 27 neighbours (o in {-1, 0, 1}^3) or the voxel itself.  A
// block takes one candidate, one offset o0 along axis 0 and a group of four
// components; each thread takes template columns (u0, u2) and walks u1,
// keeping the 3 x 3 patch f(x + o + u - c), o = (o0, o1, o2), in registers
// (three new values per step) and a 9 x 4 tile of partial sums (offsets x
// components).
// The partial sums are added over the block in a fixed order.  The last
// component group of each candidate takes the masked moments instead:
// sum m f, sum m f^2 and sum m per offset, for w (Section 2, local
// normalisation), which k_pose_direct_finish applies.
constexpr int kDirThreads = 256;
constexpr int kDirGroup = 4;   // components per block

template <int O>   // 3: the 27 neighbours; 1: the voxel only
__global__ void __launch_bounds__(kDirThreads) k_pose_direct(PoseGeo g, const float* __restrict__ image,
                                                             const float* __restrict__ comps,
                                                             const float* __restrict__ mask, int K,
                                                             const int* __restrict__ pos,
                                                             const int* __restrict__ count_dev, int count_host,
                                                             double* __restrict__ Gbuf, double* __restrict__ mom,
                                                             const int* __restrict__ active) {
  constexpr int NO = O * O;                  // offsets (o1, o2) per block
  constexpr int NBT = O * O * O;
  __shared__ double red[4][NO * kDirGroup];
  const int p = blockIdx.x;
  const int count = count_dev ? count_dev[0] : count_host;
  if (p >= count || (active && !active[p])) return;
  const int o0 = (int)blockIdx.y - (O / 2);
  const int ag = blockIdx.z;
  const int ngroups = (K + kDirGroup - 1) / kDirGroup;
  const bool moments = ag == ngroups;
  const int L0 = g.L0, L1 = g.L1, L2 = g.L2;
  const long nL = (long)L0 * L1 * L2;
  const int tid = threadIdx.x;
  // window origin: image voxel of template voxel u = 0 at offset o = 0
  const int b0 = pos[3 * p] - L0 / 2 + o0, b1 = pos[3 * p + 1] - L1 / 2, b2 = pos[3 * p + 2] - L2 / 2;
  const int H = O / 2;
  double acc[NO][kDirGroup];
#pragma unroll
  for (int j = 0; j < NO; ++j)
#pragma unroll
    for (int a = 0; a < kDirGroup; ++a) acc[j][a] = 0.0;
  // f at image (x0, x1, x2), zero outside the image (such neighbours are
  // outside the valid region and discarded)
  auto img = [&](int x0, int x1, int x2) -> double {
    const bool in = x0 >= 0 && x0 < g.n0 && x1 >= 0 && x1 < g.n1 && x2 >= 0 && x2 < g.n2;
    const float v = image[in ? ((long)x0 * g.n1 + x1) * g.n2 + x2 : 0];
    return in ? (double)v : 0.0;
  };
  // each thread walks template columns (u0, u2) along u1; neighbouring lanes
  // take neighbouring u2, so every load of the walk is coalesced
  for (int col = tid; col < L0 * L2; col += kDirThreads) {
    const int u0 = col / L2, u2 = col - u0 * L2;
    const int x0 = b0 + u0;
    // the patch rows u1 - 1, u1, u1 + 1 (O = 3) of columns o2 = -1, 0, 1:
    // win[i][j] = f at offset (o1, o2) = (i - H, j - H)
    double win[O][O];
#pragma unroll
    for (int i = 0; i + 1 < O; ++i)
#pragma unroll
      for (int j = 0; j < O; ++j) win[i + 1][j] = img(x0, b1 + i - H, b2 + u2 + j - H);
    for (int u1 = 0; u1 < L1; ++u1) {
#pragma unroll
      for (int i = 0; i + 1 < O; ++i)
#pragma unroll
        for (int j = 0; j < O; ++j) win[i][j] = win[i + 1][j];
#pragma unroll
      for (int j = 0; j < O; ++j) win[O - 1][j] = img(x0, b1 + u1 + H, b2 + u2 + j - H);
      const long tu = ((long)u0 * L1 + u1) * L2 + u2;
      double t[kDirGroup];
      if (moments) {
        const double m = (double)mask[tu];
        t[0] = m; t[1] = m; t[2] = m; t[3] = 0.0;
      } else {
#pragma unroll
        for (int a = 0; a < kDirGroup; ++a) {
          const int al = ag * kDirGroup + a;
          const float v = comps[(al < K ? al : 0) * nL + tu];
          t[a] = al < K ? (double)v : 0.0;
        }
      }
#pragma unroll
      for (int i = 0; i < O; ++i)
#pragma unroll
        for (int j = 0; j < O; ++j) {
          const double f = win[i][j];
          if (moments) {
            acc[i * O + j][0] += t[0] * f;
            acc[i * O + j][1] += t[1] * f * f;
            acc[i * O + j][2] += t[2];
          } else {
#pragma unroll
            for (int a = 0; a < kDirGroup; ++a) acc[i * O + j][a] += t[a] * f;
          }
        }
    }
  }
  // block sums in a fixed order: waves by shuffles, then the four wave sums
  const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
  for (int j = 0; j < NO; ++j)
#pragma unroll
    for (int a = 0; a < kDirGroup; ++a) {
      double v = acc[j][a];
      for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
      if (lane == 0) red[wave][j * kDirGroup + a] = v;
    }
  __syncthreads();
  if (tid < NO * kDirGroup) {
    const double sum = red[0][tid] + red[1][tid] + red[2][tid] + red[3][tid];
    const int j = tid / kDirGroup, a = tid % kDirGroup;
    // neighbour index k = 9 (o0 + 1) + 3 (o1 + 1) + (o2 + 1) (O = 3), or 0
    const int k = O == 3 ? 9 * (o0 + 1) + j : 0;
    const long b = (long)p * NBT + k;
    if (moments) {
      if (a < 3) mom[3 * b + a] = sum;
    } else {
      const int al = ag * kDirGroup + a;
      if (al < K) Gbuf[b * K + al] = sum;
    }
  }
}

// w = 1 / sqrt(sum m f^2 - (sum m f)^2 / sum m) (0 at or below the variance
// floor), the ok flag (the voxel inside the valid region), C_alpha = w G_alpha
__global__ void __launch_bounds__(256) k_pose_direct_finish(PoseGeo g, int K, const double* __restrict__ img_stats,
                                                            float eps_v, const int* __restrict__ pos,
                                                            const int* __restrict__ count_dev, int count_host,
                                                            int NB, int total, const double* __restrict__ mom,
                                                            double* __restrict__ Cbuf, double* __restrict__ wbuf,
                                                            int* __restrict__ okbuf, const int* __restrict__ active) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= total) return;
  const int p = b / NB, k = b % NB;
  const int count = count_dev ? count_dev[0] : count_host;
  if (p >= count || (active && !active[p])) return;
  int o0, o1, o2;
  neighbour_offset(k, NB, o0, o1, o2);
  const int x0 = pos[3 * p] + o0, x1 = pos[3 * p + 1] + o1, x2 = pos[3 * p + 2] + o2;
  const bool inside = x0 >= g.lo0 && x0 <= g.hi0 && x1 >= g.lo1 && x1 <= g.hi1 && x2 >= g.lo2 && x2 <= g.hi2;
  if (!inside) {
    okbuf[b] = 0;
    wbuf[b] = 0.0;
    return;
  }
  const double s1 = mom[3 * (long)b], s2 = mom[3 * (long)b + 1], msum = mom[3 * (long)b + 2];
  const double var = s2 - s1 * s1 / msum;
  const double floor_v = (double)eps_v * msum * img_stats[1];
  const double w = var > floor_v ? 1.0 / sqrt(var) : 0.0;
  for (int a = 0; a < K; ++a) Cbuf[(long)b * K + a] *= w;
  okbuf[b] = 1;
  wbuf[b] = w;
}

// Per-wave LDS table of the eigen-solver: the packed tensor entries C.
struct EigLds {
  double C[kMaxK];
};

// Dominant Z-eigenpair of one packed tensor per 256-thread block, in two
// phases.  The seed scan (all four wavefronts): lambda(s) = sum_alpha mu_alpha
// C_alpha s^alpha at every S^3 seed point s, thread t taking the seeds t,
// t + 256, ...; for each of 64 slots l the largest value over the seeds
// s = l mod 64 and its seed index (the lowest index on ties), the four threads
// t = l mod 64 merged.  Then the first wavefront alone: lane l takes slot l's
// best seed; the kStarts best mutually distant lane seeds are polished by
// SS-HOPM (shifted power iteration) accelerated with Newton steps on the
// sphere: a Newton step is taken when it is an ascent direction and a
// backtracking search along it raises lambda, otherwise the shifted power
// step; the wave keeps the best lambda.  The other wavefronts leave after the
// scan, so the polish synchronises within its wavefront only.
constexpr int kStarts = 8;
template <int N>
__global__ void __launch_bounds__(256) k_pose_eig(const double* __restrict__ seeds,
                                                  const double* __restrict__ Cbuf,
                                                  const int* __restrict__ okbuf, const int* __restrict__ count_dev,
                                                  int count_host, int NB, int n_seeds, int max_iter, double tol,
                                                  float* __restrict__ qbuf, double* __restrict__ lambuf,
                                                  int* __restrict__ flagbuf, const int* __restrict__ active) {
  constexpr int n = N;
  constexpr int K = (N + 1) * (N + 2) * (N + 3) / 6;
  __shared__ double muA[K];
  __shared__ double rb[256];
  __shared__ int ri[256];
  __shared__ EigLds t;
  __shared__ double red[64 * 6];
  const int b = blockIdx.x;
  const int p = b / NB;
  const int tid = threadIdx.x;
  const int count = count_dev ? count_dev[0] : count_host;
  if (p >= count || (active && !active[p])) return;
  if (!okbuf[b]) {
    if (tid == 0) {
      lambuf[b] = -INFINITY;
      flagbuf[b] = 0;
    }
    return;
  }
  for (int k = tid; k < K; k += 256) {
    int al[4];
    alpha_of_dev(N, k, al);
    double mu = fact_d(N);
    for (int d = 0; d < 4; ++d) mu /= fact_d(al[d]);
    const double c = Cbuf[(long)b * K + k];
    muA[k] = mu * c;
    t.C[k] = c;
  }
  __syncthreads();
  {
    double bv = -INFINITY;
    int bs = 0;
    for (int sd = tid; sd < n_seeds; sd += 256) {
      const double q[4] = {seeds[4 * sd], seeds[4 * sd + 1], seeds[4 * sd + 2], seeds[4 * sd + 3]};
      const double v = eval_lambda<N>(muA, q);
      if (v > bv) {
        bv = v;
        bs = sd;
      }
    }
    rb[tid] = bv;
    ri[tid] = bs;
  }
  __syncthreads();
  if (tid >= 64) return;
  const int lane = tid;
  // the seed scan's best seed of this lane's slot
  double best = rb[lane];
  int bseed = ri[lane];
  for (int j = 1; j < 4; ++j) {
    const double v = rb[lane + 64 * j];
    const int i = ri[lane + 64 * j];
    if (v > best || (v == best && v > -INFINITY && i < bseed)) {
      best = v;
      bseed = i;
    }
  }
  // the kStarts best lane seeds that are mutually more than 10 degrees apart
  // (|<q, q'>| < cos 5 deg) start the polish
  red[lane * 6 + 0] = best;
  red[lane * 6 + 1] = (double)bseed;
  // every lane's seed point, loaded by all lanes at once, so that the walk
  // over the slots below reads LDS only
  __shared__ double sq[64][4];
  for (int d = 0; d < 4; ++d) sq[lane][d] = seeds[4 * bseed + d];
  wave_sync();
  __shared__ int nstart;
  __shared__ double sel[kStarts][4];
  // each slot's place in the order (best first, the lower lane on ties),
  // found by all lanes at once, so that lane 0 walks the slots once instead
  // of searching the unused ones for every start it takes; NaN slot values
  // (a non-finite tensor) keep the search
  __shared__ int order[64];
  __shared__ int any_nan;
  if (lane == 0) any_nan = 0;
  wave_sync();
  {
    int rank = 0;
    for (int l = 0; l < 64; ++l) {
      const double v = red[l * 6];
      rank += (v > best) || (v == best && l < lane);
    }
    if (best != best) any_nan = 1;
    else order[rank] = lane;
  }
  wave_sync();
  if (lane == 0 && !any_nan) {
    const double cosx = 0.99619469809174553;
    int ns = 0;
    for (int k = 0; k < 64 && ns < kStarts; ++k) {
      const int bl = order[k];
      if (!(red[bl * 6] > -INFINITY)) break;
      const double q[4] = {sq[bl][0], sq[bl][1], sq[bl][2], sq[bl][3]};
      bool far = true;
      for (int i = 0; i < ns; ++i) {
        const double dp = q[0] * sel[i][0] + q[1] * sel[i][1] + q[2] * sel[i][2] + q[3] * sel[i][3];
        if (fabs(dp) > cosx) far = false;
      }
      if (!far) continue;
      for (int d = 0; d < 4; ++d) sel[ns][d] = q[d];
      ++ns;
    }
    nstart = ns;
  }
  if (lane == 0 && any_nan) {
    const double cosx = 0.99619469809174553;
    unsigned long long used = 0ull;
    int ns = 0;
    while (ns < kStarts) {
      int bl = -1;
      for (int l = 0; l < 64; ++l)
        if (!((used >> l) & 1ull) && (bl < 0 || red[l * 6] > red[bl * 6])) bl = l;
      if (bl < 0 || !(red[bl * 6] > -INFINITY)) break;
      used |= 1ull << bl;
      const double q[4] = {sq[bl][0], sq[bl][1], sq[bl][2], sq[bl][3]};
      bool far = true;
      for (int i = 0; i < ns; ++i) {
        const double dp = q[0] * sel[i][0] + q[1] * sel[i][1] + q[2] * sel[i][2] + q[3] * sel[i][3];
        if (fabs(dp) > cosx) far = false;
      }
      if (!far) continue;
      for (int d = 0; d < 4; ++d) sel[ns][d] = q[d];
      ++ns;
    }
    nstart = ns;
  }
  wave_sync();
  double lam = -INFINITY;
  double x[4] = {1.0, 0.0, 0.0, 0.0};
  bool conv = false;
  // the best seed may iterate up to max_iter; the runner-up seeds, kept for
  // near-degenerate tensors with competing maxima, stop after 12 iterations
  // (from the scan's seeds they converge in 4 to 6; the wave waits for its
  // slowest lane)
  const int lane_iters = lane == 0 ? max_iter : min(max_iter, 12);
  if (lane < nstart) {
    for (int d = 0; d < 4; ++d) x[d] = sel[lane][d];
    conv = eig_polish<N>(t.C, x, lam, lane_iters, tol);
  }
  // wave argmax of lambda (lowest lane on ties)
  wave_sync();
  red[lane * 6 + 0] = lam;
  red[lane * 6 + 1] = x[0];
  red[lane * 6 + 2] = x[1];
  red[lane * 6 + 3] = x[2];
  red[lane * 6 + 4] = x[3];
  red[lane * 6 + 5] = conv ? 0.0 : 1.0;
  wave_sync();
  if (lane == 0) {
    int bl = 0;
    for (int l = 1; l < 64; ++l)
      if (red[l * 6] > red[bl * 6]) bl = l;
    double q[4] = {red[bl * 6 + 1], red[bl * 6 + 2], red[bl * 6 + 3], red[bl * 6 + 4]};
    const double nq = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    double sgn = 1.0;
    for (int d = 0; d < 4; ++d)
      if (q[d] != 0.0) {
        sgn = q[d] > 0.0 ? 1.0 : -1.0;
        break;
      }
    for (int d = 0; d < 4; ++d) qbuf[4 * b + d] = (float)(sgn * q[d] / nq);
    lambuf[b] = red[bl * 6];
    flagbuf[b] = red[bl * 6 + 5] != 0.0 ? TTM_POSE_NOT_CONVERGED : 0;
  }
}

// The dominant eigenpair of a planar tensor (a stack of planes: every
// rotation is about axis 0, the quaternion (a, b, 0, 0) with (a, b) the unit
// complex number of half the angle, and only the volume entries
// (n - k, k, 0, 0), at packed index C(k + 2, 3), are non-zero).  On the unit
// circle phi(psi) = sum_k C(n, k) C_k cos^(n-k) psi sin^k psi; psi in [0, pi)
// covers every rotation once.  One wavefront per tensor, in float64:
// kPlanarScan samples psi_j = (j + 1/2) pi / kPlanarScan (lane l takes
// j = l, l + 64, ..., stepping its (cos, sin) by one complex product), the
// best sample (lowest j on ties); then kPlanarZoom parallel zoom levels, each
// sampling 64 points evenly over [c - h, c + h] around the best point c so
// far and narrowing h to the sample spacing (h / 31.5), which shrinks the
// bracket of one scan step (pi / 1024) to below 1e-11 rad.
constexpr int kPlanarScan = 1024;
constexpr int kPlanarZoom = 6;
template <int N>
__device__ __forceinline__ double planar_phi(const double (&a)[N + 1], double c, double s) {
  double cp[N + 1], sp[N + 1];
  cp[0] = sp[0] = 1.0;
#pragma unroll
  for (int e = 1; e <= N; ++e) {
    cp[e] = cp[e - 1] * c;
    sp[e] = sp[e - 1] * s;
  }
  double v = 0.0;
#pragma unroll
  for (int k = 0; k <= N; ++k) v += a[k] * cp[N - k] * sp[k];
  return v;
}

// wave argmax of (v, key): the larger v, the lower key on ties; every lane
// ends with the winner
__device__ __forceinline__ void wave_argmax(double& v, int& key) {
  for (int off = 32; off > 0; off >>= 1) {
    const double ov = __shfl_xor(v, off);
    const int ok = __shfl_xor(key, off);
    if (ov > v || (ov == v && ok < key)) {
      v = ov;
      key = ok;
    }
  }
}

template <int N>
__global__ void __launch_bounds__(64) k_planar_eig(const double* __restrict__ Cbuf, const int* __restrict__ okbuf,
                                                  const int* __restrict__ count_dev, int count_host, int NB,
                                                  float* __restrict__ qbuf, double* __restrict__ lambuf,
                                                  int* __restrict__ flagbuf, const int* __restrict__ active) {
  constexpr int K = (N + 1) * (N + 2) * (N + 3) / 6;
  const int b = blockIdx.x;
  const int p = b / NB;
  const int lane = threadIdx.x;
  const int count = count_dev ? count_dev[0] : count_host;
  if (p >= count || (active && !active[p])) return;
  if (!okbuf[b]) {
    if (lane == 0) {
      lambuf[b] = -INFINITY;
      flagbuf[b] = 0;
    }
    return;
  }
  double a[N + 1];
#pragma unroll
  for (int k = 0; k <= N; ++k) {
    double binom = 1.0;
    for (int i = 1; i <= k; ++i) binom = binom * (N - k + i) / i;
    a[k] = binom * Cbuf[(long)b * K + k * (k + 1) * (k + 2) / 6];
  }
  const double pi = 3.14159265358979323846;
  const double step = pi / kPlanarScan;
  // scan: lane l at psi_l = (l + 1/2) step, advanced by 64 steps per sample
  double c, s, dc, ds;
  sincos((lane + 0.5) * step, &s, &c);
  sincos(64.0 * step, &ds, &dc);
  double best = -INFINITY;
  int bj = 0;
  for (int j = lane; j < kPlanarScan; j += 64) {
    const double v = planar_phi<N>(a, c, s);
    if (v > best) {
      best = v;
      bj = j;
    }
    const double cn = c * dc - s * ds;
    s = s * dc + c * ds;
    c = cn;
  }
  wave_argmax(best, bj);
  // zoom: the best point so far stays a candidate, so lambda never drops
  double centre = (bj + 0.5) * step, h = step;
  sincos(centre, &s, &c);
  best = planar_phi<N>(a, c, s);
  for (int lev = 0; lev < kPlanarZoom; ++lev) {
    const double x = centre + (lane - 31.5) * (h / 31.5);
    sincos(x, &s, &c);
    double v = planar_phi<N>(a, c, s);
    int key = lane;
    wave_argmax(v, key);
    if (v > best) {
      best = v;
      centre = centre + (key - 31.5) * (h / 31.5);
    }
    h = h / 31.5;
  }
  if (lane != 0) return;
  double za, zb;
  sincos(centre, &zb, &za);
  if (za < 0.0 || (za == 0.0 && zb < 0.0)) {
    za = -za;
    zb = -zb;
  }
  qbuf[4 * b] = (float)za;
  qbuf[4 * b + 1] = (float)zb;
  qbuf[4 * b + 2] = 0.0f;
  qbuf[4 * b + 3] = 0.0f;
  lambuf[b] = best;
  flagbuf[b] = 0;
}

// The voxels of the mask box with m(u) != 0, packed as u0 | u1 << 10 | u2 << 20
// (extents <= 512), their mask values and their count.  Order: 4x4x4 bricks
// in C order, the voxels of a brick in C order within it, so that the 64
// lanes of a wave sample a compact region (fewer LDS bank conflicts in the
// rotated gathers).  The order is fixed, so the float sums over it are
// deterministic.  One block.
// squared distance of voxel u from the box centre L / 2 (integer division)
__device__ __forceinline__ int mask_r2(int u0, int u1, int u2, int L0, int L1, int L2) {
  const int d0 = u0 - L0 / 2, d1 = u1 - L1 / 2, d2 = u2 - L2 / 2;
  return d0 * d0 + d1 * d1 + d2 * d2;
}

__global__ void __launch_bounds__(1024) k_mask_list(const float* __restrict__ mask, int L0, int L1, int L2,
                                                    unsigned* __restrict__ list, float* __restrict__ mval,
                                                    int* __restrict__ count) {
  // bricks are handled in chunks of kChunk: one wave per brick (lane j holds
  // voxel j of the brick), the brick counts are scanned across the chunk in
  // LDS, then each wave writes its bricks' voxels
  constexpr int kChunk = 2048;
  __shared__ unsigned long long bits_s[kChunk];
  __shared__ int off_s[kChunk + 1];
  __shared__ int wpart[16];
  __shared__ int base, r2s;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int B0 = (L0 + 3) / 4, B1 = (L1 + 3) / 4, B2 = (L2 + 3) / 4, nB = B0 * B1 * B2;
  const int j0 = lane >> 4, j1 = (lane >> 2) & 3, j2 = lane & 3;
  int r2max = 0;
  if (tid == 0) {
    base = 0;
    r2s = 0;
  }
  // loads in flight per wave: the bricks of a wave are independent, so their
  // mask values are loaded in groups of kLoads before any ballot waits on one
  constexpr int kLoads = 8;
  for (int c0 = 0; c0 < nB; c0 += kChunk) {
    const int nc = min(kChunk, nB - c0);
    for (int i0 = wave; i0 < nc; i0 += 16 * kLoads) {
      float v[kLoads];
#pragma unroll
      for (int j = 0; j < kLoads; ++j) {
        const int i = i0 + 16 * j;
        const int br = c0 + i;
        const int b2 = br % B2, b1 = (br / B2) % B1, b0 = br / (B1 * B2);
        const int u0 = 4 * b0 + j0, u1 = 4 * b1 + j1, u2 = 4 * b2 + j2;
        // an unconditional load (of voxel 0 where out of range), so that the
        // compiler issues the group's loads before it waits
        const bool in = i < nc && u0 < L0 && u1 < L1 && u2 < L2;
        const float m = mask[in ? (u0 * L1 + u1) * L2 + u2 : 0];
        v[j] = in ? m : 0.0f;
      }
#pragma unroll
      for (int j = 0; j < kLoads; ++j) {
        const int i = i0 + 16 * j;
        const unsigned long long bl = __ballot(v[j] != 0.0f);
        if (lane == 0 && i < nc) bits_s[i] = bl;
      }
    }
    __syncthreads();
    // exclusive scan of the brick counts: each thread sums a run of 2 bricks
    const int per = (nc + 1023) / 1024;
    int run = 0;
    for (int k = 0; k < per; ++k) {
      const int i = tid * per + k;
      if (i < nc) run += __popcll(bits_s[i]);
    }
    int incl = run;
    for (int o = 1; o < 64; o <<= 1) {
      const int v = __shfl_up(incl, o);
      if (lane >= o) incl += v;
    }
    if (lane == 63) wpart[wave] = incl;
    __syncthreads();
    int pre = base + incl - run;
    for (int w = 0; w < wave; ++w) pre += wpart[w];
    for (int k = 0; k < per; ++k) {
      const int i = tid * per + k;
      if (i < nc) {
        off_s[i] = pre;
        pre += __popcll(bits_s[i]);
      }
    }
    __syncthreads();
    for (int i0 = wave; i0 < nc; i0 += 16 * kLoads) {
      float v[kLoads];
#pragma unroll
      for (int j = 0; j < kLoads; ++j) {
        const int i = i0 + 16 * j;
        const bool on = i < nc && ((bits_s[i] >> lane) & 1ull);
        const int br = c0 + i;
        const int b2 = br % B2, b1 = (br / B2) % B1, b0 = br / (B1 * B2);
        const int u0 = 4 * b0 + j0, u1 = 4 * b1 + j1, u2 = 4 * b2 + j2;
        const float m = mask[on ? (u0 * L1 + u1) * L2 + u2 : 0];
        v[j] = on ? m : 0.0f;
      }
#pragma unroll
      for (int j = 0; j < kLoads; ++j) {
        const int i = i0 + 16 * j;
        if (i >= nc) continue;
        const unsigned long long bl = bits_s[i];
        if ((bl >> lane) & 1ull) {
          const int br = c0 + i;
          const int b2 = br % B2, b1 = (br / B2) % B1, b0 = br / (B1 * B2);
          const int u0 = 4 * b0 + j0, u1 = 4 * b1 + j1, u2 = 4 * b2 + j2;
          const int o = off_s[i] + __popcll(bl & ((1ull << lane) - 1ull));
          list[o] = (unsigned)u0 | ((unsigned)u1 << 10) | ((unsigned)u2 << 20);
          mval[o] = v[j];
          r2max = max(r2max, mask_r2(u0, u1, u2, L0, L1, L2));
        }
      }
    }
    __syncthreads();
    if (tid == 0) {
      int tot = 0;
      for (int w = 0; w < 16; ++w) tot += wpart[w];
      base += tot;
    }
    __syncthreads();
  }
  atomicMax(&r2s, r2max);
  __syncthreads();
  if (tid == 0) {
    count[0] = base;
    count[1] = r2s;
  }
}

// the same list over the whole chip: one wavefront per brick takes the
// ballot of its voxels with m != 0 ...
__device__ __forceinline__ void mask_bits_block(int blk, const float* __restrict__ mask, int L0, int L1, int L2,
                                                int nB, unsigned long long* __restrict__ bits, int* __restrict__ count) {
  const int lane = threadIdx.x & 63;
  const int br = blk * 4 + (threadIdx.x >> 6);
  if (br == 0 && lane == 0) count[1] = 0;
  if (br >= nB) return;
  const int B1 = (L1 + 3) / 4, B2 = (L2 + 3) / 4;
  const int b2 = br % B2, b1 = (br / B2) % B1, b0 = br / (B1 * B2);
  const int u0 = 4 * b0 + (lane >> 4), u1 = 4 * b1 + ((lane >> 2) & 3), u2 = 4 * b2 + (lane & 3);
  const bool in = u0 < L0 && u1 < L1 && u2 < L2;
  const float m = in ? mask[(u0 * L1 + u1) * L2 + u2] : 0.0f;
  const unsigned long long bl = __ballot(m != 0.0f);
  if (lane == 0) bits[br] = bl;
}
__global__ void __launch_bounds__(256) k_mask_bits(const float* __restrict__ mask, int L0, int L1, int L2, int nB,
                                                   unsigned long long* __restrict__ bits, int* __restrict__ count) {
  mask_bits_block(blockIdx.x, mask, L0, L1, L2, nB, bits, count);
}

// the S^3 seed table and the mask bricks' ballots in one launch: blocks below
// seed_blocks take 256 seeds each, the others four bricks each
__global__ void __launch_bounds__(256) k_pose_tables(int n_seeds, double* __restrict__ seeds, int seed_blocks,
                                                     const float* __restrict__ mask, int L0, int L1, int L2, int nB,
                                                     unsigned long long* __restrict__ bits, int* __restrict__ count) {
  if ((int)blockIdx.x < seed_blocks) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n_seeds) seed_point(i, n_seeds, seeds + 4 * i);
    return;
  }
  mask_bits_block(blockIdx.x - seed_blocks, mask, L0, L1, L2, nB, bits, count);
}

// ... then each block places the voxels of four bricks after the count of
// all earlier bricks (a sum over their ballots)
__global__ void __launch_bounds__(256) k_mask_write(const float* __restrict__ mask, int L0, int L1, int L2, int nB,
                                                    const unsigned long long* __restrict__ bits,
                                                    unsigned* __restrict__ list, float* __restrict__ mval,
                                                    int* __restrict__ count) {
  __shared__ int wsum[4], bc[4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int first = blockIdx.x * 4;
  int acc = 0;
  for (int i = tid; i < first; i += 256) acc += __popcll(bits[i]);
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
  const int br = first + wave;
  const unsigned long long bl = br < nB ? bits[br] : 0ull;
  if (lane == 0) {
    wsum[wave] = acc;
    bc[wave] = __popcll(bl);
  }
  __syncthreads();
  int base = wsum[0] + wsum[1] + wsum[2] + wsum[3];
  for (int w = 0; w < wave; ++w) base += bc[w];
  if (br >= nB) return;
  int r2 = 0;
  if ((bl >> lane) & 1ull) {
    const int B1 = (L1 + 3) / 4, B2 = (L2 + 3) / 4;
    const int b2 = br % B2, b1 = (br / B2) % B1, b0 = br / (B1 * B2);
    const int u0 = 4 * b0 + (lane >> 4), u1 = 4 * b1 + ((lane >> 2) & 3), u2 = 4 * b2 + (lane & 3);
    const int o = base + __popcll(bl & ((1ull << lane) - 1ull));
    list[o] = (unsigned)u0 | ((unsigned)u1 << 10) | ((unsigned)u2 << 20);
    mval[o] = mask[(u0 * L1 + u1) * L2 + u2];
    r2 = mask_r2(u0, u1, u2, L0, L1, L2);
  }
  for (int off = 32; off > 0; off >>= 1) r2 = max(r2, __shfl_xor(r2, off));
  if (lane == 0 && bl != 0ull) atomicMax(count + 1, r2);
  if (br == nB - 1 && lane == 0) count[0] = base + bc[wave];
}

hipError_t launch_mask_list(const float* mask, int L0, int L1, int L2, unsigned* list, float* mval, int* count,
                            hipStream_t s, unsigned long long* bits) {
  const long nB = mask_bricks(L0, L1, L2);
  if (bits && nB <= kMaskFastBricks) {
    const unsigned nblk = (unsigned)((nB + 3) / 4);
    hipLaunchKernelGGL(k_mask_bits, dim3(nblk), dim3(256), 0, s, mask, L0, L1, L2, (int)nB, bits, count);
    hipLaunchKernelGGL(k_mask_write, dim3(nblk), dim3(256), 0, s, mask, L0, L1, L2, (int)nB, bits, list, mval,
                       count);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_mask_list, dim3(1), dim3(1024), 0, s, mask, L0, L1, L2, list, mval, count);
  return hipGetLastError();
}

// ----------------------------------------------------------------------------
// the pick of each candidate's neighbour
// ----------------------------------------------------------------------------
struct PickArgs {
  const float* score;
  int K, NB;
  const int* pos_in;
  const double* C;
  const double* w;
  const float* q;
  const double* lam;
  const double* key;
  const int* flags;
  int* out_pos;
  float* out_quat;
  double* out_lambda;
  float* out_score;
  int* out_flags;
  double* out_C;
  const int* active;
  int* moved;
};

// Per candidate, one wavefront: the neighbour with the largest key (lambda
// for refine 1, the NCC at its own rotation for refine 2), the centre first
// on ties, then the lower neighbour index; lane 0 writes the scalars to the
// candidate's row, the lanes copy the picked tensor together.  moved (if
// given) records whether the candidate left its position; a candidate that
// active (if given) marks as settled is left as it is, with moved 0.
__global__ void __launch_bounds__(64) k_pose_pick(PoseGeo g, PickArgs a, const int* __restrict__ count_dev,
                                                  int count_host) {
  __shared__ double keys[27];
  __shared__ int pickv;
  const int p = blockIdx.x;
  const int count = count_dev ? count_dev[0] : count_host;
  if (p >= count) return;
  const int lane = threadIdx.x;
  if (a.active && !a.active[p]) {
    if (lane == 0 && a.moved) a.moved[p] = 0;
    return;
  }
  const int NB = a.NB;
  if (lane < NB) keys[lane] = a.key[(long)p * NB + lane];
  __syncthreads();
  if (lane == 0) {
    const int centre = NB == 27 ? 13 : 0;
    int bk = centre;
    double bv = keys[centre];
    for (int k = 0; k < NB; ++k)
      if (keys[k] > bv) {
        bv = keys[k];
        bk = k;
      }
    pickv = bk;
    const long b = (long)p * NB + bk;
    int o0, o1, o2;
    neighbour_offset(bk, NB, o0, o1, o2);
    const int x0 = a.pos_in[3 * p] + o0, x1 = a.pos_in[3 * p + 1] + o1, x2 = a.pos_in[3 * p + 2] + o2;
    a.out_pos[3 * p] = x0;
    a.out_pos[3 * p + 1] = x1;
    a.out_pos[3 * p + 2] = x2;
    for (int d = 0; d < 4; ++d) a.out_quat[4 * p + d] = a.q[4 * b + d];
    a.out_lambda[p] = a.lam[b];
    int flags = a.flags[b];
    if (!(a.w[b] > 0.0)) flags |= TTM_POSE_ZERO_NORM;
    a.out_flags[p] = flags;
    if (a.out_score) a.out_score[p] = a.score ? a.score[((long)x0 * g.n1 + x1) * g.n2 + x2] : 0.0f;
    if (a.moved) a.moved[p] = bk != centre ? 1 : 0;
  }
  if (a.out_C) {
    __syncthreads();
    const long b = (long)p * NB + pickv;
    for (int k = lane; k < a.K; k += 64) a.out_C[(long)p * a.K + k] = a.C[b * a.K + k];
  }
}

// c(y, R(q_y)) = w(y) <tau_y f, s_R> for the rotation q_y found at voxel y
// (Section 2, the normalised correlation of Algorithm 1, with s_R the raw
// template rotated by R and normalised under the mask):
//   <tau_y f, s_R> = (sum m g f - mu sum m f) / sqrt(sum m g^2 - mu sum m g),
//   g = t_R sampled trilinearly (zero outside the box), mu = sum m g / sum m,
//   f the image window.
// Per-thread partial sums in float32 over the compacted mask voxels, the block
// reduction and the normalisation in float64.  -inf outside the valid region;
// 0 where w(y) = 0 or the rotated template has no masked variance.
// k_pose_ncc takes one block per (candidate, neighbour); ncc_one is the NCC of neighbour k of candidate p
// (its w > 0, its window in the image) by the block's 256 threads, written to
// *out by thread 0.
__device__ void ncc_one(const PoseGeo& g, const float* __restrict__ image, const float* __restrict__ tmpl,
                        const unsigned* __restrict__ mlist, const float* __restrict__ mval,
                        const int* __restrict__ mcount, const int* __restrict__ pos, int p, int k, int NB, double w,
                        const float* __restrict__ q4, double* __restrict__ out) {
  __shared__ double red[4][5];
  const int tid = threadIdx.x;
  int o0, o1, o2;
  neighbour_offset(k, NB, o0, o1, o2);
  const int x0 = pos[3 * p] + o0, x1 = pos[3 * p + 1] + o1, x2 = pos[3 * p + 2] + o2;
  const int L0 = g.L0, L1 = g.L1, L2 = g.L2;
  const int c0 = L0 / 2, c1 = L1 / 2, c2 = L2 / 2;
  // okbuf: the window lies inside the image (valid region), no wrap needed
  const float* __restrict__ base = image + ((long)(x0 - c0) * g.n1 + (x1 - c1)) * g.n2 + (x2 - c2);
  const int rs1 = g.n2, rs0 = g.n1 * g.n2;       // window strides (< 2^31 elements)
  const Rot R = quat_rot(q4);
  const int nm = mcount[0];
  float v0 = 0.0f, v1 = 0.0f, v2 = 0.0f, v3 = 0.0f, v4 = 0.0f;   // m, m g, m g^2, m f, m g f
  for (int i = tid; i < nm; i += 256) {
    const unsigned pk = mlist[i];
    const int u0 = (int)(pk & 1023u), u1 = (int)((pk >> 10) & 1023u), u2 = (int)(pk >> 20);
    const float mv = mval[i];
    const float gv = sample_rotated(tmpl, L0, L1, L2, R, u0, u1, u2);
    const float fv = base[u0 * rs0 + u1 * rs1 + u2];
    const float mg = mv * gv;
    v0 += mv;
    v1 += mg;
    v2 += mg * gv;
    v3 += mv * fv;
    v4 += mg * fv;
  }
  double v[5] = {v0, v1, v2, v3, v4};
#pragma unroll
  for (int i = 0; i < 5; ++i)
    for (int off = 32; off > 0; off >>= 1) v[i] += __shfl_xor(v[i], off);
  const int lane = tid & 63, wave = tid >> 6;
  if (lane == 0)
#pragma unroll
    for (int i = 0; i < 5; ++i) red[wave][i] = v[i];
  __syncthreads();
  if (tid == 0) {
    double t[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) t[i] = red[0][i] + red[1][i] + red[2][i] + red[3][i];
    const double mu = t[0] > 0.0 ? t[1] / t[0] : 0.0;
    const double var = t[2] - mu * t[1];
    *out = var > 1e-6 * (t[2] > 0.0 ? t[2] : 1.0) ? w * (t[4] - mu * t[3]) / sqrt(var) : 0.0;
  }
}

__global__ void __launch_bounds__(256) k_pose_ncc(PoseGeo g, const float* __restrict__ image,
                                                  const float* __restrict__ tmpl, const unsigned* __restrict__ mlist,
                                                  const float* __restrict__ mval,
                                                  const int* __restrict__ mcount, const int* __restrict__ pos,
                                                  const int* __restrict__ count_dev, int count_host, int NB,
                                                  const double* __restrict__ wbuf, const int* __restrict__ okbuf,
                                                  const float* __restrict__ qbuf, double* __restrict__ nccbuf,
                                                  const int* __restrict__ active) {
  const int b = blockIdx.x;
  const int p = b / NB, k = b % NB;
  const int count = count_dev ? count_dev[0] : count_host;
  if (p >= count || (active && !active[p])) return;
  const int tid = threadIdx.x;
  if (!okbuf[b]) {
    if (tid == 0) nccbuf[b] = -INFINITY;
  } else if (!(wbuf[b] > 0.0)) {
    if (tid == 0) nccbuf[b] = 0.0;
  } else {
    ncc_one(g, image, tmpl, mlist, mval, mcount, pos, p, k, NB, wbuf[b], qbuf + 4 * (long)b, nccbuf + b);
  }
}

// The same NCC with the template held in LDS: one block of NT threads per
// (candidate, group of its neighbours) loads the template once and
// evaluates the group's neighbours one after another, sampling trilinearly
// from LDS (the padded, zero-guarded layout of sample_rotated_lds: its
// pitches spread a wave's gathers over the banks, and with the 4x4x4 brick
// order of the mask voxels a wave samples a compact region).  The layout must
// fit CAP floats.  Every box whose padded layout fits kNccLdsSmall floats
// (the depth-1 boxes of a planar stack, and volumes up to about 13^3) takes
// 256 threads and that much LDS, four blocks per CU at
// its register use: such a window holds too few mask voxels to occupy 1024
// threads, and with the large LDS reservation its blocks would run one per
// CU.  Larger boxes take 1024 threads and CAP = kNccLdsCap (one block per
// CU).
constexpr int kNccLdsSmall = 4096;
template <int NT, int CAP>
__global__ void __launch_bounds__(NT, 1024 / NT) k_pose_ncc_lds(PoseGeo g, int ngroups, const float* __restrict__ image,
                                                       const float* __restrict__ tmpl,
                                                       const unsigned* __restrict__ mlist,
                                                       const float* __restrict__ mval,
                                                       const int* __restrict__ mcount, const int* __restrict__ pos,
                                                       const int* __restrict__ count_dev, int count_host,
                                                       const double* __restrict__ wbuf,
                                                       const int* __restrict__ okbuf, const float* __restrict__ qbuf,
                                                       double* __restrict__ nccbuf,
                                                       const int* __restrict__ active) {
  constexpr int NW = NT / 64;
  __shared__ float tl[CAP];
  __shared__ double red[NW][15];
  constexpr int NB = 27;
  const int p = blockIdx.x / ngroups, grp = blockIdx.x % ngroups;
  const int gsize = (NB + ngroups - 1) / ngroups;
  const int k_lo = grp * gsize, k_hi = min(NB, k_lo + gsize);
  const int count = count_dev ? count_dev[0] : count_host;
  if (p >= count || (active && !active[p])) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int L0 = g.L0, L1 = g.L1, L2 = g.L2, nL = L0 * L1 * L2;
  const int P2 = ncc_lds_p2(L2), P01 = ncc_lds_p01(L1, L2);
  fill_lds_box(tl, tmpl, L0, L1, L2, P2, P01, tid, NT);
  __syncthreads();
  const int c0 = L0 / 2, c1 = L1 / 2, c2 = L2 / 2;
  const int rs1 = g.n2, rs0 = g.n1 * g.n2;
  const int nm = mcount[0];
  // mcount[1]: the largest squared distance of a mask voxel from the centre;
  // below the squared inscribed radius min(L / 2) every rotated sample point
  // lies inside [0, L) on every axis (with a margin of at least 1 / L voxel,
  // far above the float error of the rotated coordinates)
  const int cmin = min(L0 / 2, min(L1 / 2, L2 / 2));
  const bool inner = mcount[1] < cmin * cmin;
  // the block's neighbours in passes of up to kNccPass: one pass over the
  // mask voxels loads each list entry once and samples it under every live
  // neighbour's rotation (each neighbour's sums keep the voxel order of a
  // pass of its own)
  constexpr int kNccPass = 3;
  constexpr int kNccLoads = 4;
  for (int k0 = k_lo; k0 < k_hi; k0 += kNccPass) {
    bool live[kNccPass];
    double wk[kNccPass];
    const float* bases[kNccPass];
    Rot R[kNccPass];
    bool any = false;
#pragma unroll
    for (int j = 0; j < kNccPass; ++j) {
      const int k = k0 + j;
      live[j] = false;
      wk[j] = 0.0;
      bases[j] = image;
      for (int i = 0; i < 9; ++i) R[j].r[i] = 0.0f;
      if (k >= k_hi) continue;
      // block-uniform: the neighbour's validity and w
      const long b = (long)p * NB + k;
      if (!okbuf[b]) {
        if (tid == 0) nccbuf[b] = -INFINITY;
        continue;
      }
      const double w = wbuf[b];
      if (!(w > 0.0)) {
        if (tid == 0) nccbuf[b] = 0.0;
        continue;
      }
      int o0, o1, o2;
      neighbour_offset(k, NB, o0, o1, o2);
      const int x0 = pos[3 * p] + o0, x1 = pos[3 * p + 1] + o1, x2 = pos[3 * p + 2] + o2;
      bases[j] = image + ((long)(x0 - c0) * g.n1 + (x1 - c1)) * g.n2 + (x2 - c2);
      const Rot Rj = quat_rot(qbuf + 4 * b);
      // the same matrix in every lane: kept in scalar registers
#pragma unroll
      for (int i = 0; i < 9; ++i)
        R[j].r[i] = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(Rj.r[i])));
      wk[j] = w;
      live[j] = true;
      any = true;
    }
    if (!any) continue;
    float v[kNccPass][5];
#pragma unroll
    for (int j = 0; j < kNccPass; ++j)
#pragma unroll
      for (int i = 0; i < 5; ++i) v[j][i] = 0.0f;
    // kNccLoads of a thread's mask voxels at a time: their list entries, then
    // their image values, are loaded before any sample waits on them.  Past
    // the list's end a slot holds voxel 0 with weight 0 and adds nothing, so
    // each thread's sums are those of the plain loop over its voxels.  INNER:
    // every mask voxel lies in the box's inscribed ball, so every sample
    // takes the sampler's fast path and the test is left out.
    auto pass = [&](auto inner_tag) {
      constexpr bool INNER = decltype(inner_tag)::value;
      for (int i0 = tid; i0 < nm; i0 += NT * kNccLoads) {
        unsigned pk[kNccLoads];
        float mv[kNccLoads], fv[kNccPass][kNccLoads];
#pragma unroll
        for (int jj = 0; jj < kNccLoads; ++jj) {
          const int i = i0 + NT * jj;
          pk[jj] = i < nm ? mlist[i] : 0u;
          mv[jj] = i < nm ? mval[i] : 0.0f;
        }
#pragma unroll
        for (int jj = 0; jj < kNccLoads; ++jj) {
          const int u0 = (int)(pk[jj] & 1023u), u1 = (int)((pk[jj] >> 10) & 1023u), u2 = (int)(pk[jj] >> 20);
          // the voxel's offset in every neighbour's window
          const int off = u0 * rs0 + u1 * rs1 + u2;
#pragma unroll
          for (int j = 0; j < kNccPass; ++j) fv[j][jj] = live[j] ? bases[j][off] : 0.0f;
        }
#pragma unroll
        for (int jj = 0; jj < kNccLoads; ++jj) {
          const int u0 = (int)(pk[jj] & 1023u), u1 = (int)((pk[jj] >> 10) & 1023u), u2 = (int)(pk[jj] >> 20);
#pragma unroll
          for (int j = 0; j < kNccPass; ++j) {
            if (!live[j]) continue;
            const float gv = INNER ? sample_rotated_lds_inner(tl, L0, L1, L2, P2, P01, R[j], u0, u1, u2)
                                   : sample_rotated_lds(tl, L0, L1, L2, P2, P01, R[j], u0, u1, u2);
            const float mg = mv[jj] * gv;
            v[j][0] += mv[jj];
            v[j][1] += mg;
            v[j][2] += mg * gv;
            v[j][3] += mv[jj] * fv[j][jj];
            v[j][4] += mg * fv[j][jj];
          }
        }
      }
    };
    if (inner)
      pass(std::true_type{});
    else
      pass(std::false_type{});
#pragma unroll
    for (int j = 0; j < kNccPass; ++j) {
      if (!live[j]) continue;
      double d[5] = {v[j][0], v[j][1], v[j][2], v[j][3], v[j][4]};
#pragma unroll
      for (int i = 0; i < 5; ++i)
        for (int off = 32; off > 0; off >>= 1) d[i] += __shfl_xor(d[i], off);
      if (lane == 0)
#pragma unroll
        for (int i = 0; i < 5; ++i) red[wave][j * 5 + i] = d[i];
    }
    __syncthreads();
    if (tid == 0) {
#pragma unroll
      for (int j = 0; j < kNccPass; ++j) {
        if (!live[j]) continue;
        double t[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
        for (int wv = 0; wv < NW; ++wv)
#pragma unroll
          for (int i = 0; i < 5; ++i) t[i] += red[wv][j * 5 + i];
        const double mu = t[0] > 0.0 ? t[1] / t[0] : 0.0;
        const double var = t[2] - mu * t[1];
        nccbuf[(long)p * NB + k0 + j] = var > 1e-6 * (t[2] > 0.0 ? t[2] : 1.0) ? wk[j] * (t[4] - mu * t[3]) / sqrt(var)
                                                                              : 0.0;
      }
    }
    __syncthreads();
  }
}

static PoseGeo make_posegeo(const Geo& gg) {
  PoseGeo g;
  g.n0 = gg.n0; g.n1 = gg.n1; g.n2 = gg.n2;
  g.L0 = gg.L0; g.L1 = gg.L1; g.L2 = gg.L2;
  g.lo0 = gg.c0; g.hi0 = gg.n0 - gg.L0 + gg.c0;
  g.lo1 = gg.c1; g.hi1 = gg.n1 - gg.L1 + gg.c1;
  g.lo2 = gg.c2; g.hi2 = gg.n2 - gg.L2 + gg.c2;
  g.planar = gg.planar;
  return g;
}

hipError_t launch_pose_tensor(const Geo& gg, const float* image, const float* comps, const float* mask,
                              int order_n, const double* img_stats, float eps_v, int max_peaks, int refine,
                              const int* pos_in, const int* count_dev, int count_host, const PoseScratch& ps,
                              hipStream_t s) {
  const PoseGeo g = make_posegeo(gg);
  const int K = num_components(order_n);
  const int NB = refine ? 27 : 1;
  if (!g.planar) {
    const int ngroups = (K + kDirGroup - 1) / kDirGroup;
    if (refine)
      hipLaunchKernelGGL(k_pose_direct<3>, dim3((unsigned)max_peaks, 3, (unsigned)(ngroups + 1)), dim3(kDirThreads),
                         0, s, g, image, comps, mask, K, pos_in, count_dev, count_host, ps.C, ps.mom, ps.active);
    else
      hipLaunchKernelGGL(k_pose_direct<1>, dim3((unsigned)max_peaks, 1, (unsigned)(ngroups + 1)), dim3(kDirThreads),
                         0, s, g, image, comps, mask, K, pos_in, count_dev, count_host, ps.C, ps.mom, ps.active);
    const int total = max_peaks * NB;
    hipLaunchKernelGGL(k_pose_direct_finish, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, g, K, img_stats,
                       eps_v, pos_in, count_dev, count_host, NB, total, ps.mom, ps.C, ps.w, ps.ok, ps.active);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_pose_tensor, dim3((unsigned)(max_peaks * NB)), dim3(256), 0, s, g, image, comps, mask, K,
                     img_stats, eps_v, pos_in, count_dev, count_host, NB, ps.C, ps.w, ps.ok, ps.active);
  return hipGetLastError();
}

hipError_t launch_pose_solve(const Geo& gg, const float* score, int order_n, int n_seeds, int max_iter,
                             double tol, int max_peaks, int refine, const int* pos_in, const int* count_dev,
                             int count_host, const float* image, const float* tmpl, const float* mask,
                             int* out_pos, float* out_quat, double* out_lambda, float* out_score, int* out_flags,
                             double* out_C, const PoseScratch& ps, hipStream_t s, bool reuse_tables,
                             int ncc_groups, int* moved) {
  const PoseGeo g = make_posegeo(gg);
  const int K = num_components(order_n);
  const int NB = refine ? 27 : 1;
  // the mask list's first kernel (the bricks' ballots) joins the seed table's
  // launch where both are built here
  const long nB = mask_bricks(g.L0, g.L1, g.L2);
  const bool tables = !reuse_tables && !g.planar && refine == 2 && ps.mbits && nB <= kMaskFastBricks;
  const int seed_blocks = (n_seeds + 255) / 256;
  if (tables)
    hipLaunchKernelGGL(k_pose_tables, dim3((unsigned)(seed_blocks + (nB + 3) / 4)), dim3(256), 0, s, n_seeds,
                       ps.seeds, seed_blocks, mask, g.L0, g.L1, g.L2, (int)nB, ps.mbits, ps.mcount);
  else if (!reuse_tables && !g.planar)
    hipLaunchKernelGGL(k_seed_table, dim3((unsigned)seed_blocks), dim3(256), 0, s, n_seeds, ps.seeds);
  const dim3 eg((unsigned)(max_peaks * NB));
  if (g.planar) {
    switch (order_n) {
      case 2:
        hipLaunchKernelGGL(k_planar_eig<2>, eg, dim3(64), 0, s, ps.C, ps.ok, count_dev, count_host, NB, ps.q,
                           ps.lam, ps.flags, ps.active);
        break;
      case 4:
        hipLaunchKernelGGL(k_planar_eig<4>, eg, dim3(64), 0, s, ps.C, ps.ok, count_dev, count_host, NB, ps.q,
                           ps.lam, ps.flags, ps.active);
        break;
      case 6:
        hipLaunchKernelGGL(k_planar_eig<6>, eg, dim3(64), 0, s, ps.C, ps.ok, count_dev, count_host, NB, ps.q,
                           ps.lam, ps.flags, ps.active);
        break;
      case 8:
        hipLaunchKernelGGL(k_planar_eig<8>, eg, dim3(64), 0, s, ps.C, ps.ok, count_dev, count_host, NB, ps.q,
                           ps.lam, ps.flags, ps.active);
        break;
      default: return hipErrorInvalidValue;
    }
  } else switch (order_n) {
    case 2:
      hipLaunchKernelGGL(k_pose_eig<2>, eg, dim3(256), 0, s, ps.seeds, ps.C, ps.ok, count_dev, count_host, NB,
                         n_seeds, max_iter, tol, ps.q, ps.lam, ps.flags, ps.active);
      break;
    case 4:
      hipLaunchKernelGGL(k_pose_eig<4>, eg, dim3(256), 0, s, ps.seeds, ps.C, ps.ok, count_dev, count_host, NB,
                         n_seeds, max_iter, tol, ps.q, ps.lam, ps.flags, ps.active);
      break;
    case 6:
      hipLaunchKernelGGL(k_pose_eig<6>, eg, dim3(256), 0, s, ps.seeds, ps.C, ps.ok, count_dev, count_host, NB,
                         n_seeds, max_iter, tol, ps.q, ps.lam, ps.flags, ps.active);
      break;
    case 8:
      hipLaunchKernelGGL(k_pose_eig<8>, eg, dim3(256), 0, s, ps.seeds, ps.C, ps.ok, count_dev, count_host, NB,
                         n_seeds, max_iter, tol, ps.q, ps.lam, ps.flags, ps.active);
      break;
    default: return hipErrorInvalidValue;
  }
  if (refine == 2) {
    if (tables)
      hipLaunchKernelGGL(k_mask_write, dim3((unsigned)((nB + 3) / 4)), dim3(256), 0, s, mask, g.L0, g.L1, g.L2,
                         (int)nB, ps.mbits, ps.mlist, ps.mval, ps.mcount);
    else if (!reuse_tables)
      (void)launch_mask_list(mask, g.L0, g.L1, g.L2, ps.mlist, ps.mval, ps.mcount, s, ps.mbits);
    const long lds = ncc_lds_floats(g.L0, g.L1, g.L2);
    const int ngroups = ncc_groups;
    if (lds <= kNccLdsSmall) {
      // small boxes: 256 threads and 16 KiB of LDS per block
      hipLaunchKernelGGL((k_pose_ncc_lds<256, kNccLdsSmall>), dim3((unsigned)(max_peaks * ngroups)), dim3(256), 0, s,
                         g, ngroups, image, tmpl, ps.mlist, ps.mval, ps.mcount, pos_in, count_dev, count_host, ps.w,
                         ps.ok, ps.q, ps.ncc, ps.active);
    } else if (lds <= kNccLdsCap) {
      // one block per CU (the template fills most of the LDS); each block
      // loads the template once for 27 / ngroups neighbours of a candidate
      hipLaunchKernelGGL((k_pose_ncc_lds<1024, kNccLdsCap>), dim3((unsigned)(max_peaks * ngroups)), dim3(1024), 0,
                         s, g, ngroups, image, tmpl, ps.mlist, ps.mval, ps.mcount, pos_in, count_dev, count_host,
                         ps.w, ps.ok, ps.q, ps.ncc, ps.active);
    } else {
      hipLaunchKernelGGL(k_pose_ncc, eg, dim3(256), 0, s, g, image, tmpl, ps.mlist, ps.mval, ps.mcount, pos_in,
                         count_dev, count_host, NB, ps.w, ps.ok, ps.q, ps.ncc, ps.active);
    }
  }
  PickArgs pa;
  pa.score = score;
  pa.K = K;
  pa.NB = NB;
  pa.pos_in = pos_in;
  pa.C = ps.C;
  pa.w = ps.w;
  pa.q = ps.q;
  pa.lam = ps.lam;
  pa.key = refine == 2 ? ps.ncc : ps.lam;
  pa.flags = ps.flags;
  pa.out_pos = out_pos;
  pa.out_quat = out_quat;
  pa.out_lambda = out_lambda;
  pa.out_score = out_score;
  pa.out_flags = out_flags;
  pa.out_C = out_C;
  pa.active = ps.active;
  pa.moved = moved;
  hipLaunchKernelGGL(k_pose_pick, dim3((unsigned)max_peaks), dim3(64), 0, s, g, pa, count_dev, count_host);
  return hipGetLastError();
}

}  // namespace ttm
