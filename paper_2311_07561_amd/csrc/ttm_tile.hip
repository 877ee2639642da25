// Overlap-save tiling: images of any extent are correlated on cubic tiles of
// a power-of-two edge T.  A tile at origin o holds image[o + t] (zero beyond
// the image); the correlation of the tile is exact at the tile's valid
// positions t in [c, c + T - L] per axis (the window lies inside the tile),
// and tiles step by T - L + 1 so that these positions partition the image's
// valid region.  Positions whose window leaves the image are dropped.
#include "ttm_internal.h"

namespace ttm {

// tile[t0][t1][t2] = image[o + t] inside the image, 0 outside; one block per
// tile row (t0, t1)
__global__ void __launch_bounds__(256) k_tile_gather(const float* __restrict__ image, TileGeo g,
                                                     float* __restrict__ tile) {
  const int row = blockIdx.x;
  const int t0 = row / g.T, t1 = row % g.T;
  const int y0 = g.o0 + t0, y1 = g.o1 + t1;
  const bool in = y0 < g.n0 && y1 < g.n1;
  const float* __restrict__ src = image + ((long)y0 * g.n1 + y1) * g.n2 + g.o2;
  float* __restrict__ dst = tile + (long)row * g.T;
  const int lim = in ? min(g.T, g.n2 - g.o2) : 0;
  for (int t2 = threadIdx.x; t2 < g.T; t2 += blockDim.x) dst[t2] = t2 < lim ? src[t2] : 0.0f;
}

// the tile's valid positions that are valid positions of the image: score
// (and w) copied to the image's maps; one block per valid tile row
__global__ void __launch_bounds__(256) k_tile_scatter(const float* __restrict__ tscore, const float* __restrict__ tw,
                                                      TileGeo g, float* __restrict__ score, float* __restrict__ w) {
  const int W1 = g.T - g.L1 + 1, W2 = g.T - g.L2 + 1;
  const int r = blockIdx.x;
  const int t0 = g.c0 + r / W1, t1 = g.c1 + r % W1;
  const int x0 = g.o0 + t0, x1 = g.o1 + t1;
  if (x0 > g.n0 - g.L0 + g.c0 || x1 > g.n1 - g.L1 + g.c1) return;
  const int x2lim = g.n2 - g.L2 + g.c2 - g.o2;            // tile coordinate of the last valid image column
  const long ts = ((long)t0 * g.T + t1) * g.T;
  const long is = ((long)x0 * g.n1 + x1) * g.n2 + g.o2;
  for (int i = threadIdx.x; i < W2; i += blockDim.x) {
    const int t2 = g.c2 + i;
    if (t2 > x2lim) break;
    score[is + t2] = tscore[ts + t2];
    if (w) w[is + t2] = tw[ts + t2];
  }
}

hipError_t launch_tile_gather(const float* image, const TileGeo& g, float* tile, hipStream_t s) {
  hipLaunchKernelGGL(k_tile_gather, dim3((unsigned)(g.T * g.T)), dim3(g.T < 256 ? g.T : 256), 0, s, image, g,
                     tile);
  return hipGetLastError();
}

hipError_t launch_tile_scatter(const float* tscore, const float* tw, const TileGeo& g, float* score, float* w,
                               hipStream_t s) {
  const int W0 = g.T - g.L0 + 1, W1 = g.T - g.L1 + 1, W2 = g.T - g.L2 + 1;
  hipLaunchKernelGGL(k_tile_scatter, dim3((unsigned)(W0 * W1)), dim3(W2 < 256 ? W2 : 256), 0, s, tscore, tw, g,
                     score, w);
  return hipGetLastError();
}

}  // namespace ttm
