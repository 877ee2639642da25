// Host-side internal interface between the libttm translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "ttm.h"

namespace ttm {

constexpr int kMaxOrder = 8;
constexpr int kMaxK = 165;          // C(8+3, 3)

inline int num_components(int n) { return (n + 1) * (n + 2) * (n + 3) / 6; }
inline bool supported_len(int n) { return n >= 16 && n <= 512 && (n & (n - 1)) == 0; }

// Reduction modes of the last inverse pass (axis-2 C2R).
// P3_FIELD: w (as P3_W) and C_alpha(x) = w(x) G_alpha(x) per component
enum Pass3Mode { P3_SCORE = 0, P3_W = 1, P3_MAX = 2, P3_FIELD = 3 };

struct Geo {
  int n0, n1, n2;      // image extents
  int h2;              // n2 / 2 + 1 columns of a half spectrum
  int p2;              // row pitch of a half spectrum (= h2, unpadded: a
                       // plane of n1 rows is a whole number of 128-byte
                       // lines, so axis-0 tiles of 16 pencils are aligned;
                       // axis-1 tiles straddle lines shared with the next
                       // tile, which the XCD-aware tile order keeps in one L2)
  int L0, L1, L2;      // template extents
  int c0, c1, c2;      // template centre (L / 2)
  int planar = 0;      // a stack of planes: the pose neighbourhood stays in each plane
  long vol() const { return (long)n0 * n1 * n2; }
  long half() const { return (long)n0 * n1 * p2; }     // complex elements of a half spectrum
  long bank_slab() const { return (long)L0 * n1 * p2; } // complex elements per bank entry
  // valid region (window inside the image), inclusive bounds per axis
  int lo0() const { return c0; }
  int hi0() const { return n0 - L0 + c0; }
  int lo1() const { return c1; }
  int hi1() const { return n1 - L1 + c1; }
};
__host__ __device__ constexpr int row_pitch(int n2) { return n2 / 2 + 1; }

// --- FFT passes (ttm_fft.hip) -------------------------------------------------
// image moments in float64: stats[0] = mean, stats[1] = population variance
// and, if mask is given, stats[2] = m_sum over its nm values; partials holds
// 3 * kStatPartials doubles.  mu (optional): the multiplicities of order
// mu_order (as launch_multiplicities), written by the same launches.
constexpr int kStatPartials = 512;
hipError_t launch_image_stats(const float* img, long n, const float* mask, long nm, double* partials,
                              double* stats, hipStream_t s, int mu_order = 0, float* mu = nullptr);
// axis-2 R2C of rows.  mode 0: src rows (len_valid <= n2 values, rest zero)
// -> dst0; mode 1: image rows, (f - mean) -> dst0 and (f - mean)^2 -> dst1.
// dst row of source row r: (r / grp) * grp_stride + r % grp (rows of h2).
hipError_t launch_r2c_rows(int n2, const float* src, long src_stride, int len_valid, long nrows,
                           float2* dst0, float2* dst1, long grp, long grp_stride, int mode,
                           const double* stats, hipStream_t s);   // rows of pitch row_pitch(n2)
// strided pencil FFT along one axis, in place: pencil p has base
// (p / Q) * S_outer + p % Q and element j at base + j * S_axis; only j < nin
// is read (the rest is zero); output index j goes to position
// x = (j + shift) mod N, and is stored only if slo <= x <= shi.  Pencils in
// the row padding are transformed too (they hold no data and are never read
// as data).  blockIdx.y walks nbatch arrays batch_stride apart.
hipError_t launch_pencils(int N, bool inverse, float2* data, long npencils, long Q, long S_outer, long S_axis,
                          int nin, int shift, int slo, int shi, int nbatch, long batch_stride, hipStream_t s);
// first inverse pass, fused: forward axis-0 FFT of the image pencils in src0,
// then for each of nt0 template entries from tmpl0 (bank layout
// [L0][n1][p2], tmpl_stride apart): pruned forward axis-0 FFT, product with
// conj, inverse axis-0 FFT, store into out + i * out_stride with the centre
// shift; then the same for src1 with nt1 entries from tmpl1 (outputs
// nt0 .. nt0 + nt1 - 1).  Only the planes x0 of the valid region are stored.
struct Pass1Args {
  const float2* src0;
  const float2* tmpl0;
  int nt0;
  const float2* src1;
  const float2* tmpl1;
  int nt1;
  long tmpl_stride;
  float2* out;
  long out_stride;
};
hipError_t launch_pass1(const Geo& g, const Pass1Args& a, hipStream_t s);
// the two-pass inverse (axes 1 and 2 of 256): pass A writes the arrays as
// Z[x0][ja][kb][k2] (axis 0 and the 4-point digit of axis 1 done), pass B
// reduces them to the score and w (P3_SCORE only)
bool two_pass_supported(const Geo& g);
hipError_t launch_pass1x(const Geo& g, const Pass1Args& a, hipStream_t s);
// last inverse pass (axis-2 C2R) fused with the per-voxel reduction.  Only
// rows (x0, x1) of the valid region are read; outputs outside it are zero
// (P3_SCORE, P3_W) or left untouched (P3_MAX).
struct Pass3Args {
  const float2* H;     // pair arrays [n0][n1][h2]
  long pstride;        // complex elements between pair arrays
  int npairs;          // arrays to reduce (components / rotations)
  int mode;            // Pass3Mode
  const float* mu;     // P3_SCORE: multiplicities (npairs)
  const double* stats; // [0] mean [1] var(f); msum at stats[2]
  float eps_v;
  float* out_score;    // P3_SCORE
  float* out_w;        // P3_SCORE (optional) / P3_W
  float* best;         // P3_MAX running maximum of G (unscaled)
  int* best_idx;       // P3_MAX
  int first_index;     // P3_MAX index of pair 0
  int init;            // P3_MAX: 1 = first batch (ignore best/best_idx contents)
  float* out_C;        // P3_FIELD: planes [npairs][W0][W1][W2] over the valid box
  long c_plane;        // P3_FIELD: W0 W1 W2
};
hipError_t launch_pass3(const Geo& g, const Pass3Args& a, hipStream_t s);
hipError_t launch_pass3x(const Geo& g, const Pass3Args& a, hipStream_t s);
// classical epilogue: ncc = best * w / V inside the valid region where w > 0
hipError_t launch_classical_final(const Geo& g, const float* w, float* best, int* idx,
                                  hipStream_t s);
hipError_t launch_fill_f32(float* p, long n, float v, hipStream_t s);
hipError_t launch_fill_i32(int* p, long n, int v, hipStream_t s);

// --- template build (ttm_build.hip) -------------------------------------------
// per-rotation masked statistics of the rotated raw template:
// stats[j] = (mean_j, scale_j) with scale = 1/sqrt(masked variance) (0 if none)
hipError_t launch_rot_stats(const float* tmpl, const float* mask, int L0, int L1, int L2,
                            const float* quats, int nrot, double* rstats, hipStream_t s);
// coef[j*K + alpha] = omega_j * Q_j^alpha * scale_j
hipError_t launch_build_coef(const float* quats, const double* weights, const double* rstats,
                             int nrot, int order_n, double* coef, hipStream_t s);
// components[alpha][u] = sum_j coef[j][alpha] * m(u) (g_j(u) - mean_j)
hipError_t launch_build_accum(const float* tmpl, const float* mask, int L0, int L1, int L2,
                              const float* quats, const double* rstats, const double* coef,
                              int nrot, int K, float* comps, float* rtab, hipStream_t s);
// normalised rotated templates s_j for j in [j0, j0+nb) -> out[nb][L0][L1][L2]
hipError_t launch_rot_write(const float* tmpl, const float* mask, int L0, int L1, int L2,
                            const float* quats, const double* rstats, int j0, int nb,
                            float* out, hipStream_t s);
hipError_t launch_multiplicities(int order_n, float* mu, hipStream_t s);

// --- peaks and pose (ttm_pose.hip) --------------------------------------------
struct PeakWs {
  unsigned* hist;                 // kHistBins bins of the candidates' key top bits
  unsigned* ctrl;                 // kPeakCtrlWords control words
  unsigned long long* allc;       // every strict local maximum, in kPeakSubs sub-lists (peaks_bigcap entries)
  unsigned long long* cand;       // the sorted list of a round (kCandCap entries)
};
long peaks_bigcap(const Geo& g);  // kPeakSubs sub-lists, each long enough for its share of the scan's blocks
constexpr int kHistBins = 32768;
constexpr int kCandCap = 16384;
constexpr int kPeakSubs = 64;                    // sub-lists of the scan's maxima (one counter each)
constexpr int kPeakCtrlWords = 16 + kPeakSubs;   // control words, then the sub-lists' counters
// planes > 1: `planes` maps of g's extents stored one after another (the
// planes of a stack), each searched on its own; the workspace holds planes
// copies of each buffer (kHistBins bins, kPeakCtrlWords control words,
// peaks_bigcap(g) and kCandCap keys) and the outputs are max_peaks x 3
// positions, max_peaks scores and 2 count words per map
hipError_t launch_peaks(const Geo& g, const float* score, float threshold, float min_dist,
                        int max_peaks, const PeakWs& w, int* out_pos, float* out_score,
                        int* out_count, hipStream_t s, int planes = 1);
struct PoseScratch {
  double* seeds;  // n_seeds * 4: the S^3 seed points
  double* C;      // max_peaks * NB * K
  double* w;      // max_peaks * NB
  int* ok;        // max_peaks * NB
  float* q;       // max_peaks * NB * 4
  double* lam;    // max_peaks * NB
  int* flags;     // max_peaks * NB
  double* ncc;    // max_peaks * NB: NCC at the voxel's own rotation (refine 2)
  unsigned* mlist;  // L0 L1 L2: packed coordinates of the mask voxels (refine 2)
  float* mval;      // L0 L1 L2: their mask values
  int* mcount;      // 2: their number, their largest squared distance from the box centre L / 2
  double* mom;      // max_peaks * NB * 3: sum m f, sum m f^2, sum m (direct tensor)
  unsigned long long* mbits;  // mask_bricks(L): per 4x4x4 brick of the mask box, its voxels with m != 0
  // max_peaks or null: the candidates a refinement round refines (a
  // candidate p with active[p] == 0 is skipped by every pose kernel and its
  // outputs are left as they are); null: all of them
  const int* active;
};

// iterated refinement (refine 3): the rounds after the first (fewer
// candidates move in each, so from the third round on the NCC kernel spreads
// each candidate's 27 neighbours over 27 blocks instead of 9, trading
// template loads for latency).  Each round refines the candidates whose
// moved flag the previous round set (its flags are the round's active mask)
// from their current rows and writes its results to the same rows, with
// moved flags of its own (0 for the candidates it skips).
constexpr int kRefineRounds = 4;
// C_n(x) in float64 by direct window sums at max_peaks candidates (count from
// count_dev if non-null, else count_host), at the 27 neighbours if refine
hipError_t launch_pose_tensor(const Geo& g, const float* image, const float* comps, const float* mask,
                              int order_n, const double* img_stats, float eps_v, int max_peaks, int refine,
                              const int* pos_in, const int* count_dev, int count_host, const PoseScratch& ps,
                              hipStream_t s);
// C_n(x) read from the correlated field: the K inverse-transformed arrays
// before their last (axis-2) pass, evaluated at the (neighbour) voxels by a
// direct inverse real DFT of their rows, times w(x)/V
hipError_t launch_field_at(const Geo& g, const float2* H, long pstride, int K, const float* wmap,
                           int max_peaks, int refine, const int* pos_in, const int* count_dev, int count_host,
                           const PoseScratch& ps, hipStream_t s);
// dominant Z-eigenpairs of the tensors in ps and, per candidate, the
// neighbour with the largest lambda (refine 1) or with the largest NCC of the
// image window against the template rotated by the voxel's own eigenvector
// (refine 2: image, tmpl and mask are read).  Candidate p's outputs go to
// row p; moved (if given) gets, per row, whether the candidate left its
// position.  Candidates that ps.active marks as settled are skipped.
hipError_t launch_pose_solve(const Geo& g, const float* score, int order_n, int n_seeds, int max_iter,
                             double tol, int max_peaks, int refine, const int* pos_in, const int* count_dev,
                             int count_host, const float* image, const float* tmpl, const float* mask,
                             int* out_pos, float* out_quat, double* out_lambda, float* out_score, int* out_flags,
                             double* out_C, const PoseScratch& ps, hipStream_t s, bool reuse_tables = false,
                             int ncc_groups = 9, int* moved = nullptr);

// the mask voxels with m != 0 (packed u0 | u1 << 10 | u2 << 20), their
// values, their count (count[0]) and their largest squared distance from the
// box centre L / 2 (count[1]), in 4x4x4 bricks in C order (C order within a
// brick).  With bits (mask_bricks words) and at most kMaskFastBricks bricks:
// the bricks' ballots, then the entries at prefix-sum offsets, over the
// whole chip; otherwise one block.
constexpr long kMaskFastBricks = 4096;
inline long mask_bricks(int L0, int L1, int L2) { return (long)((L0 + 3) / 4) * ((L1 + 3) / 4) * ((L2 + 3) / 4); }
hipError_t launch_mask_list(const float* mask, int L0, int L1, int L2, unsigned* list, float* mval, int* count,
                            hipStream_t s, unsigned long long* bits = nullptr);

// --- two-dimensional TTM (ttm_planar.hip) -----------------------------------
constexpr int kPlanarMaxOrder = 8;
struct PlanarIdx {
  int k3[kPlanarMaxOrder + 1];   // volume index of the multi-index (n - k, k, 0, 0)
};
hipError_t launch_planar_quats(const float* z, int nrot, float* quats, hipStream_t s);
hipError_t launch_planar_mu(int order_n, float* mu, hipStream_t s);
hipError_t launch_planar_gather(const float* comps3, const PlanarIdx& idx, int np, long A, float* comps2,
                                hipStream_t s);
hipError_t launch_planar_embed(const float* comps2, const PlanarIdx& idx, int np, int K3, long A, float* comps3,
                               hipStream_t s);
// the candidates of every plane (counts[2 b], cand [B][P][3] with plane
// coordinates) in one list of stack positions (b, x1, x2), with the flat index
// b P + p of each and their total
hipError_t launch_planar_compact(int B, int P, const int* counts, const int* cand, int* list, int* idx, int* total,
                                 hipStream_t s);
// the compact-order poses back to [B][P]: positions (x1, x2), z = (a, b) / |(a, b)|
hipError_t launch_planar_scatter(int cap, const int* total, const int* idx, const int* pos3, const float* quat3,
                                 const double* lam3, const float* score3, const int* flags3, int* pos2, float* z2,
                                 double* lam, float* score, int* flags, hipStream_t s);

// --- S'-consistent normalisation (ttm_snorm.hip) ------------------------------
constexpr double kSnormFlatRel = 1e-6;
struct SnormGeo {
  int n0, n1, n2;      // image
  int L0, L1, L2;      // template box
  int max_pos;         // windows 0..max_pos-1 are image boxes, max_pos the template
  int n_pad;           // rotations padded to a multiple of 8
};
struct SnormWs {
  float* quats; double* weights;   // n_rot: the caller's quadrature
  float* rtab; double* kap;        // n_pad: rotation table, omega_j a_j^n
  unsigned* mlist; float* mval; int* mcount;
  float* slabs;                    // (max_pos + 1) L0 L1 L2: h~ per window
  double* stat;                    // (max_pos + 1) x 4
  double* partial;                 // (max_pos + 1) x chunks
};
int snorm_pad(int n_rot);
int snorm_chunks(int n_win, int n_pad);
hipError_t launch_snorm(const SnormGeo& g, const float* image, const float* tmpl, const float* mask,
                        const float* quats, const double* weights, int n_rot, int order_n, const int* pos,
                        const int* count_dev, const double* lambda, const SnormWs& w, float* out_rho, double* out_D,
                        int* out_flags, hipStream_t s);

// --- isotropic low-pass filter (ttm_filter.hip) -----------------------------
constexpr int kMaxFilterRadius = 32;
struct FilterTaps {
  int R;                               // taps k = -R..R
  float h[2 * kMaxFilterRadius + 1];   // h[k + R]
};
// out = in * h along axes 2, 1, 0 (through tmp_a, tmp_b; out may equal in)
hipError_t launch_lowpass(const float* in, float* out, float* tmp_a, float* tmp_b, int n0, int n1, int n2,
                          int periodic, const FilterTaps& taps, hipStream_t s);

// --- gradient of the score at fixed positions (ttm_grad.hip) ---------------
struct GradGeo {
  int n0, n1, n2, L0, L1, L2;
  int lo0, hi0, lo1, hi1, lo2, hi2;   // valid region, inclusive
};
struct GradWs {
  double* wv;      // n_pos: w at the position (0 where it contributes nothing)
  double* mean;    // n_pos: masked window mean
  double* dC;      // n_pos * K: gF mu_alpha C_alpha / F
  double* a;       // n_pos: sum_alpha dC_alpha G_alpha
  float* dT;       // K * L^3: gradient with respect to the tensor components
  double* part;    // ceil(L^3 / 256) * n_rot * 2: per-tile rotation sums
  double* H;       // n_rot * 2: H1_j, H2_j
};
// per position: window statistics, G, F, dC and a (stats[1] = var(f))
hipError_t launch_grad_field(const GradGeo& g, const float* image, const float* comps, const float* mask,
                             int order_n, const double* img_stats, float eps_v, const int* pos, int n_pos,
                             const float* grad_F, const GradWs& w, hipStream_t s);
// the image gradient added onto grad_image (zeroed by the caller)
hipError_t launch_grad_image(const GradGeo& g, const float* image, const float* comps, const float* mask,
                             int order_n, const int* pos, int n_pos, const GradWs& w, float* grad_image,
                             hipStream_t s);
// dT, then the template gradient through the rotations (coef, rstats of the
// tensor build; stats[2] = m_sum) added onto grad_tmpl (zeroed by the caller);
// needs L0 L1 L2 <= 32768
hipError_t launch_grad_tmpl(const GradGeo& g, const float* image, const float* tmpl, const float* mask,
                            int order_n, const float* quats, int nrot, const double* coef, const double* rstats,
                            const double* stats, const int* pos, int n_pos, const GradWs& w, float* grad_tmpl,
                            hipStream_t s);
constexpr int kGradMaxTemplate = 32768;

// --- overlap-save tiles (ttm_tile.hip) ------------------------------------------
struct TileGeo {
  int n0, n1, n2;      // image extents (any)
  int o0, o1, o2;      // tile origin in the image
  int T;               // tile edge (a supported FFT length)
  int L0, L1, L2;      // template extents
  int c0, c1, c2;      // template centre
};
constexpr int kBatchMaxStreams = 8;
hipError_t launch_tile_gather(const float* image, const TileGeo& g, float* tile, hipStream_t s);
hipError_t launch_tile_scatter(const float* tscore, const float* tw, const TileGeo& g, float* score, float* w,
                               hipStream_t s);

// --- all-voxel rotation map (ttm_rmap.hip) ------------------------------------
// planes: C_alpha over the valid box, [K][W0][W1][W2] (pass 3 in P3_FIELD mode).
// n_seeds is a multiple of 32; the table holds rmap_table_uint4 entries.
constexpr int kRmapMaxSeeds = 131072;
long rmap_table_uint4(int order_n, int n_seeds);
hipError_t launch_rmap_table(int order_n, const float* seeds, int n_seeds, uint4* table, hipStream_t s);
// per valid voxel: the winning group of 16 seeds (2 tile + lane half)
hipError_t launch_rmap_scan(const Geo& g, int order_n, const float* planes, const uint4* table, int n_seeds,
                            int* group, hipStream_t s);
// per valid voxel: the score |C_n(x)|_F, the quaternion and lambda written at
// the voxel's image index
hipError_t launch_rmap_polish(const Geo& g, int order_n, const float* planes, const float* seeds,
                              const int* group, int max_iter, double tol, float* out_score, float* out_quat,
                              float* out_lambda, int* unconv, hipStream_t s);

}  // namespace ttm
