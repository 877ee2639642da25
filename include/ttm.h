/*
 * ttm.h -- C ABI of libttm, an MI355X (gfx950) implementation of tensorial
 * template matching (TTM) and of classical rotation-sampled normalised
 * cross-correlation (TM), after Almira, Phelippeau, Martinez-Sanchez, "Fast
 * Normalized Cross-Correlation for Template Matching with Rotations"
 * (arXiv 2311.07561).
 *
 * General rules for every entry point
 * ------------------------------------
 * - Volumes are C-order float32 arrays [n0][n1][n2] (n2 fastest); the voxel
 *   (i0,i1,i2) is the point u = (i0,i1,i2).  Templates and masks are [L0][L1][L2]
 *   with their centre at the integer voxel c = (L0/2, L1/2, L2/2) (floor).
 * - Pointers are DEVICE pointers unless the argument name ends in "_host".
 *   The caller owns all memory: the library never allocates, frees or keeps a
 *   pointer after a call returns.  Scratch memory is a caller-provided
 *   workspace of at least the size the matching *_workspace_bytes call returns
 *   (256-byte alignment or better).
 * - Every call is asynchronous on `stream`: arguments are validated on the
 *   host before anything is enqueued, and a non-OK status means nothing was
 *   enqueued (TTM_E_HIP: a launch failed part-way; the stream's work is then
 *   undefined).  Host arrays are only read during the call: the calls that
 *   copy host arrays to the device (the tensor builds, ttm_snorm,
 *   ttm_score_backward, tm_classical) wait for those copies, and so for the
 *   stream's earlier work, before they return, and cannot be recorded into a
 *   graph.
 * - Correlation is circular: (f * g)(x) = sum_u f((x + u - c) mod N) g(u)
 *   (Section 2, eq. "correlation", with the template measured from its
 *   centre).  Outputs are defined in the VALID region, the positions whose
 *   window [x - c, x - c + L) lies inside the volume on every axis; every
 *   per-voxel output is 0 outside it (indices -1).
 * - The SSP operator is the paper's practical one with an identity filter:
 *   S(f) = m . f for the given mask m (Section 2, lemma "opSSP" with h = delta).
 * - Supported FFT lengths: every axis of N must satisfy
 *   ttm_supported_length() (powers of two from 16 to 512).
 * - No C++ exception crosses this interface.
 */
#ifndef TTM_H
#define TTM_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  TTM_OK = 0,
  TTM_E_ARG = -1,        /* a pointer, order, count or option is invalid       */
  TTM_E_SIZE = -2,       /* a dimension is unsupported or inconsistent         */
  TTM_E_WORKSPACE = -3,  /* the workspace is NULL or smaller than required     */
  TTM_E_HIP = -4,        /* a HIP launch or call failed                        */
  TTM_E_NONFINITE = -5   /* a NaN or infinity in the image or mask, found by
                            the check that ttm_options.check_finite asks for  */
} ttm_status;

typedef struct {
  int32_t n0, n1, n2;    /* extents, C order, n2 fastest */
} ttm_dims;

/* Options for correlation, peak picking and pose recovery. */
typedef struct {
  float eps_v;           /* w(x) = 0 where the local masked variance v(x) is
                            <= eps_v * m_sum * var(f); default 1e-5            */
  float threshold;       /* peak candidates need F(x) > threshold (>= 0)       */
  float min_dist;        /* greedy suppression radius between peaks (voxels)   */
  int32_t max_peaks;     /* at most this many peaks (1..4096)                  */
  int32_t n_seeds;       /* S^3 seed points scanned before SS-HOPM (64..65536) */
  int32_t hopm_max_iter; /* SS-HOPM iteration cap                              */
  double hopm_tol;       /* stop when |d lambda| <= tol * max(1, |lambda|)     */
  int32_t refine;        /* 0: pose at each candidate as found; 1: move each
                            candidate to the voxel of its 3x3x3 neighbourhood
                            with the largest dominant Z-eigenvalue (the
                            spectral norm the Frobenius score stands in for,
                            Section 3.4); 2: move it to the voxel whose NCC
                            c(y, R(q_y)) at its own dominant rotation q_y is
                            largest (needs the raw template); 3: repeat 2 from
                            the moved positions until no candidate moves, at
                            most 4 rounds in all (only moving candidates are
                            recomputed; two candidates may end on the same
                            voxel); default 0                                 */
  int32_t check_finite;  /* 1: ttm_correlate, ttm_match, ttm_correlate_tiled and
                            ttm_rotation_map first reduce the image and the
                            mask to their float64 moments (sum f, sum f^2,
                            sum m), copy those to the host and wait for them;
                            a non-finite moment (a NaN or an infinity in
                            either input) returns TTM_E_NONFINITE with only
                            that reduction enqueued and no output written.
                            The call then synchronises with the stream once,
                            so it cannot be recorded into a graph (the batch
                            calls reject it with TTM_E_ARG).  0 (default): no
                            check; a non-finite input gives NaN outputs     */
} ttm_options;

/* Pose flags (bit set in out_flags). */
#define TTM_POSE_NOT_CONVERGED 1   /* SS-HOPM hit hopm_max_iter               */
#define TTM_POSE_ZERO_NORM     2   /* w(x) = 0 at the peak: pose undefined    */
#define TTM_PEAKS_TRUNCATED    4   /* the candidate list overflowed; fewer
                                      than max_peaks may have been accepted   */

/* Fills *opt with the defaults (eps_v 1e-5, threshold 0, min_dist 8,
 * max_peaks 64, n_seeds 4096, hopm_max_iter 1000, hopm_tol 1e-12, refine 0,
 * check_finite 0). */
void ttm_default_options(ttm_options* opt);

/* Number of independent components of a symmetric tensor of order n on R^4:
 * C(n+3, 3) (Section 3.1).  Returns TTM_E_ARG for odd n or n < 2 (the main
 * theorem needs an even order, Section 3.3) and for n > 8. */
int32_t ttm_num_components(int32_t order_n);

/* 1 if an FFT axis of this length is supported, else 0. */
int32_t ttm_supported_length(int32_t n);

/* Human-readable name of a status code (static storage). */
const char* ttm_status_string(int32_t status);

/* ---------------------------------------------------------------------------
 * Tensor template (Section 3.2): T(z) = int_SO(3) R^{(.)n} S(t)_R(z) dR, in
 * packed form T_alpha(u) = sum_j omega_j Q_j^alpha s_j(u), where s_j is the raw
 * template rotated by Q_j (t_R(u) = t(c + R^-1 (u - c)), trilinear, zero
 * outside the box) and then normalised under the mask
 * (s = m (g - <g,m>/m_sum) / sqrt(<g^2,m> - <g,m>^2/m_sum), Algorithm 1).
 * Packed order of alpha (|alpha| = n): alpha1 from n down to 0, then alpha2,
 * then alpha3; alpha4 is the remainder.  Q = (a,b,c,d) = a + bi + cj + dk,
 * active Hamilton rotation, vector part on axes (0,1,2).
 *
 *   tmpl, mask        [L0][L1][L2] float32; mask values >= 0 with m_sum > 0
 *   order_n           even, 2..8; K = ttm_num_components(order_n)
 *   quats_host        n_rot x 4 float32 unit quaternions (normalised here)
 *   weights_host      n_rot float64 quadrature weights, sum = 1 (+-1e-6)
 *   out_components    K x [L0][L1][L2] float32 (written)
 *   N, out_bank       optional: the correlation bank for images of extent N
 *                     (ttm_bank_bytes(N, L, K) bytes, opaque); NULL = skip
 *
 * The bank holds the K components and the mask, each transformed along axes
 * 2 and 1 (an R2C then a C2C FFT of the zero-padded [L0][n1][n2/2+1] block); it
 * is built once per template and image extent and read by ttm_correlate.
 * Errors: TTM_E_ARG (NULL, odd order, n_rot < 1, a zero or non-finite
 * quaternion, weights not summing to 1 within 1e-6), TTM_E_SIZE (L larger than
 * N, unsupported N), TTM_E_WORKSPACE, TTM_E_HIP.  The mask must have a positive
 * sum; a rotation under which the template has zero masked variance (or a
 * zero mask) contributes nothing to the components.
 * ------------------------------------------------------------------------- */
size_t ttm_bank_bytes(ttm_dims N, ttm_dims L, int32_t K);
size_t ttm_build_workspace_bytes(ttm_dims L, int32_t order_n, int32_t n_rot,
                                 ttm_dims N);
ttm_status ttm_build_tensor_template(
    const float* tmpl, const float* mask, ttm_dims L, int32_t order_n,
    const float* quats_host, const double* weights_host, int32_t n_rot,
    float* out_components, ttm_dims N, void* out_bank,
    void* ws, size_t ws_bytes, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Correlation (Sections 2, 3.2, 3.4): for every valid voxel x
 *   w(x)      = 1 / ||P_S tau_x f||_S
 *             = 1 / sqrt(<(tau_x f)^2, m> - <tau_x f, m>^2 / m_sum)
 *               (0 where v(x) <= eps_v m_sum var(f))
 *   C_alpha(x)= w(x) <tau_x f, T_alpha>            (the correlated tensor field)
 *   F(x)      = ||C_n(x)||_F = sqrt(sum_alpha mu_alpha C_alpha(x)^2),
 *               mu_alpha = n!/prod(alpha_i!)       (Frobenius position proxy)
 * Path: image mean shift (allowed by the affine invariance of Theorem "ThCTM"),
 * R2C FFT of f and f^2, K+2 spectral products fanned out from one read of the
 * image spectrum, batched C2R inverse FFTs, local normalisation and score
 * fused into the last inverse pass.  All arithmetic in float32 except the
 * image moments and the variance subtraction (float64).
 *
 *   image      [n0][n1][n2] float32
 *   bank       from ttm_build_tensor_template with the same N, L, order
 *   mask       [L0][L1][L2] float32, the mask used to build the bank
 *   opt        options (eps_v is used)
 *   out_score  [n0][n1][n2] float32 F(x) (written)
 *   out_w      [n0][n1][n2] float32 w(x), or NULL
 * Errors: TTM_E_ARG, TTM_E_SIZE, TTM_E_WORKSPACE, TTM_E_HIP, and
 * TTM_E_NONFINITE when opt->check_finite is set and the image or the mask
 * holds a NaN or an infinity.
 * ------------------------------------------------------------------------- */
size_t ttm_correlate_workspace_bytes(ttm_dims N, ttm_dims L, int32_t K);
ttm_status ttm_correlate(
    const float* image, ttm_dims N, const void* bank, ttm_dims L,
    int32_t order_n, const float* mask, const ttm_options* opt,
    float* out_score, float* out_w, void* ws, size_t ws_bytes,
    hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Position and rotation recovery (Sections 3.3, 3.4).
 * Peaks: valid voxels with F(x) > threshold and F(x) strictly greater than all
 * 26 neighbours, ordered by F descending (ties: lower linear index first),
 * greedily suppressed within min_dist of an accepted peak, at most max_peaks.
 * At each peak the tensor C_n(x) is recomputed directly in float64 from the
 * image window and the components (two-pass local variance), and its dominant
 * Z-eigenpair (max C Q^n on |Q| = 1, eq. "Zeigen") is found by a scan of
 * n_seeds S^3 points, each of 64 lanes polishing its own best seed with
 * Newton steps on the sphere that fall back to a shifted power step (SS-HOPM)
 * whenever they do not increase lambda; by Theorem "main" the eigenvector is
 * the rotation of the match.  With opt->refine = 1 this is done at the 27
 * voxels around each peak and the one with the largest lambda is reported.
 * With opt->refine = 2 each of the 27 voxels y is scored by the classical
 * normalised correlation at its own rotation, c(y, R(q_y)) = w(y) <tau_y f,
 * s_R> with s_R the raw template rotated by R(q_y) and normalised under the
 * mask (Section 2, Algorithm 1; float64 sums), and the voxel with the largest
 * NCC is reported (ties: the centre, then the lower neighbour index).
 *
 *   score            [n0][n1][n2] float32 from ttm_correlate or
 *                    ttm_correlate_tiled (no FFT here: any extents n_i >= L_i,
 *                    n_i <= 8192, volume < 2^31)
 *   image            the correlated image; components: K x [L0][L1][L2] float32
 *   mask             the mask used for the components
 *   tmpl             the raw template [L0][L1][L2] float32 the components were
 *                    built from; read only when opt->refine >= 2 (else may be
 *                    NULL; NULL with refine >= 2 is TTM_E_ARG)
 *   out_pos          max_peaks x 3 int32 (i0,i1,i2)
 *   out_quat         max_peaks x 4 float32, canonical (a > 0)
 *   out_lambda       max_peaks float64 dominant Z-eigenvalue C Q^n
 *   out_peak_score   max_peaks float32 F at the peak
 *   out_flags        max_peaks int32 TTM_POSE_* bits
 *   out_C            max_peaks x K float64 C_alpha at the peak, or NULL
 *   out_count        2 int32: [0] number of peaks written, [1] flags
 *                    (TTM_PEAKS_TRUNCATED when the bounded candidate list ran
 *                    out before max_peaks peaks were accepted)
 * Only the first out_count[0] rows are defined.  The mask must have a
 * positive sum (otherwise w = 0 and every pose is flagged TTM_POSE_ZERO_NORM).
 * ------------------------------------------------------------------------- */
size_t ttm_pose_workspace_bytes(ttm_dims N, ttm_dims L, int32_t order_n,
                                const ttm_options* opt);
/* Pose at caller-given positions (no peak search): the same tensor and
 * eigenpair computation as ttm_recover_pose at n_pos positions
 * (positions: n_pos x 3 int32 device array, each inside the valid region, else
 * its lambda is -inf and its flags TTM_POSE_ZERO_NORM), with opt->refine as
 * there.  out_pos receives the (refined) positions; out_C may be NULL.
 * n_pos <= opt->max_peaks; workspace from ttm_pose_workspace_bytes. */
ttm_status ttm_pose_at(
    const float* image, const float* components, const float* mask,
    const float* tmpl, ttm_dims N, ttm_dims L, int32_t order_n,
    const ttm_options* opt,
    const int32_t* positions, int32_t n_pos, int32_t* out_pos,
    float* out_quat, double* out_lambda, int32_t* out_flags, double* out_C,
    void* ws, size_t ws_bytes, hipStream_t stream);
/* ttm_pose_at for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same computation and outputs as ttm_pose_at, with its scratch (the
 * image moments, the seed table, the tensors, eigenpairs and NCC values of
 * the max_peaks x 27 voxels, the mask list and the refinement rounds) in a
 * static 8 MiB device array of the library instead of a workspace.  The call
 * allocates nothing (no hipMalloc, no library allocation, no profiler
 * events) and takes the array's device address once per GPU.
 *   Limit: the pose scratch of (max_peaks, K = C(n+3,3), refine, n_seeds, L)
 *   must fit 8 MiB, else TTM_E_WORKSPACE; e.g. max_peaks 64 at refine 3 with
 *   n_seeds 4096 fits for K <= 84 and L0 L1 L2 <= 64^3.
 *   The array is one per GPU and shared by every call on it, and keeps the
 *   last call's contents (nothing in it needs clearing): calls that overlap
 *   on one GPU (two streams, two threads) race and must be serialised by the
 *   caller.  `stream` must belong to the current device (else TTM_E_ARG).
 * Arguments and the other errors as ttm_pose_at. */
ttm_status ttm_pose_at_noalloc(
    const float* image, const float* components, const float* mask,
    const float* tmpl, ttm_dims N, ttm_dims L, int32_t order_n,
    const ttm_options* opt,
    const int32_t* positions, int32_t n_pos, int32_t* out_pos,
    float* out_quat, double* out_lambda, int32_t* out_flags, double* out_C,
    hipStream_t stream);
ttm_status ttm_recover_pose(
    const float* score, const float* image, const float* components,
    const float* mask, const float* tmpl, ttm_dims N, ttm_dims L,
    int32_t order_n, const ttm_options* opt, int32_t* out_pos, float* out_quat,
    double* out_lambda, float* out_peak_score, int32_t* out_flags,
    double* out_C, int32_t* out_count, void* ws, size_t ws_bytes,
    hipStream_t stream);

/* ---------------------------------------------------------------------------
 * The whole per-tomogram path in one call (Sections 2, 3.2-3.4): the
 * correlation of ttm_correlate, the peaks of ttm_recover_pose, and the pose at
 * each peak with C_n(x) taken from the correlated tensor field itself (the K
 * transformed arrays are evaluated at the candidate voxels by a point inverse
 * DFT of their last axis, times w(x)) instead of being recomputed from the
 * image window.  Arguments as in ttm_correlate and ttm_recover_pose; out_w
 * and out_C may be NULL.  Workspace from ttm_match_workspace_bytes.
 * ------------------------------------------------------------------------- */
size_t ttm_match_workspace_bytes(ttm_dims N, ttm_dims L, int32_t order_n,
                                 const ttm_options* opt);
ttm_status ttm_match(
    const float* image, ttm_dims N, const void* bank, ttm_dims L,
    int32_t order_n, const float* mask, const float* tmpl,
    const ttm_options* opt,
    float* out_score, float* out_w, int32_t* out_pos, float* out_quat,
    double* out_lambda, float* out_peak_score, int32_t* out_flags,
    double* out_C, int32_t* out_count, void* ws, size_t ws_bytes,
    hipStream_t stream);

/* ---------------------------------------------------------------------------
 * All-voxel rotation map (Section 3.4 with Theorem "main"): the rotation at
 * every voxel of the valid region, not only at peaks, as the dominant
 * Z-eigenpair of C_n(x) (eq. "Zeigen": max over unit Q of C_n(x) Q^n):
 *   1. the correlation of ttm_correlate, keeping C_alpha(x) for every valid
 *      voxel (float32, K planes over the valid box, in the workspace);
 *   2. a seed scan: phi(x, Q_j) = sum_alpha mu_alpha C_alpha(x) Q_j^alpha at
 *      every seed Q_j, a [V x K] . [K x J] product on the matrix cores in
 *      fp16 with float32 accumulation, keeping per voxel the group of 16
 *      seeds holding the largest value;
 *   3. a float64 polish per voxel: lambda at those 16 seeds, then the
 *      safeguarded Newton / shifted power iteration of ttm_recover_pose from
 *      the best of them.
 * The seed scan decides only the starting basin: where two local maxima of
 * phi are within the fp16 rounding of each other the map may hold the
 * second; elsewhere it is the global maximiser.
 *
 *   image, bank, mask, N, L, order_n   as in ttm_correlate
 *   opt         eps_v, hopm_max_iter, hopm_tol are used
 *   seeds       n_seeds x 4 float32 device array of quaternions (normalised
 *               here; sign irrelevant: the order is even); n_seeds a
 *               multiple of 32 in [32, 131072]
 *   out_score   [n0][n1][n2] F = |C_n(x)|_F as ttm_correlate, here summed in
 *               float64 from the stored float32 C_alpha
 *   out_w       [n0][n1][n2] w, or NULL
 *   out_quat    [n0][n1][n2][4] float32: the dominant rotation (unit, first
 *               nonzero component positive); zero outside the valid region;
 *               the identity where C_n(x) = 0 (w(x) = 0)
 *   out_lambda  [n0][n1][n2] float32: its Z-eigenvalue C_n(x) q^n; zero
 *               outside the valid region and where C_n(x) = 0
 *   out_unconverged  one int32 (device), or NULL: the number of voxels whose
 *               polish stopped at hopm_max_iter
 * All outputs are device arrays written on `stream`; the workspace holds
 * K float32 values per valid voxel (ttm_rotation_map_workspace_bytes).
 * Errors: TTM_E_ARG (NULL, order, n_seeds, options), TTM_E_SIZE,
 * TTM_E_WORKSPACE, TTM_E_HIP.
 * ------------------------------------------------------------------------- */
size_t ttm_rotation_map_workspace_bytes(ttm_dims N, ttm_dims L,
                                        int32_t order_n, int32_t n_seeds);
ttm_status ttm_rotation_map(
    const float* image, ttm_dims N, const void* bank, ttm_dims L,
    int32_t order_n, const float* mask, const ttm_options* opt,
    const float* seeds, int32_t n_seeds, float* out_score, float* out_w,
    float* out_quat, float* out_lambda, int32_t* out_unconverged, void* ws,
    size_t ws_bytes, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Two-dimensional TTM (Sections 2 and 3 with d = 2; Theorem 1 is stated for
 * R^3 only, so the planar case has its own checks).
 * A plane rotation is described by the unit complex number z = (a, b) of
 * half its angle: R(z) = [[a^2 - b^2, -2ab], [2ab, a^2 - b^2]], the rotation
 * by theta = 2 atan2(b, a) of the (axis 1, axis 2) plane; z and -z give the
 * same rotation, and even orders make them equivalent (with the full angle an
 * even order could not tell theta from theta + pi).  The planar tensor
 * C_n(x) in S^n(R^2) has the n + 1 entries C_k of the multi-indices
 * (n - k, k), multiplicity C(n, k); its Frobenius norm is the score and its
 * dominant eigenvector on the unit circle the rotation.
 *
 * Images come as a stack of B planes [B][n1][n2] (B, n1, n2 supported
 * lengths), the template and mask as [L1][L2] (L1 <= n1, L2 <= n2, L2 <= 512,
 * L1 <= 1023); orders n = 2, 4, 6, 8.  The planes are correlated together and
 * never mix; the mean shift and the variance floor of ttm_options.eps_v are
 * those of the whole stack.
 *
 * ttm_build_tensor_template_2d: T_k(u) = sum_j omega_j a_j^(n-k) b_j^k s_j(u)
 * (s_j the raw template rotated bilinearly by R(z_j) about (L1/2, L2/2), zero
 * outside the box, then normalised under the mask), written to
 * out_components [(n+1)][L1][L2]; with out_bank non-NULL also the correlation
 * bank for stacks of shape (B, n1, n2) (ttm_bank_bytes_2d bytes).
 *   z_host        n_rot x 2 float32 host array of unit complex numbers
 *                 (normalised here); weights_host n_rot float64, sum 1
 * ttm_match_2d: per plane b, the score and w maps (out_score, out_w
 * [B][n1][n2]; out_w may be NULL), the candidates of the 3-D rule restricted
 * to the plane (strict maxima over the 8 neighbours inside the valid region,
 * sorted, suppression within opt->min_dist, at most opt->max_peaks), the
 * tensor at each by direct float64 window sums and its dominant eigenpair
 * (on the circle: a 1024-point scan of the half-angle, then a parallel zoom
 * to below 1e-11 rad, in float64; opt->n_seeds, hopm_max_iter and hopm_tol
 * are not used and TTM_POSE_NOT_CONVERGED is never set), refined as
 * opt->refine (0..3, the neighbourhood being the 3 x 3 pixels):
 *   out_pos        [B][max_peaks][2] int32 (x1, x2)
 *   out_z          [B][max_peaks][2] float32, unit, a > 0 (or a = 0, b > 0)
 *   out_lambda     [B][max_peaks] float64
 *   out_peak_score [B][max_peaks] float32, out_flags [B][max_peaks] int32
 *   out_count      [B][2] int32: the count of each plane and TTM_PEAKS_* bits
 * Entries past each plane's count are not written.  tmpl ([L1][L2]) is read
 * when opt->refine >= 2.  Classical matching of a stack is tm_classical with
 * L = (1, L1, L2) and the quaternions (a, b, 0, 0).
 * Errors: TTM_E_ARG, TTM_E_SIZE, TTM_E_WORKSPACE, TTM_E_HIP.
 * ------------------------------------------------------------------------- */
size_t ttm_bank_bytes_2d(int32_t B, int32_t n1, int32_t n2, int32_t L1,
                         int32_t L2, int32_t order_n);
size_t ttm_build_workspace_bytes_2d(int32_t L1, int32_t L2, int32_t order_n,
                                    int32_t n_rot);
ttm_status ttm_build_tensor_template_2d(
    const float* tmpl, const float* mask, int32_t L1, int32_t L2,
    int32_t order_n, const float* z_host, const double* weights_host,
    int32_t n_rot, float* out_components, int32_t B, int32_t n1, int32_t n2,
    void* out_bank, void* ws, size_t ws_bytes, hipStream_t stream);
size_t ttm_match_2d_workspace_bytes(int32_t B, int32_t n1, int32_t n2,
                                    int32_t L1, int32_t L2, int32_t order_n,
                                    const ttm_options* opt);
ttm_status ttm_match_2d(
    const float* images, int32_t B, int32_t n1, int32_t n2, const void* bank,
    const float* components, const float* tmpl, const float* mask,
    int32_t L1, int32_t L2, int32_t order_n, const ttm_options* opt,
    float* out_score, float* out_w, int32_t* out_pos, float* out_z,
    double* out_lambda, float* out_peak_score, int32_t* out_flags,
    int32_t* out_count, void* ws, size_t ws_bytes, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * S'-consistent normalisation of peak scores (Section 3.4, the discussion of
 * false positives; S_2 and S' = S_2 S from the proof of Theorem 1).
 * The tensor correlation lambda(x) = w(x) <tau_x f, t_Q>_{S'} is an inner
 * product under S' normalised under S, so it is not bounded by 1 and favours
 * smooth windows.  The paper states the quantity and no algorithm; here the
 * SO(3) convolution S_2 (kernel a^n of the identity's features) takes the
 * tensor template's own rotation quadrature.  Per window h (the image box of
 * each position, and the template):
 *   D(h) = sum_j omega_j a_j^n <h~, N_m(I_{R_j} h~)>,
 *   h~ = (h - <h,m>/m_sum) / ||h - <h,m>/m_sum||_S,
 * with I_R the trilinear rotation about the box centre (zero outside the box)
 * and N_m the masked normalisation of the tensor build; then
 *   rho'(x) = lambda(x) / sqrt(D(tau_x f) D(t)),
 * which is 1 at a noiseless copy and lies in [-1, 1] wherever the discrete S'
 * form is positive semidefinite.
 *
 *   image, N     [n0][n1][n2] float32 (any extents, n_i <= 8192, volume < 2^31)
 *   tmpl, mask, L, order_n, quats_host, weights_host, n_rot
 *                as given to ttm_build_tensor_template (the same quadrature)
 *   pos          max_pos x 3 int32 device positions (e.g. ttm_recover_pose's
 *                out_pos); a window that leaves the image is flagged
 *   lambda       max_pos float64 device: lambda at each position (e.g.
 *                ttm_recover_pose's out_lambda)
 *   count        one int32 on the device, the number of positions used
 *                (clamped to [0, max_pos]), or NULL for max_pos
 *   out_rho      max_pos float32: rho' (0 where flagged)
 *   out_D        max_pos + 1 float64: D of each window, then D of the
 *                template (NaN for a flat or outside window)
 *   out_flags    max_pos int32 TTM_SNORM_* bits
 * Entries past count are not written.  Masked variance at most 1e-6 of the
 * masked second moment marks a window flat; a rotated copy with as little
 * variance adds nothing to D.  The mask's nonzero voxels must lie in the box
 * (each extent of L at most 1023).  Workspace from
 * ttm_snorm_workspace_bytes.  Errors: TTM_E_ARG (NULL pointers, order,
 * quadrature, max_pos), TTM_E_SIZE, TTM_E_WORKSPACE, TTM_E_HIP.
 * ------------------------------------------------------------------------- */
#define TTM_SNORM_FLAT      1   /* the window's masked variance vanishes    */
#define TTM_SNORM_NONPOS    2   /* D(window) <= 0 in this quadrature        */
#define TTM_SNORM_OUTSIDE   4   /* the window leaves the image              */
#define TTM_SNORM_TEMPLATE  8   /* D(template) is not positive              */
size_t ttm_snorm_workspace_bytes(ttm_dims L, int32_t n_rot, int32_t max_pos);
ttm_status ttm_snorm(
    const float* image, ttm_dims N, const float* tmpl, const float* mask,
    ttm_dims L, int32_t order_n, const float* quats_host,
    const double* weights_host, int32_t n_rot, const int32_t* pos,
    const double* lambda, const int32_t* count, int32_t max_pos,
    float* out_rho, double* out_D, int32_t* out_flags, void* ws,
    size_t ws_bytes, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Tomograms of any extent: overlap-save tiling onto power-of-two FFT tiles.
 * The correlation of Section 2 (ttm_correlate's score F and w) is computed on
 * cubic tiles of edge T (a supported length, T >= each template extent).
 * Tiles step by T - L + 1 per axis, so the positions where a tile's window
 * lies inside the tile partition the image's valid region; positions whose
 * window leaves the image are dropped and the maps are 0 there (as for
 * ttm_correlate).  The image statistics (mean shift, variance floor of
 * ttm_options.eps_v, mask sum) are those of the whole image, so the result is
 * ttm_correlate's for any tiling, up to float32 rounding.  The bank is the
 * template's built with image_shape = (T, T, T).
 *
 *   image      [n0][n1][n2] float32, any extents with n_i >= L_i, n_i <= 8192,
 *              volume < 2^31
 *   out_score  [n0][n1][n2]; out_w likewise or NULL
 * Workspace from ttm_correlate_tiled_workspace_bytes (independent of the
 * image size).  ttm_tile_count returns the number of tiles (or TTM_E_SIZE).
 * ttm_recover_pose and ttm_pose_at accept the same image extents.
 * Errors: TTM_E_ARG, TTM_E_SIZE, TTM_E_WORKSPACE, TTM_E_HIP.
 * ------------------------------------------------------------------------- */
int32_t ttm_tile_count(ttm_dims N, ttm_dims L, int32_t T);
size_t ttm_correlate_tiled_workspace_bytes(ttm_dims L, int32_t order_n,
                                           int32_t T);
ttm_status ttm_correlate_tiled(
    const float* image, ttm_dims N, const void* bank, ttm_dims L,
    int32_t order_n, int32_t T, const float* mask, const ttm_options* opt,
    float* out_score, float* out_w, void* ws, size_t ws_bytes,
    hipStream_t stream);

/* Autotuner of the tile schedule (no counterpart in the paper).
 * ttm_autotune_tiles times one tile correlation (gather, the FFT passes of
 * the tile edge with their radix plan, scatter) for each candidate edge
 * tiles_host[i] with the template's bank banks_host[i] (built for that
 * edge), `repeats` times after one untimed run, and writes the median
 * milliseconds to ms_host[i].  It synchronises `stream`.  Workspace from
 * ttm_autotune_workspace_bytes.
 * ttm_choose_tile returns the candidate edge minimising
 * ttm_tile_count(N, L, T) x ms (the larger edge on ties), or TTM_E_SIZE when
 * none fits.  Host only. */
size_t ttm_autotune_workspace_bytes(ttm_dims L, int32_t order_n,
                                    const int32_t* tiles_host, int32_t n);
ttm_status ttm_autotune_tiles(
    const void* const* banks_host, const int32_t* tiles_host, int32_t n,
    ttm_dims L, int32_t order_n, const float* mask, const ttm_options* opt,
    int32_t repeats, float* ms_host, void* ws, size_t ws_bytes,
    hipStream_t stream);
int32_t ttm_choose_tile(ttm_dims N, ttm_dims L, const int32_t* tiles_host,
                        const float* ms_host, int32_t n);

/* ---------------------------------------------------------------------------
 * Batches of tomograms and templates of uneven sizes (no counterpart in the
 * paper).  A job is one tomogram against one template: the tiled correlation
 * above at the job's tile edge, then ttm_recover_pose on the stitched score
 * map (peaks, C_n(x) from direct float64 window sums, the eigenpair, the
 * refinement of opt->refine).  ttm_batch_match runs the jobs eagerly, one
 * after another on `stream`, sharing one workspace.  ttm_batch_graph_create
 * records them into one hipGraph by stream capture (stream must be a created
 * stream, not the legacy default; profiling records nothing while
 * capturing): the jobs are split over n_streams branches (1..8, longest jobs
 * first onto the least loaded branch, a job's cost taken as its tiles times
 * the tile volume) that run concurrently, each with its own slice of the
 * workspace; ttm_graph_launch replays the graph as one launch on any stream.
 * ttm_batch_workspace_bytes gives n_streams times the largest job's need
 * (n_streams = 1 for ttm_batch_match).  The graph holds the job
 * descriptors' pointers and the workspace: they must stay valid, and be used
 * by nothing else while a replay runs.  Outputs per job as
 * ttm_recover_pose's (max_peaks rows; out_C is not produced).
 * Errors: TTM_E_ARG, TTM_E_SIZE, TTM_E_WORKSPACE, TTM_E_HIP.
 * ------------------------------------------------------------------------- */
typedef struct {
  const float* image;        /* [n0][n1][n2] device */
  ttm_dims N;
  const void* bank;          /* the template's bank at (tile, tile, tile) */
  int32_t tile;              /* tile edge T */
  const float* components;   /* K x [L0][L1][L2] */
  const float* mask;         /* [L0][L1][L2] */
  const float* tmpl;         /* [L0][L1][L2], needed with refine >= 2 */
  ttm_dims L;
  float* out_score;          /* [n0][n1][n2] */
  float* out_w;              /* [n0][n1][n2] or NULL */
  int32_t* out_pos;          /* max_peaks x 3 */
  float* out_quat;           /* max_peaks x 4 */
  double* out_lambda;        /* max_peaks */
  float* out_peak_score;     /* max_peaks */
  int32_t* out_flags;        /* max_peaks */
  int32_t* out_count;        /* 2 */
} ttm_batch_job;
typedef struct ttm_graph_s* ttm_graph;
size_t ttm_batch_workspace_bytes(const ttm_batch_job* jobs_host,
                                 int32_t n_jobs, int32_t order_n,
                                 const ttm_options* opt, int32_t n_streams);
ttm_status ttm_batch_match(const ttm_batch_job* jobs_host, int32_t n_jobs,
                           int32_t order_n, const ttm_options* opt,
                           int32_t n_streams, void* ws, size_t ws_bytes,
                           hipStream_t stream);
ttm_status ttm_batch_graph_create(const ttm_batch_job* jobs_host,
                                  int32_t n_jobs, int32_t order_n,
                                  const ttm_options* opt, int32_t n_streams,
                                  void* ws, size_t ws_bytes,
                                  hipStream_t stream, ttm_graph* out_graph);
ttm_status ttm_graph_launch(ttm_graph graph, hipStream_t stream);
void ttm_graph_destroy(ttm_graph graph);

/* ---------------------------------------------------------------------------
 * Classical template matching with rotations (Algorithm 1 with a loop over
 * the rotation list): for every valid voxel
 *   out_best_ncc(x) = max_j c(x, R_j),  c(x,R) = w(x) (f * s_R)(x)
 *   out_best_rot(x) = lowest j attaining the maximum
 * with s_R the rotated-then-normalised template as in the tensor build.
 * Where w(x) = 0 every c is 0 and the index is 0.
 *
 *   image [n0][n1][n2]; tmpl, mask [L0][L1][L2]; quats_host n_rot x 4 float32
 * Errors: TTM_E_ARG, TTM_E_SIZE, TTM_E_WORKSPACE, TTM_E_HIP.
 * ------------------------------------------------------------------------- */
size_t tm_classical_workspace_bytes(ttm_dims N, ttm_dims L, int32_t n_rot);
ttm_status tm_classical(
    const float* image, ttm_dims N, const float* tmpl, const float* mask,
    ttm_dims L, const float* quats_host, int32_t n_rot,
    const ttm_options* opt, float* out_best_ncc, int32_t* out_best_rot,
    void* ws, size_t ws_bytes, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Isotropic low-pass filter (Section 2: the matching is applied to f * h and
 * t * h for an isotropic low-pass h with h * 1 = 1).  h is a sampled Gaussian
 * of standard deviation sigma voxels on k = -R..R, R = ceil(3 sigma) <= 32,
 * normalised to unit sum, applied along each axis:
 *   out(x) = sum_k h(k) in(x - k)
 * with indices modulo the extent (periodic = 1, for images: the correlation
 * is circular) or zero outside the array (periodic = 0, for the template
 * box).  sigma = 0 copies.  in and out are [n0][n1][n2] float32 device arrays
 * and may be the same.
 * Errors: TTM_E_ARG (NULL, sigma < 0 or too large, periodic not 0/1),
 * TTM_E_SIZE, TTM_E_WORKSPACE, TTM_E_HIP.
 * ------------------------------------------------------------------------- */
size_t ttm_lowpass_workspace_bytes(ttm_dims N);
ttm_status ttm_lowpass(const float* in, ttm_dims N, float sigma,
                       int32_t periodic, float* out, void* ws,
                       size_t ws_bytes, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Gradient of the score at fixed positions (the adjoint of the tensor build,
 * Section 3.2, the window correlation and local normalisation, Section 2, and
 * the Frobenius norm, Section 3.4): for L = sum_p grad_score[p] F(x_p), with
 * F evaluated as ttm_correlate does (in float64 window sums here), writes
 * dL/dt (the raw template) and dL/df (the image).  The tensor components are
 * not differentiated through storage: the rotations are re-sampled from the
 * template, so the components only supply T_alpha for the image gradient.
 *
 *   image [n0][n1][n2] (any extents: no FFT is involved); tmpl, mask
 *               [L0][L1][L2]; quats_host, weights_host,
 *   n_rot       the quadrature of the tensor build (same checks)
 *   components  K x [L0][L1][L2] from ttm_build_tensor_template with them
 *   positions   n_pos x 3 int32 device; positions outside the valid region,
 *               or where w = 0 or F = 0, contribute nothing
 *   grad_score  n_pos float32 device
 *   opt         eps_v is used
 *   out_grad_tmpl   [L0][L1][L2] float32 (written), or NULL; needs
 *                   L0 L1 L2 <= 32768 (TTM_E_SIZE otherwise)
 *   out_grad_image  [n0][n1][n2] float32 (written: zero outside the
 *                   positions' windows), or NULL
 * Errors: TTM_E_ARG, TTM_E_SIZE, TTM_E_WORKSPACE, TTM_E_HIP.
 * ------------------------------------------------------------------------- */
size_t ttm_score_backward_workspace_bytes(ttm_dims L, int32_t order_n,
                                          int32_t n_rot, int32_t n_pos);
ttm_status ttm_score_backward(
    const float* image, ttm_dims N, const float* tmpl, const float* mask,
    ttm_dims L, int32_t order_n, const float* quats_host,
    const double* weights_host, int32_t n_rot, const float* components,
    const int32_t* positions, int32_t n_pos, const float* grad_score,
    const ttm_options* opt, float* out_grad_tmpl, float* out_grad_image,
    void* ws, size_t ws_bytes, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Instrumentation (not part of the method).  When enabled, every call records
 * a HIP event pair on its stream around each kernel group, by class:
 *   0 image moments, 1 axis-2 R2C rows, 2 axis-1 forward pencils,
 *   3 pass 1 (axis-0 fan-out), 4 axis-1 inverse pencils, 5 pass 3 (axis-2 C2R
 *   + reduction), 6 peaks, 7 pose, 8 tensor build, 9 classical epilogue,
 *   10 rotation-map seed scan, 11 rotation-map seed table, fills and polish,
 *   12 S'-normalisation.
 * ttm_profile_read waits for the recorded events, writes the summed
 * milliseconds and launch counts of the first n classes, clears the record
 * and returns the number of classes (or TTM_E_HIP).  Event pairs are created
 * on first use and reused; with profiling off nothing is recorded.
 * ------------------------------------------------------------------------- */
#define TTM_PROFILE_CLASSES 13
void ttm_profile_enable(int32_t on);
int32_t ttm_profile_read(double* ms_out, int64_t* launches_out, int32_t n);
const char* ttm_profile_class_name(int32_t cls);

#ifdef __cplusplus
}
#endif

#endif /* TTM_H */
