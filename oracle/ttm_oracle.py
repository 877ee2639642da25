"""FP64 CPU oracle for tensorial template matching (TTM) and classical template
matching (TM).

TEST INFRASTRUCTURE ONLY.  Nothing in the library's product path imports,
calls or links this module: it is used by ``tests/``, by the smoke check and by
the benchmark's CPU-baseline leg.  It is a plain, slow, obviously correct
implementation written from the paper (Almira, Phelippeau, Martinez-Sanchez,
"Fast Normalized Cross-Correlation for Template Matching with Rotations",
arXiv 2311.07561).  Every correlation is a *direct spatial sum* (no FFT), every
reduction is in float64, and each function cites the passage it follows.

Readings of points where the paper is silent:

* grid: C-order ``[n0][n1][n2]``; correlation is circular,
  ``(f * g)(x) = sum_u f((x + u - c) mod N) g(u)`` with ``c = L // 2`` the
  template centre (Section 2, eq. "correlation", with the template measured from
  its centre); results are compared in the *valid region* where the window
  ``[x - c, x - c + L)`` lies inside the image on every axis;
* unit quaternion ``Q = (a, b, c, d)`` scalar first, active Hamilton rotation;
* ``t_R(u) = t(c + R^-1 (u - c))`` (Section 2, ``t_R = O_{R^-1}(t)``), sampled
  trilinearly with zero outside the L-box;
* mask ``m`` and filter ``h = delta``: ``S(f) = m f`` (Section 2, the practical
  SSP operator with an identity filter);
* rotate the raw template, then normalise it under the mask, per rotation, so
  that every rotated template satisfies ``<s,1>_S = 0`` and ``||s||_S = 1``
  exactly on the grid;
* ``w(x) = 0`` where the local masked variance ``v`` is at most
  ``eps_v * m_sum * var(f)``;
* symmetric tensors of ``S^n(R^4)`` are stored packed, one entry per multi-index
  ``alpha`` with ``|alpha| = n`` (order: ``alpha_1`` from ``n`` down to 0, then
  ``alpha_2``, then ``alpha_3``; ``alpha_4`` is the remainder), with
  multiplicity ``mu_alpha = n! / prod(alpha_i!)``;
* the SO(3) integral is a caller-supplied quadrature ``{(Q_j, omega_j)}`` over
  unit quaternions, ``sum omega_j = 1`` (normalised Haar measure).
"""
from __future__ import annotations

import functools
import itertools
import math

import numpy as np

EPS_V_DEFAULT = 1e-5


# ----------------------------------------------------------------------------
# quaternions (Section 2, quaternion facts; Section 4, the S^3 parametrisation)
# ----------------------------------------------------------------------------

def quat_to_matrix(q) -> np.ndarray:
    """Rotation matrix of the unit quaternion ``q = a + b i + c j + d k``: the
    map ``v -> q v q*`` on pure quaternions ``v = (0, v0, v1, v2)``."""
    q = np.asarray(q, dtype=np.float64)
    a, b, c, d = q / np.linalg.norm(q)
    # written out from q v q* with the Hamilton product
    return np.array([
        [a * a + b * b - c * c - d * d, 2.0 * (b * c - a * d), 2.0 * (b * d + a * c)],
        [2.0 * (b * c + a * d), a * a - b * b + c * c - d * d, 2.0 * (c * d - a * b)],
        [2.0 * (b * d - a * c), 2.0 * (c * d + a * b), a * a - b * b - c * c + d * d],
    ])


def quat_mul(p, q) -> np.ndarray:
    """Hamilton product ``p q``."""
    a1, b1, c1, d1 = p
    a2, b2, c2, d2 = q
    return np.array([
        a1 * a2 - b1 * b2 - c1 * c2 - d1 * d2,
        a1 * b2 + b1 * a2 + c1 * d2 - d1 * c2,
        a1 * c2 - b1 * d2 + c1 * a2 + d1 * b2,
        a1 * d2 + b1 * c2 - c1 * b2 + d1 * a2,
    ])


def quat_canonical(q) -> np.ndarray:
    """Unit quaternion with scalar part > 0 (first nonzero component > 0 when
    the scalar part is 0): ``q`` and ``-q`` are the same rotation."""
    q = np.asarray(q, dtype=np.float64)
    q = q / np.linalg.norm(q)
    for v in q:
        if v != 0.0:
            return q if v > 0 else -q
    return q


def rotation_angle_deg(q1, q2) -> float:
    """Angle of the rotation taking ``q1`` to ``q2``: ``2 acos |<q1, q2>|``
    (the inner product of unit quaternions is ``Re(q2^-1 q1)``, Section 2)."""
    q1 = np.asarray(q1, dtype=np.float64)
    q2 = np.asarray(q2, dtype=np.float64)
    d = abs(float(np.dot(q1 / np.linalg.norm(q1), q2 / np.linalg.norm(q2))))
    return math.degrees(2.0 * math.acos(min(1.0, d)))


# ----------------------------------------------------------------------------
# packed symmetric tensors (Section 3.1)
# ----------------------------------------------------------------------------

@functools.lru_cache(maxsize=None)
def multi_indices(n: int) -> np.ndarray:
    """Multi-indices ``alpha`` of ``S^n(R^4)`` in storage order (one shared,
    read-only array per order)."""
    out = []
    for a1 in range(n, -1, -1):
        for a2 in range(n - a1, -1, -1):
            for a3 in range(n - a1 - a2, -1, -1):
                out.append((a1, a2, a3, n - a1 - a2 - a3))
    arr = np.array(out, dtype=np.int64)
    arr.setflags(write=False)
    return arr


def num_components(n: int) -> int:
    """``dim S^n(R^4) = C(n + 3, 3)`` (Section 3.1)."""
    return math.comb(n + 3, 3)


@functools.lru_cache(maxsize=None)
def multiplicities(n: int) -> np.ndarray:
    """How many of the ``4^n`` entries of a symmetric tensor equal the packed
    entry ``alpha``: ``n! / (alpha_1! alpha_2! alpha_3! alpha_4!)`` (one
    shared, read-only array per order)."""
    f = math.factorial
    arr = np.array([f(n) // (f(a[0]) * f(a[1]) * f(a[2]) * f(a[3]))
                    for a in multi_indices(n)], dtype=np.float64)
    arr.setflags(write=False)
    return arr


def monomials(q: np.ndarray, n: int) -> np.ndarray:
    """``Q^alpha = a^alpha1 b^alpha2 c^alpha3 d^alpha4`` for each packed alpha;
    ``q`` has shape (..., 4); result (..., K).  These are the packed entries of
    the tensor power ``Q^{(.)n}`` (Section 3.1)."""
    q = np.asarray(q, dtype=np.float64)
    al = multi_indices(n)
    out = np.ones(q.shape[:-1] + (len(al),))
    for i in range(4):
        out *= q[..., i, None] ** al[:, i]
    return out


def unpack_symmetric(A: np.ndarray, n: int) -> np.ndarray:
    """Full ``4^n`` array of a packed symmetric tensor (brute-force helper)."""
    al = multi_indices(n)
    lookup = {tuple(a): k for k, a in enumerate(al)}
    full = np.zeros((4,) * n)
    for idx in itertools.product(range(4), repeat=n):
        cnt = [0, 0, 0, 0]
        for i in idx:
            cnt[i] += 1
        full[idx] = A[lookup[tuple(cnt)]]
    return full


def tensor_apply(A: np.ndarray, n: int, q: np.ndarray) -> float:
    """``A x^n = <A, x^{(.)n}> = sum_alpha mu_alpha A_alpha x^alpha``
    (Section 3.1)."""
    return float(np.dot(multiplicities(n) * A, monomials(q, n)))


def _safe_pow(q: np.ndarray, e: np.ndarray) -> np.ndarray:
    """prod_d q_d^e_d per row of exponents, with negative exponents giving 0
    (they only occur with a zero coefficient)."""
    return np.prod(np.where(e >= 0, q[None, :] ** np.maximum(e, 0), 0.0), axis=1)


def tensor_apply_nm1(A: np.ndarray, n: int, q: np.ndarray) -> np.ndarray:
    """``A x^{n-1}``: the vector with ``(A x^{n-1})_i = (1/n) d(A x^n)/dx_i``
    (Section 3.1, the gradient identity)."""
    q = np.asarray(q, dtype=np.float64)
    al = multi_indices(n)
    c = multiplicities(n) * np.asarray(A, dtype=np.float64)
    out = np.zeros(4)
    for i in range(4):
        e = al.copy()
        e[:, i] -= 1
        out[i] = np.sum(c * al[:, i] / n * _safe_pow(q, e))
    return out


def tensor_apply_nm2(A: np.ndarray, n: int, q: np.ndarray) -> np.ndarray:
    """``A x^{n-2}``: the 4x4 matrix with Hessian ``n (n-1) A x^{n-2}``."""
    q = np.asarray(q, dtype=np.float64)
    al = multi_indices(n)
    c = multiplicities(n) * np.asarray(A, dtype=np.float64)
    out = np.zeros((4, 4))
    for i in range(4):
        for j in range(4):
            e = al.copy()
            e[:, i] -= 1
            e[:, j] -= 1
            coef = al[:, i] * (al[:, j] - (1 if i == j else 0))
            out[i, j] = np.sum(c * coef / (n * (n - 1)) * _safe_pow(q, e))
    return out


def frobenius_norm(A: np.ndarray, n: int) -> float:
    """Frobenius norm over all ``4^n`` entries of a packed symmetric tensor."""
    return float(math.sqrt(np.dot(multiplicities(n), np.asarray(A) ** 2)))


# ----------------------------------------------------------------------------
# template geometry: mask, rotation, normalisation (Section 2, Algorithm 1)
# ----------------------------------------------------------------------------

def template_centre(L) -> np.ndarray:
    return np.array([int(l) // 2 for l in L], dtype=np.int64)


def rotate_trilinear(t: np.ndarray, q) -> np.ndarray:
    """``t_R(u) = t(c + R^-1 (u - c))`` sampled trilinearly, zero outside the
    box (Section 2: ``t_R = O_{R^-1}(t)``)."""
    t = np.asarray(t, dtype=np.float64)
    L = np.array(t.shape)
    c = template_centre(L).astype(np.float64)
    r_inv = quat_to_matrix(q).T
    grids = np.meshgrid(*[np.arange(l, dtype=np.float64) for l in L], indexing="ij")
    u = np.stack(grids, axis=-1) - c
    p = u @ r_inv.T + c                      # p = c + R^-1 (u - c)
    p0 = np.floor(p)
    fr = p - p0
    p0 = p0.astype(np.int64)
    out = np.zeros(t.shape)
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                idx = p0 + np.array([dz, dy, dx])
                wgt = ((fr[..., 0] if dz else 1 - fr[..., 0]) *
                       (fr[..., 1] if dy else 1 - fr[..., 1]) *
                       (fr[..., 2] if dx else 1 - fr[..., 2]))
                inside = np.all((idx >= 0) & (idx < L), axis=-1)
                vals = np.zeros(t.shape)
                ii = idx[inside]
                vals[inside] = t[ii[:, 0], ii[:, 1], ii[:, 2]]
                out += wgt * vals
    return out


def masked_normalize(g: np.ndarray, m: np.ndarray) -> np.ndarray:
    """``m * (g - <g,m>/m_sum) / sqrt(<g^2,m> - <g,m>^2/m_sum)``: the template
    made S-orthogonal to the constant image and of unit S-norm, then passed
    through ``S`` (Algorithm 1, template pre-processing; Section 2, closed form
    of ``m (h * P_S(t) / ||P_S(t)||_S)``)."""
    g = np.asarray(g, dtype=np.float64)
    m = np.asarray(m, dtype=np.float64)
    msum = m.sum()
    if not msum > 0:
        raise ValueError("mask has no mass")
    s1 = float((g * m).sum())
    s2 = float((g * g * m).sum())
    var = s2 - s1 * s1 / msum
    if not var > 0:
        raise ValueError("template has zero variance under the mask")
    return m * (g - s1 / msum) / math.sqrt(var)


def rotated_template(t, m, q) -> np.ndarray:
    """``s_R``: raw template rotated by ``R(q)``, then normalised under ``m``."""
    return masked_normalize(rotate_trilinear(t, q), m)


# ----------------------------------------------------------------------------
# direct spatial correlation and local normalisation (Section 2)
# ----------------------------------------------------------------------------

def valid_region(N, L) -> tuple:
    """Inclusive-exclusive bounds ``[lo, hi)`` per axis of the positions whose
    template window lies inside the image."""
    c = template_centre(L)
    lo = c
    hi = np.array(N) - np.array(L) + c + 1
    return lo, hi


def valid_mask(N, L) -> np.ndarray:
    lo, hi = valid_region(N, L)
    out = np.zeros(tuple(N), dtype=bool)
    out[lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]] = True
    return out


def windows(f: np.ndarray, xs: np.ndarray, L) -> np.ndarray:
    """``W[p, u] = f((x_p + u - c) mod N)`` for the positions ``xs`` (P, 3):
    the translated image ``tau_x f`` restricted to the template box."""
    f = np.asarray(f, dtype=np.float64)
    N = np.array(f.shape)
    c = template_centre(L)
    xs = np.asarray(xs, dtype=np.int64).reshape(-1, 3)
    i0 = (xs[:, 0, None] + np.arange(L[0]) - c[0]) % N[0]
    i1 = (xs[:, 1, None] + np.arange(L[1]) - c[1]) % N[1]
    i2 = (xs[:, 2, None] + np.arange(L[2]) - c[2]) % N[2]
    return f[i0[:, :, None, None], i1[:, None, :, None], i2[:, None, None, :]]


def correlate_at(f: np.ndarray, g: np.ndarray, xs: np.ndarray,
                 chunk: int = 512) -> np.ndarray:
    """Cross-correlation ``(f * g)(x) = sum_u f(x + u - c) g(u)`` (Section 2,
    eq. "correlation") at positions ``xs``; ``g`` is one template (L^3) or a
    stack (K, L^3).  Returns (P,) or (P, K)."""
    g = np.asarray(g, dtype=np.float64)
    single = g.ndim == 3
    gs = g[None] if single else g
    L = gs.shape[1:]
    xs = np.asarray(xs, dtype=np.int64).reshape(-1, 3)
    out = np.empty((len(xs), gs.shape[0]))
    gm = gs.reshape(gs.shape[0], -1).T
    for s in range(0, len(xs), chunk):
        w = windows(f, xs[s:s + chunk], L).reshape(-1, gm.shape[0])
        out[s:s + chunk] = w @ gm
    return out[:, 0] if single else out


def local_norm_at(f: np.ndarray, m: np.ndarray, xs: np.ndarray,
                  eps_v: float = EPS_V_DEFAULT, chunk: int = 512) -> np.ndarray:
    """``w(x) = 1 / ||P_S tau_x f||_S`` (Section 2) by the two-pass definition:
    masked mean ``mu_x``, then ``v_x = sum_u m(u) (f(x+u-c) - mu_x)^2``; ``w = 0``
    where ``v_x <= eps_v * m_sum * var(f)``."""
    f = np.asarray(f, dtype=np.float64)
    m = np.asarray(m, dtype=np.float64)
    msum = m.sum()
    floor = eps_v * msum * float(f.var())
    xs = np.asarray(xs, dtype=np.int64).reshape(-1, 3)
    out = np.empty(len(xs))
    mv = m.reshape(-1)
    for s in range(0, len(xs), chunk):
        w = windows(f, xs[s:s + chunk], m.shape).reshape(-1, mv.size)
        mu = (w @ mv) / msum
        v = ((w - mu[:, None]) ** 2) @ mv
        out[s:s + chunk] = np.where(v > floor, 1.0 / np.sqrt(np.maximum(v, 1e-300)), 0.0)
    return out


def all_positions(N) -> np.ndarray:
    g = np.meshgrid(*[np.arange(n) for n in N], indexing="ij")
    return np.stack([x.reshape(-1) for x in g], axis=1)


# ----------------------------------------------------------------------------
# classical template matching (Algorithm 1 with a loop over rotations)
# ----------------------------------------------------------------------------

def classical_ncc_at(f, t, m, quats, xs, eps_v: float = EPS_V_DEFAULT):
    """``c(x, R_j) = w(x) (f * s_{R_j})(x)`` for every rotation (Section 2,
    eq. for c(x,R); Algorithm 1).  Returns the (P, J) matrix."""
    s = np.stack([rotated_template(t, m, q) for q in quats])
    corr = correlate_at(f, s, xs)
    w = local_norm_at(f, m, xs, eps_v)
    return corr * w[:, None]


def classical_best_at(f, t, m, quats, xs, eps_v: float = EPS_V_DEFAULT):
    """Per position the largest NCC over the rotation list and its index
    (lowest index on ties)."""
    c = classical_ncc_at(f, t, m, quats, xs, eps_v)
    idx = np.argmax(c, axis=1)        # first maximum
    return c[np.arange(len(c)), idx], idx


# ----------------------------------------------------------------------------
# tensor template, tensor field, score (Section 3.2, 3.4)
# ----------------------------------------------------------------------------

def tensor_template(t, m, n: int, quats, weights) -> np.ndarray:
    """Packed tensor template ``T_alpha(u) = sum_j omega_j Q_j^alpha s_{R_j}(u)``:
    the quadrature form of ``T(z) = int R^{(.)n} S(t)_R(z) dR`` (Section 3.2)."""
    if n < 2 or n % 2:
        raise ValueError("tensor order must be even and >= 2")
    quats = np.asarray(quats, dtype=np.float64)
    weights = np.asarray(weights, dtype=np.float64)
    K = num_components(n)
    T = np.zeros((K,) + tuple(np.shape(t)))
    mono = monomials(quats / np.linalg.norm(quats, axis=1, keepdims=True), n)
    for j, q in enumerate(quats):
        s = rotated_template(t, m, q)
        T += (weights[j] * mono[j])[:, None, None, None] * s[None]
    return T


def tensor_field_at(f, T, m, xs, eps_v: float = EPS_V_DEFAULT) -> np.ndarray:
    """``C_alpha(x) = w(x) <tau_x f, T_alpha>`` (Section 3.2): (P, K)."""
    corr = correlate_at(f, T, xs)
    w = local_norm_at(f, m, xs, eps_v)
    return corr * w[:, None]


def score_from_field(C: np.ndarray, n: int) -> np.ndarray:
    """Frobenius norm of each packed ``C_n(x)`` (Section 3.4)."""
    C = np.asarray(C, dtype=np.float64)
    return np.sqrt(C ** 2 @ multiplicities(n))


def score_map(f, T, m, n: int, eps_v: float = EPS_V_DEFAULT,
              chunk: int = 512) -> np.ndarray:
    """Frobenius score ``F(x) = ||C_n(x)||_F`` over the whole image; zero
    outside the valid region."""
    f = np.asarray(f, dtype=np.float64)
    N = f.shape
    L = T.shape[1:]
    vm = valid_mask(N, L)
    xs = np.argwhere(vm)
    out = np.zeros(N)
    vals = np.empty(len(xs))
    for s in range(0, len(xs), chunk * 8):
        C = tensor_field_at(f, T, m, xs[s:s + chunk * 8], eps_v)
        vals[s:s + chunk * 8] = score_from_field(C, n)
    out[vm] = vals
    return out


def w_map(f, m, eps_v: float = EPS_V_DEFAULT) -> np.ndarray:
    """``w(x)`` over the whole image; zero outside the valid region."""
    N = np.shape(f)
    vm = valid_mask(N, np.shape(m))
    out = np.zeros(N)
    out[vm] = local_norm_at(f, m, np.argwhere(vm), eps_v)
    return out


# ----------------------------------------------------------------------------
# candidate positions (Section 3.4: Frobenius norm as the position proxy)
# ----------------------------------------------------------------------------

def find_peaks(F: np.ndarray, L, threshold: float, min_dist: float,
               max_peaks: int) -> np.ndarray:
    """Candidates are valid-region voxels strictly above all 26 neighbours and
    above ``threshold``; sorted by score (descending, ties by lower linear
    index); greedy suppression of any candidate within Euclidean distance
    ``min_dist`` of an accepted one; at most ``max_peaks`` kept.  Returns
    (P, 3) int64 positions in acceptance order."""
    F = np.asarray(F)
    N = F.shape
    lo, hi = valid_region(N, L)
    cands = []
    for x0 in range(lo[0], hi[0]):
        for x1 in range(lo[1], hi[1]):
            for x2 in range(lo[2], hi[2]):
                v = F[x0, x1, x2]
                if not v > threshold:
                    continue
                ok = True
                for d0 in (-1, 0, 1):
                    for d1 in (-1, 0, 1):
                        for d2 in (-1, 0, 1):
                            if d0 == d1 == d2 == 0:
                                continue
                            y0, y1, y2 = x0 + d0, x1 + d1, x2 + d2
                            if 0 <= y0 < N[0] and 0 <= y1 < N[1] and 0 <= y2 < N[2]:
                                if not v > F[y0, y1, y2]:
                                    ok = False
                    if not ok:
                        break
                if ok:
                    cands.append((v, (x0 * N[1] + x1) * N[2] + x2, (x0, x1, x2)))
    cands.sort(key=lambda e: (-e[0], e[1]))
    acc = []
    for v, lin, p in cands:
        if len(acc) >= max_peaks:
            break
        if all((p[0] - a[0]) ** 2 + (p[1] - a[1]) ** 2 + (p[2] - a[2]) ** 2
               >= min_dist * min_dist for a in acc):
            acc.append(p)
    return np.array(acc, dtype=np.int64).reshape(-1, 3)


def find_peaks_fast(F: np.ndarray, L, threshold: float, min_dist: float,
                    max_peaks: int) -> np.ndarray:
    """Same result as :func:`find_peaks`, with the local-maximum test done by
    array comparisons (for larger maps)."""
    F = np.asarray(F)
    N = F.shape
    lo, hi = valid_region(N, L)
    is_max = np.zeros(N, dtype=bool)
    sub = (slice(lo[0], hi[0]), slice(lo[1], hi[1]), slice(lo[2], hi[2]))
    core = F[sub]
    ok = core > threshold
    pad = np.pad(F, 1, mode="constant", constant_values=-np.inf)
    for d0 in (-1, 0, 1):
        for d1 in (-1, 0, 1):
            for d2 in (-1, 0, 1):
                if d0 == d1 == d2 == 0:
                    continue
                nb = pad[lo[0] + 1 + d0:hi[0] + 1 + d0,
                         lo[1] + 1 + d1:hi[1] + 1 + d1,
                         lo[2] + 1 + d2:hi[2] + 1 + d2]
                ok &= core > nb
    is_max[sub] = ok
    pts = np.argwhere(is_max)
    vals = F[is_max]
    lin = (pts[:, 0] * N[1] + pts[:, 1]) * N[2] + pts[:, 2]
    order = np.lexsort((lin, -vals))
    acc = []
    d2min = min_dist * min_dist
    for k in order:
        if len(acc) >= max_peaks:
            break
        p = pts[k]
        if all(((p - a) ** 2).sum() >= d2min for a in acc):
            acc.append(p)
    return np.array(acc, dtype=np.int64).reshape(-1, 3)


# ----------------------------------------------------------------------------
# rotation at a candidate: dominant Z-eigenpair (Section 3.3, Theorem "main";
# Section 3.1, eq. "Zeigen"; Section 3.4, SS-HOPM)
# ----------------------------------------------------------------------------

def sshopm(A: np.ndarray, n: int, q0, tol: float = 1e-14,
           max_iter: int = 20000, tau: float = 1e-6):
    """Shifted symmetric higher-order power method for ``max A x^n`` on the
    unit sphere: ``x <- (A x^{n-1} + alpha x) / ||.||`` with the shift chosen at
    each step so that ``(1/n) A x^n + (alpha/2)||x||^2`` is locally convex,
    ``alpha = max(0, tau - (n-1) lambda_min(A x^{n-2}))``.  Stops when
    ``|delta lambda| <= tol * max(1, |lambda|)``.  Returns (x, lambda, iters,
    converged)."""
    x = np.asarray(q0, dtype=np.float64)
    x = x / np.linalg.norm(x)
    lam = tensor_apply(A, n, x)
    for it in range(1, max_iter + 1):
        hmin = float(np.linalg.eigvalsh(tensor_apply_nm2(A, n, x))[0])
        alpha = max(0.0, tau - (n - 1) * hmin)
        y = tensor_apply_nm1(A, n, x) + alpha * x
        x = y / np.linalg.norm(y)
        new = tensor_apply(A, n, x)
        if abs(new - lam) <= tol * max(1.0, abs(new)):
            return x, new, it, True
        lam = new
    return x, lam, max_iter, False


def oracle_sphere_points(count: int) -> np.ndarray:
    """Dense near-uniform set on S^3 (super-Fibonacci spiral, Alexa 2022) used
    for the brute-force search."""
    phi = math.sqrt(2.0)
    psi = 1.533751168755204288118041
    s = np.arange(count, dtype=np.float64) + 0.5
    r = np.sqrt(s / count)
    rr = np.sqrt(1.0 - s / count)
    a = 2.0 * np.pi * s / phi
    b = 2.0 * np.pi * s / psi
    return np.stack([r * np.sin(a), r * np.cos(a), rr * np.sin(b), rr * np.cos(b)], axis=1)


def dominant_z_eigenpair(A: np.ndarray, n: int, n_brute: int = 200000,
                         n_polish: int = 4):
    """Global maximiser of ``phi(Q) = A Q^n`` on S^3: brute force over a dense
    point set, then SS-HOPM polish from the best few points.  Returns
    (q canonical, lambda, second_best_lambda_far) where the last is the best
    polished value at least 5 degrees away (for ambiguity checks)."""
    pts = oracle_sphere_points(n_brute)
    vals = monomials(pts, n) @ (multiplicities(n) * A)
    order = np.argsort(-vals)
    polished = []
    seen = []
    for k in order:
        p = pts[k]
        if any(rotation_angle_deg(p, s) < 10.0 for s in seen):
            continue
        seen.append(p)
        x, lam, _, _ = sshopm(A, n, p)
        polished.append((lam, quat_canonical(x)))
        if len(seen) >= n_polish:
            break
    polished.sort(key=lambda e: -e[0])
    best_lam, best_q = polished[0]
    second = -np.inf
    for lam, q in polished[1:]:
        if rotation_angle_deg(q, best_q) > 5.0:
            second = max(second, lam)
    return best_q, best_lam, second


def rotation_map_at(f, T, m, n: int, xs, eps_v: float = EPS_V_DEFAULT,
                    n_brute: int = 100000):
    """The rotation at each listed voxel rather than only at peaks (Section
    3.4 read at every position, with Theorem "main"): the dominant
    Z-eigenpair of ``C_n(x)`` (eq. "Zeigen").  Returns (q (P, 4) canonical,
    lambda (P,), second (P,)) with ``second`` as in ``dominant_z_eigenpair``.
    Where ``C_n(x) = 0`` (``w(x) = 0``) every ``Q`` attains ``phi = 0``: the map
    holds the identity with ``lambda = 0`` (and ``second = 0``)."""
    C = tensor_field_at(f, T, m, np.asarray(xs), eps_v)
    P = len(C)
    qs = np.zeros((P, 4))
    lams = np.zeros(P)
    secs = np.zeros(P)
    for p in range(P):
        if not np.any(C[p]):
            qs[p] = (1.0, 0.0, 0.0, 0.0)
            continue
        qs[p], lams[p], secs[p] = dominant_z_eigenpair(C[p], n, n_brute=n_brute)
    return qs, lams, secs


def neighbourhood_offsets() -> np.ndarray:
    """The 27 offsets of a 3x3x3 neighbourhood, index k = 9 (d0+1) + 3 (d1+1) + (d2+1)."""
    return np.array([(k // 9 - 1, (k // 3) % 3 - 1, k % 3 - 1) for k in range(27)], dtype=np.int64)


def refine_by_eigenvalue(f, T, m, n: int, x, eps_v: float = EPS_V_DEFAULT,
                         n_brute: int = 100000):
    """Reading of Section 3.4: the Frobenius norm stands in for the spectral
    norm ``||C_n(x)||_sigma = max_Q |C_n(x) Q^n|``; a candidate position is moved
    to the voxel of its 3x3x3 neighbourhood (inside the valid region) whose
    dominant Z-eigenvalue is largest (the centre first on ties, then the lower
    neighbour index).  Returns (position, q, lambda, lambdas of the 27 voxels)."""
    N = np.shape(f)
    L = np.shape(T)[1:]
    lo, hi = valid_region(N, L)
    offs = neighbourhood_offsets()
    lams = np.full(27, -np.inf)
    qs = np.zeros((27, 4))
    for k, o in enumerate(offs):
        y = np.asarray(x) + o
        if np.any(y < lo) or np.any(y >= hi):
            continue
        C = tensor_field_at(f, T, m, y[None], eps_v)[0]
        q, lam, _ = dominant_z_eigenpair(C, n, n_brute=n_brute)
        lams[k] = lam
        qs[k] = q
    best = 13
    for k in range(27):
        if lams[k] > lams[best]:
            best = k
    return np.asarray(x) + offs[best], qs[best], lams[best], lams


def refine_by_ncc(f, t, m, T, n: int, x, eps_v: float = EPS_V_DEFAULT,
                  n_brute: int = 100000):
    """A second reading of Section 3.4's position selection: each voxel y of the
    3x3x3 neighbourhood of a candidate (inside the valid region) gets its own
    rotation, the dominant Z-eigenvector q_y of C_n(y) (Theorem "main"), and the
    classical NCC at that rotation, c(y, R(q_y)) (Section 2, the normalised
    correlation of Algorithm 1).  The candidate moves to the voxel with the
    largest such NCC (the centre first on ties, then the lower neighbour
    index).  Returns (position, q, lambda, ncc, the 27 NCC values)."""
    N = np.shape(f)
    L = np.shape(T)[1:]
    lo, hi = valid_region(N, L)
    offs = neighbourhood_offsets()
    nccs = np.full(27, -np.inf)
    qs = np.zeros((27, 4))
    lams = np.full(27, -np.inf)
    for k, o in enumerate(offs):
        y = np.asarray(x) + o
        if np.any(y < lo) or np.any(y >= hi):
            continue
        C = tensor_field_at(f, T, m, y[None], eps_v)[0]
        q, lam, _ = dominant_z_eigenpair(C, n, n_brute=n_brute)
        qs[k] = q
        lams[k] = lam
        nccs[k] = classical_ncc_at(f, t, m, q[None], y[None], eps_v)[0, 0]
    best = 13
    for k in range(27):
        if nccs[k] > nccs[best]:
            best = k
    return np.asarray(x) + offs[best], qs[best], lams[best], nccs[best], nccs


def refine_by_ncc_iterated(f, t, m, T, n: int, x, eps_v: float = EPS_V_DEFAULT,
                           n_brute: int = 100000, max_rounds: int = 4, trace=None):
    """The NCC refinement of :func:`refine_by_ncc` repeated from its own result
    until the position no longer moves, at most ``max_rounds`` times (a hill
    climb on the NCC at each voxel's own rotation, for Frobenius-score peaks
    more than one voxel from the copy's centre).  Returns (position, q,
    lambda, ncc, rounds taken).  ``trace`` (a list, optional) receives the
    start position and the 27 NCC values of every round."""
    x = np.asarray(x)
    for r in range(1, max_rounds + 1):
        pos, q, lam, ncc, nccs = refine_by_ncc(f, t, m, T, n, x, eps_v, n_brute)
        if trace is not None:
            trace.append((x.copy(), nccs))
        if np.array_equal(pos, x) or r == max_rounds:
            return pos, q, lam, ncc, r
        x = pos
    raise ValueError("max_rounds must be >= 1")


# ----------------------------------------------------------------------------
# gradient of the Frobenius score at fixed positions: the adjoint of the whole
# forward path (rotation, masked normalisation, tensor accumulation, window
# correlation, local normalisation, Frobenius norm), written out by the chain
# rule in float64
# ----------------------------------------------------------------------------

def rotate_trilinear_adjoint(h: np.ndarray, q, L) -> np.ndarray:
    """Adjoint of :func:`rotate_trilinear` in its template argument: the array
    ``a`` with ``<rotate_trilinear(t, q), h> = <t, a>`` for every ``t`` (each
    sample's weight scattered back to its eight corners)."""
    h = np.asarray(h, dtype=np.float64)
    L = np.array(L)
    c = template_centre(L).astype(np.float64)
    r_inv = quat_to_matrix(q).T
    grids = np.meshgrid(*[np.arange(l, dtype=np.float64) for l in L], indexing="ij")
    u = np.stack(grids, axis=-1) - c
    p = u @ r_inv.T + c
    p0 = np.floor(p)
    fr = p - p0
    p0 = p0.astype(np.int64)
    out = np.zeros(tuple(L))
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                idx = p0 + np.array([dz, dy, dx])
                wgt = ((fr[..., 0] if dz else 1 - fr[..., 0]) *
                       (fr[..., 1] if dy else 1 - fr[..., 1]) *
                       (fr[..., 2] if dx else 1 - fr[..., 2]))
                inside = np.all((idx >= 0) & (idx < L), axis=-1)
                ii = idx[inside]
                np.add.at(out, (ii[:, 0], ii[:, 1], ii[:, 2]), (wgt * h)[inside])
    return out


def score_at(f, t, m, n: int, quats, weights, xs, eps_v: float = EPS_V_DEFAULT) -> np.ndarray:
    """``F(x)`` at the positions ``xs`` from the raw template: tensor template
    (Section 3.2), tensor field and Frobenius norm (Section 3.4); 0 outside
    the valid region, where the score is not defined."""
    T = tensor_template(t, m, n, quats, weights)
    xs = np.asarray(xs, dtype=np.int64).reshape(-1, 3)
    lo, hi = valid_region(np.shape(f), np.shape(t))
    inside = np.all((xs >= lo) & (xs < hi), axis=1)
    return np.where(inside, score_from_field(tensor_field_at(f, T, m, xs, eps_v), n), 0.0)


def score_grad(f, t, m, n: int, quats, weights, xs, grad_F, eps_v: float = EPS_V_DEFAULT):
    """Gradient of ``sum_p grad_F[p] F(x_p)`` with respect to the raw template
    ``t`` and the image ``f``.  With ``C = w G``, ``G_alpha = <tau_x f,
    T_alpha>``, ``F = sqrt(sum mu C^2)``:

    * ``dF/dC_alpha = mu_alpha C_alpha / F``;
    * ``d/dT_alpha(u) = sum_p dC_alpha(p) w_p (tau_{x_p} f)(u)``;
    * ``d/df`` on each window: ``w_p sum_alpha dC_alpha T_alpha(u)
      - w_p^3 m(u) (f - mu_p) sum_alpha dC_alpha G_alpha`` (from
      ``dw/df = -w^3 m (f - mu)``, Section 2's local norm);
    * through ``T_alpha = sum_j omega_j Q_j^alpha s_j``, ``s = m (g - mu)/sigma``
      of the rotated template ``g``: ``dg = (m/sigma)(h - H1/M - (g - mu)
      H2/sigma^2)`` with ``h = omega_j sum_alpha Q_j^alpha dT_alpha``,
      ``H1 = sum m h``, ``H2 = sum m h (g - mu)``, ``M = sum m``; then the
      adjoint of the trilinear rotation.

    Positions outside the valid region (where F is 0 by definition), or where
    ``w = 0`` (the variance floor) or ``F = 0``, contribute nothing.  Returns
    (grad_t, grad_f)."""
    f = np.asarray(f, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    m = np.asarray(m, dtype=np.float64)
    quats = np.asarray(quats, dtype=np.float64)
    weights = np.asarray(weights, dtype=np.float64)
    xs = np.asarray(xs, dtype=np.int64).reshape(-1, 3)
    grad_F = np.asarray(grad_F, dtype=np.float64).reshape(-1)
    L = np.shape(t)
    N = np.shape(f)
    c = template_centre(L)
    mu_n = multiplicities(n)
    T = tensor_template(t, m, n, quats, weights)
    K = T.shape[0]
    Tf = T.reshape(K, -1)
    W = windows(f, xs, L).reshape(len(xs), -1)
    mv = m.reshape(-1)
    msum = mv.sum()
    mean = (W * mv).sum(axis=1) / msum
    var = ((W - mean[:, None]) ** 2 * mv).sum(axis=1)
    floor = eps_v * msum * float(f.var())
    w = np.where(var > floor, 1.0 / np.sqrt(np.maximum(var, 1e-300)), 0.0)
    G = W @ Tf.T
    C = G * w[:, None]
    F = np.sqrt(C ** 2 @ mu_n)
    lo, hi = valid_region(N, L)
    inside = np.all((xs >= lo) & (xs < hi), axis=1)
    ok = inside & (w > 0) & (F > 0)
    w = np.where(ok, w, 0.0)
    dC = np.where(ok[:, None], grad_F[:, None] * mu_n[None] * C / np.where(F > 0, F, 1.0)[:, None], 0.0)
    # template tensor
    dT = (dC * w[:, None]).T @ W                                   # (K, L^3)
    # image: each window's gradient scattered back
    grad_f = np.zeros(N)
    a = (dC * G).sum(axis=1)
    b = dC @ Tf
    dW = w[:, None] * b - (w ** 3)[:, None] * mv[None] * (W - mean[:, None]) * a[:, None]
    for p, x in enumerate(xs):
        i0 = (x[0] + np.arange(L[0]) - c[0]) % N[0]
        i1 = (x[1] + np.arange(L[1]) - c[1]) % N[1]
        i2 = (x[2] + np.arange(L[2]) - c[2]) % N[2]
        grad_f[np.ix_(i0, i1, i2)] += dW[p].reshape(L)
    # raw template through the rotations and the masked normalisation
    mono = monomials(quats / np.linalg.norm(quats, axis=1, keepdims=True), n)
    grad_t = np.zeros(L)
    for j, q in enumerate(quats):
        g = rotate_trilinear(t, q).reshape(-1)
        s1 = (mv * g).sum()
        mu_j = s1 / msum
        sig = math.sqrt((mv * g * g).sum() - s1 * s1 / msum)
        h = weights[j] * (mono[j] @ dT)
        H1 = (mv * h).sum()
        H2 = (mv * h * (g - mu_j)).sum()
        dg = mv / sig * (h - H1 / msum - (g - mu_j) * H2 / sig ** 2)
        grad_t += rotate_trilinear_adjoint(dg.reshape(L), q, L)
    return grad_t, grad_f


# ----------------------------------------------------------------------------
# isotropic low-pass filter and soft mask (Section 2: matching is applied to
# f * h and t * h for an isotropic low-pass h with h * 1 = 1, under a
# rotationally symmetric mask that is 1 inside one radius and 0 outside a
# slightly larger one)
# ----------------------------------------------------------------------------

def lowpass_kernel(sigma: float) -> np.ndarray:
    """Reading of the unspecified filter: a sampled Gaussian of standard
    deviation ``sigma`` voxels on ``k = -R..R``, ``R = ceil(3 sigma)``,
    normalised to unit sum (so ``h * 1 = 1``); ``sigma = 0`` is the identity.
    The 3-D filter is its product along the three axes."""
    if sigma < 0:
        raise ValueError("sigma must be >= 0")
    if sigma == 0:
        return np.ones(1)
    R = int(math.ceil(3.0 * sigma))
    k = np.arange(-R, R + 1, dtype=np.float64)
    h = np.exp(-0.5 * (k / sigma) ** 2)
    return h / h.sum()


def lowpass(f: np.ndarray, sigma: float, periodic: bool = True) -> np.ndarray:
    """``f * h`` with the filter of :func:`lowpass_kernel`, one axis at a
    time: ``out(x) = sum_k h(k) f(x - k)``, indices taken modulo the extent
    (``periodic``, as the FFT correlation treats the image) or with ``f = 0``
    outside the array (the template box)."""
    h = lowpass_kernel(sigma)
    R = (len(h) - 1) // 2
    out = np.asarray(f, dtype=np.float64)
    for axis in range(out.ndim):
        n = out.shape[axis]
        acc = np.zeros_like(out)
        for i, k in enumerate(range(-R, R + 1)):
            src = np.arange(n) - k
            if periodic:
                acc += h[i] * np.take(out, src % n, axis=axis)
            else:
                ok = (src >= 0) & (src < n)
                shape = [1] * out.ndim
                shape[axis] = n
                acc += h[i] * np.take(out, np.clip(src, 0, n - 1), axis=axis) * ok.reshape(shape)
        out = acc
    return out


def soft_mask(L, r_in: float, r_out: float) -> np.ndarray:
    """Rotationally symmetric mask about the template centre: 1 for
    ``||u - c|| <= r_in``, 0 for ``>= r_out``, a raised cosine in between."""
    L = (L, L, L) if np.isscalar(L) else tuple(L)
    c = template_centre(L)
    g = np.meshgrid(*[np.arange(l) - c[i] for i, l in enumerate(L)], indexing="ij")
    r = np.sqrt(g[0] ** 2 + g[1] ** 2 + g[2] ** 2)
    t = np.clip((r - r_in) / (r_out - r_in), 0.0, 1.0)
    return 0.5 * (1.0 + np.cos(np.pi * t))


# ----------------------------------------------------------------------------
# S'-consistent normalisation (Section 3.4, the false-positive discussion;
# S_2 and S' = S_2 S from the proof of Theorem "main")
# ----------------------------------------------------------------------------
#
# The tensor correlation is an inner product under S' = S_2 S, where S_2 is the
# convolution on SO(3) with the kernel K(P) = (P . I)^n = a_P^n of the
# polynomial features Q^{(.)n}, but it is normalised under S.  The
# S'-consistent score divides lambda by the S'-norms of the (S-normalised)
# window and template.  The paper states the quantity and no algorithm; the
# SO(3) integral of S_2 is taken with the tensor template's own quadrature
# {(Q_j, omega_j)}, and every rotated copy is re-normalised under the mask,
# as the rotated templates of the tensor template are:
#
#   D(h) = sum_j omega_j a_j^n <h~, N_m(I_{R_j} h~)>,
#   h~ = P_S h / ||P_S h||_S,  P_S h = h - <h,m>/m_sum,
#
# with I_R the trilinear rotation about the box centre and N_m the masked
# normalisation.  In the continuum D(h) = ||h~||^2_{S'}.  The S'-normalised
# score at a candidate x with dominant eigenvalue lambda(x) is
#
#   rho'(x) = lambda(x) / sqrt(D(tau_x f) D(t)),
#
# which lies in [-1, 1] where the discrete S' form is positive semidefinite
# (exactly so for a quadrature that is a finite rotation group with equal
# weights and grid-exact rotations) and is 1 at a noiseless copy.

SNORM_FLAT_REL = 1e-6


def s_prime_norm2(h, m, n: int, quats, weights) -> float:
    """``D(h)``: the squared S'-norm of the S-normalised box ``h`` (see the
    section comment).  A window whose masked variance is at most
    ``1e-6 sum m h^2`` is flat: NaN.  A rotated copy whose masked variance is at
    most ``1e-6`` of its masked second moment contributes 0."""
    h = np.asarray(h, dtype=np.float64)
    m = np.asarray(m, dtype=np.float64)
    msum = m.sum()
    mu = float((m * h).sum()) / msum
    g = h - mu
    v = float((m * g * g).sum())
    if not v > SNORM_FLAT_REL * float((m * h * h).sum()):
        return math.nan
    ht = g / math.sqrt(v)
    quats = np.asarray(quats, dtype=np.float64)
    quats = quats / np.linalg.norm(quats, axis=1, keepdims=True)
    D = 0.0
    for q, om in zip(quats, np.asarray(weights, dtype=np.float64)):
        r = rotate_trilinear(ht, q)
        s1 = float((m * r).sum())
        s2 = float((m * r * r).sum())
        var = s2 - s1 * s1 / msum
        if not var > SNORM_FLAT_REL * s2:
            continue
        nr = m * (r - s1 / msum) / math.sqrt(var)          # N_m(I_R h~)
        D += om * q[0] ** n * float((ht * nr).sum())
    return D


def s_prime_norms_at(f, t, m, n: int, quats, weights, xs):
    """``D`` of the image window ``tau_x f`` at each position of ``xs`` (which
    must lie in the valid region) and of the template: (Dx (P,), Dt)."""
    L = np.shape(t)
    W = windows(f, np.asarray(xs, dtype=np.int64).reshape(-1, 3), L)
    Dx = np.array([s_prime_norm2(W[p], m, n, quats, weights) for p in range(len(W))])
    return Dx, s_prime_norm2(t, m, n, quats, weights)


def s_prime_score(lam, Dx, Dt):
    """``rho' = lambda / sqrt(Dx Dt)``; 0 where either norm is not positive
    (a flat window, or a quadrature whose discrete S' form is not positive
    there)."""
    lam = np.asarray(lam, dtype=np.float64)
    Dx = np.asarray(Dx, dtype=np.float64)
    ok = (Dx > 0) & (Dt > 0)
    with np.errstate(invalid="ignore", divide="ignore"):
        return np.where(ok, lam / np.sqrt(np.where(ok, Dx * Dt, 1.0)), 0.0)


# ----------------------------------------------------------------------------
# two-dimensional TTM (Sections 2 and 3 with d = 2)
# ----------------------------------------------------------------------------
#
# Readings for d = 2 (Theorem "main" is stated for R^3 only):
# * a rotation R(z) of the plane is described by a unit complex number
#   z = (a, b) = e^{i theta / 2}, the half angle (the planar analogue of the
#   unit quaternion: z and -z give the same rotation, and an even order n makes
#   them equivalent); R(z) = [[a^2 - b^2, -2ab], [2ab, a^2 - b^2]] is the
#   rotation by theta = 2 atan2(b, a).  With the full angle (cos theta,
#   sin theta) instead, an even power of z . z' could not tell theta from
#   theta + pi;
# * C_n(x) in S^n(R^2), stored as its n + 1 entries C_k with multi-index
#   (n - k, k), multiplicity mu_k = C(n, k);
# * the image is C-order [n1][n2], the template box [L1][L2] with centre
#   c = L // 2 per axis, the SO(2) integral a quadrature {(z_j, omega_j)}.


def rot2_matrix(z) -> np.ndarray:
    """Rotation of the plane described by the unit complex number ``z``."""
    a, b = np.asarray(z, dtype=np.float64) / np.linalg.norm(z)
    return np.array([[a * a - b * b, -2 * a * b], [2 * a * b, a * a - b * b]])


def rotate_bilinear(t: np.ndarray, z) -> np.ndarray:
    """``t_R(u) = t(c + R^-1 (u - c))`` sampled bilinearly, zero outside the
    box (Section 2, ``t_R = O_{R^-1}(t)``, in the plane)."""
    t = np.asarray(t, dtype=np.float64)
    L = np.array(t.shape)
    c = np.array([int(l) // 2 for l in L], dtype=np.float64)
    r_inv = rot2_matrix(z).T
    g = np.meshgrid(*[np.arange(l, dtype=np.float64) for l in L], indexing="ij")
    u = np.stack(g, axis=-1) - c
    p = u @ r_inv.T + c
    p0 = np.floor(p)
    fr = p - p0
    p0 = p0.astype(np.int64)
    out = np.zeros(t.shape)
    for dy in (0, 1):
        for dx in (0, 1):
            idx = p0 + np.array([dy, dx])
            wgt = (fr[..., 0] if dy else 1 - fr[..., 0]) * (fr[..., 1] if dx else 1 - fr[..., 1])
            inside = np.all((idx >= 0) & (idx < L), axis=-1)
            vals = np.zeros(t.shape)
            ii = idx[inside]
            vals[inside] = t[ii[:, 0], ii[:, 1]]
            out += wgt * vals
    return out


def planar_multiplicities(n: int) -> np.ndarray:
    return np.array([math.comb(n, k) for k in range(n + 1)], dtype=np.float64)


def planar_monomials(zs: np.ndarray, n: int) -> np.ndarray:
    """``a^(n-k) b^k`` for k = 0..n per unit complex number: (J, n + 1)."""
    zs = np.asarray(zs, dtype=np.float64).reshape(-1, 2)
    zs = zs / np.linalg.norm(zs, axis=1, keepdims=True)
    k = np.arange(n + 1)
    return zs[:, :1] ** (n - k)[None] * zs[:, 1:] ** k[None]


def tensor_template_2d(t, m, n: int, zs, weights) -> np.ndarray:
    """``T_k(u) = sum_j omega_j a_j^(n-k) b_j^k s_{R_j}(u)``, k = 0..n, with
    ``s_R`` the raw template rotated by ``R(z_j)`` and normalised under ``m``
    (Section 3.2 with d = 2)."""
    if n < 2 or n % 2:
        raise ValueError("tensor order must be even and >= 2")
    mono = planar_monomials(zs, n)
    T = np.zeros((n + 1,) + tuple(np.shape(t)))
    for j, z in enumerate(np.asarray(zs, dtype=np.float64).reshape(-1, 2)):
        s = masked_normalize(rotate_bilinear(t, z), m)
        T += (weights[j] * mono[j])[:, None, None] * s[None]
    return T


def windows_2d(f: np.ndarray, xs: np.ndarray, L) -> np.ndarray:
    """``W[p, u] = f((x_p + u - c) mod N)`` in the plane: (P, L1, L2)."""
    f = np.asarray(f, dtype=np.float64)
    N = np.array(f.shape)
    c = [int(l) // 2 for l in L]
    xs = np.asarray(xs, dtype=np.int64).reshape(-1, 2)
    i0 = (xs[:, 0, None] + np.arange(L[0]) - c[0]) % N[0]
    i1 = (xs[:, 1, None] + np.arange(L[1]) - c[1]) % N[1]
    return f[i0[:, :, None], i1[:, None, :]]


def local_norm_at_2d(f, m, xs, eps_v: float = EPS_V_DEFAULT) -> np.ndarray:
    """``w(x) = 1 / ||P_S tau_x f||_S`` by the two-pass definition, with the
    floor of the 3-D case (``w = 0`` where ``v <= eps_v m_sum var(f)``)."""
    f = np.asarray(f, dtype=np.float64)
    m = np.asarray(m, dtype=np.float64)
    msum = m.sum()
    floor = eps_v * msum * float(f.var())
    W = windows_2d(f, xs, m.shape).reshape(len(np.reshape(xs, (-1, 2))), -1)
    mv = m.reshape(-1)
    mu = (W @ mv) / msum
    v = ((W - mu[:, None]) ** 2) @ mv
    return np.where(v > floor, 1.0 / np.sqrt(np.maximum(v, 1e-300)), 0.0)


def tensor_field_at_2d(f, T, m, xs, eps_v: float = EPS_V_DEFAULT) -> np.ndarray:
    """``C_k(x) = w(x) <tau_x f, T_k>``: (P, n + 1)."""
    T = np.asarray(T, dtype=np.float64)
    W = windows_2d(f, xs, T.shape[1:]).reshape(-1, T[0].size)
    return (W @ T.reshape(len(T), -1).T) * local_norm_at_2d(f, m, xs, eps_v)[:, None]


def score_from_field_2d(C: np.ndarray, n: int) -> np.ndarray:
    """Frobenius norm over all 2^n entries: ``sqrt(sum_k C(n,k) C_k^2)``."""
    C = np.asarray(C, dtype=np.float64)
    return np.sqrt((C * C) @ planar_multiplicities(n))


def tensor_apply_2d(C: np.ndarray, n: int, z) -> float:
    """``C z^n = sum_k C(n,k) C_k a^(n-k) b^k``."""
    return float(planar_monomials(np.asarray(z)[None], n)[0] @ (planar_multiplicities(n) * C))


def score_map_2d(f, T, m, n: int, eps_v: float = EPS_V_DEFAULT) -> np.ndarray:
    """``F(x)`` over the image's valid region (zero elsewhere)."""
    N = np.shape(f)
    L = np.shape(T)[1:]
    c = [l // 2 for l in L]
    out = np.zeros(N)
    g = np.meshgrid(np.arange(c[0], N[0] - L[0] + c[0] + 1), np.arange(c[1], N[1] - L[1] + c[1] + 1),
                    indexing="ij")
    xs = np.stack([g[0].reshape(-1), g[1].reshape(-1)], axis=1)
    out[xs[:, 0], xs[:, 1]] = score_from_field_2d(tensor_field_at_2d(f, T, m, xs, eps_v), n)
    return out


def classical_ncc_at_2d(f, t, m, zs, xs, eps_v: float = EPS_V_DEFAULT) -> np.ndarray:
    """``c(x, R_j) = w(x) <tau_x f, s_{R_j}>`` in the plane: (P, J)."""
    s = np.stack([masked_normalize(rotate_bilinear(t, z), m) for z in np.asarray(zs).reshape(-1, 2)])
    W = windows_2d(f, xs, np.shape(t)).reshape(-1, s[0].size)
    return (W @ s.reshape(len(s), -1).T) * local_norm_at_2d(f, m, xs, eps_v)[:, None]


def dominant_eigen_2d(C: np.ndarray, n: int, n_brute: int = 20000):
    """Global maximiser of ``phi(z) = C z^n`` on the unit circle: a brute-force
    scan of z = (cos psi, sin psi), psi in [0, pi) (z and -z are equivalent),
    then golden-section refinement around the best point.  Returns
    (z with a > 0 (or a = 0, b > 0), lambda, the best value at least 5 degrees
    of rotation away)."""
    mu = planar_multiplicities(n) * np.asarray(C, dtype=np.float64)
    k = np.arange(n + 1)

    def phi(psi):
        psi = np.asarray(psi, dtype=np.float64)
        return (np.cos(psi)[..., None] ** (n - k) * np.sin(psi)[..., None] ** k) @ mu

    grid = (np.arange(n_brute) + 0.5) * (math.pi / n_brute)
    vals = phi(grid)
    i = int(np.argmax(vals))
    h = math.pi / n_brute
    lo, hi = grid[i] - h, grid[i] + h
    g = (math.sqrt(5.0) - 1.0) / 2.0
    for _ in range(80):
        a1, a2 = hi - g * (hi - lo), lo + g * (hi - lo)
        if phi(a1) >= phi(a2):
            hi = a2
        else:
            lo = a1
    psi = 0.5 * (lo + hi)
    lam = float(phi(psi))
    z = np.array([math.cos(psi), math.sin(psi)])
    if z[0] < 0 or (z[0] == 0 and z[1] < 0):
        z = -z
    # rotation angle between psi and grid points: 2 |delta psi| (mod pi)
    d = np.abs(((grid - psi) + math.pi / 2) % math.pi - math.pi / 2) * 2.0
    far = d > math.radians(5.0)
    second = float(vals[far].max()) if np.any(far) else -np.inf
    return z, lam, second


def rotation_angle_2d_deg(z1, z2) -> float:
    """Angle of the plane rotation taking ``R(z1)`` to ``R(z2)``, in [0, 180]."""
    t1 = 2.0 * math.atan2(z1[1], z1[0])
    t2 = 2.0 * math.atan2(z2[1], z2[0])
    d = (t2 - t1 + math.pi) % (2.0 * math.pi) - math.pi
    return abs(math.degrees(d))


def find_peaks_2d(F: np.ndarray, L, threshold: float, min_dist: float, max_peaks: int) -> np.ndarray:
    """The candidate rule of the 3-D case in the plane: strict maxima over the
    8 neighbours inside the valid region, above ``threshold``, sorted by score
    (ties by lower linear index), greedy suppression within ``min_dist``, at
    most ``max_peaks``: (P, 2)."""
    F3 = np.asarray(F)[None]
    return find_peaks_fast(F3, (1,) + tuple(L), threshold, min_dist, max_peaks)[:, 1:]


def refine_by_ncc_2d(f, t, m, T, n: int, x, eps_v: float = EPS_V_DEFAULT):
    """The NCC refinement in the plane: each pixel y of the 3x3 neighbourhood
    (inside the valid region) gets its own rotation, the dominant eigenvector
    of C_n(y); the candidate moves to the pixel with the largest NCC at that
    rotation (the centre first on ties, then the lower index 3 (d1+1) +
    (d2+1)).  Returns (position, z, lambda, ncc)."""
    N = np.shape(f)
    L = np.shape(t)
    c = [l // 2 for l in L]
    offs = [(d1, d2) for d1 in (-1, 0, 1) for d2 in (-1, 0, 1)]
    best, res = None, None
    for k in [4] + [i for i in range(9) if i != 4]:
        y = np.asarray(x) + np.array(offs[k])
        if not all(c[i] <= y[i] <= N[i] - L[i] + c[i] for i in range(2)):
            continue
        C = tensor_field_at_2d(f, T, m, y[None], eps_v)[0]
        z, lam, _ = dominant_eigen_2d(C, n)
        ncc = float(classical_ncc_at_2d(f, t, m, z[None], y[None], eps_v)[0, 0])
        if best is None or ncc > best or (ncc == best and k < res[4] and res[4] != 4):
            best, res = ncc, (y, z, lam, ncc, k)
    return res[0], res[1], res[2], res[3]
