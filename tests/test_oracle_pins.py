"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: closed forms,
brute force over all 4^n tensor entries, a library FFT, exact grid rotations,
Cauchy-Schwarz, the planted-copy theorem, or values the paper prints.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import ttm_oracle as O
from paper_2311_07561_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rng(s):
    return np.random.default_rng(s)


# --------------------------------------------------------------------------
# packed symmetric tensors (Section 3.1)
# --------------------------------------------------------------------------

def test_paper_dimension_counts():
    facts = json.load(open(os.path.join(GOLDEN, "paper_facts.json")))
    assert O.num_components(4) == facts["dim_S4_R4"]["value"]
    assert len(O.multi_indices(4)) == facts["components_order4"]["value"]
    assert int(O.multiplicities(4).sum()) == facts["dim_T4_R4"]["value"]
    rot = facts["rotations_for_accuracy"]["value"]
    assert rot["13"] // O.num_components(4) == facts["speedup_13deg"]["value"]
    for n, k in [(2, 10), (4, 35), (6, 84), (8, 165)]:
        al = O.multi_indices(n)
        assert len(al) == k == O.num_components(n)
        assert len({tuple(a) for a in al}) == k
        assert np.all(al.sum(axis=1) == n) and np.all(al >= 0)
        assert int(O.multiplicities(n).sum()) == 4 ** n
    assert tuple(O.multi_indices(4)[0]) == (4, 0, 0, 0)
    assert tuple(O.multi_indices(4)[-1]) == (0, 0, 0, 4)


@pytest.mark.parametrize("n", [2, 4, 6])
def test_power_inner_product_identity(n):
    # x^{(.)n} . y^{(.)n} = (x . y)^n  (Section 3.1, multinomial theorem)
    r = _rng(n)
    for _ in range(5):
        x, y = r.standard_normal(4), r.standard_normal(4)
        packed = float(np.sum(O.multiplicities(n) * O.monomials(x, n) * O.monomials(y, n)))
        assert packed == pytest.approx(float(np.dot(x, y)) ** n, rel=1e-12, abs=1e-12)


@pytest.mark.parametrize("n", [2, 4])
def test_packed_norm_and_contraction_vs_all_entries(n):
    r = _rng(10 + n)
    A = r.standard_normal(O.num_components(n))
    full = O.unpack_symmetric(A, n)
    # symmetric under index permutation
    assert np.allclose(full, np.transpose(full, list(reversed(range(n)))))
    assert O.frobenius_norm(A, n) == pytest.approx(math.sqrt(float((full ** 2).sum())), rel=1e-13)
    x = r.standard_normal(4)
    brute = full
    for _ in range(n):
        brute = brute @ x
    assert O.tensor_apply(A, n, x) == pytest.approx(float(brute), rel=1e-12)
    v = full
    for _ in range(n - 1):
        v = v @ x
    assert np.allclose(O.tensor_apply_nm1(A, n, x), v, rtol=1e-12, atol=1e-12)
    M = full
    for _ in range(n - 2):
        M = M @ x
    assert np.allclose(O.tensor_apply_nm2(A, n, x), M, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("n", [2, 4, 6])
def test_gradient_identity_finite_differences(n):
    # grad (A x^n) = n A x^{n-1}  (Section 3.1)
    r = _rng(20 + n)
    A = r.standard_normal(O.num_components(n))
    x = r.standard_normal(4)
    h = 1e-6
    fd = np.array([(O.tensor_apply(A, n, x + h * e) - O.tensor_apply(A, n, x - h * e)) / (2 * h)
                   for e in np.eye(4)])
    assert np.allclose(fd, n * O.tensor_apply_nm1(A, n, x), rtol=1e-6, atol=1e-6)
    hfd = np.array([(O.tensor_apply_nm1(A, n, x + h * e) - O.tensor_apply_nm1(A, n, x - h * e)) / (2 * h)
                    for e in np.eye(4)]).T * n
    assert np.allclose(hfd, n * (n - 1) * O.tensor_apply_nm2(A, n, x), rtol=1e-5, atol=1e-5)


def _closed_form_moment(alpha):
    # E_{S^3}[prod Q_i^{2 b_i}] = prod (2 b_i - 1)!! / prod_{k<|b|} (4 + 2k); 0 if an exponent is odd
    if any(a % 2 for a in alpha):
        return 0.0
    b = [a // 2 for a in alpha]
    num = 1.0
    for bi in b:
        for k in range(1, 2 * bi, 2):
            num *= k
    den = 1.0
    for k in range(sum(b)):
        den *= 4 + 2 * k
    return num / den


def test_closed_form_moments_sanity():
    assert _closed_form_moment((2, 0, 0, 0)) == pytest.approx(0.25)
    assert _closed_form_moment((4, 0, 0, 0)) == pytest.approx(1 / 8)
    assert _closed_form_moment((2, 2, 0, 0)) == pytest.approx(1 / 24)
    assert _closed_form_moment((6, 0, 0, 0)) == pytest.approx(5 / 64)
    # Monte Carlo cross-check of the formula
    q = synth.random_quaternions(_rng(3), 400000)
    assert np.mean(q[:, 1] ** 2 * q[:, 2] ** 2) == pytest.approx(1 / 24, rel=0.03)
    # the binary octahedral group is a 7-design: group averages equal the moments
    g = synth.binary_octahedral()
    for n in (2, 4, 6):
        mono = O.monomials(g, n).mean(axis=0)
        ref = np.array([_closed_form_moment(tuple(a)) for a in O.multi_indices(n)])
        assert np.allclose(mono, ref, atol=1e-14)


# --------------------------------------------------------------------------
# quaternions and rotations (Section 2)
# --------------------------------------------------------------------------

def test_quaternion_matrix_is_hamilton_conjugation():
    r = _rng(5)
    for _ in range(10):
        q = r.standard_normal(4)
        q /= np.linalg.norm(q)
        v = r.standard_normal(3)
        qc = q * np.array([1, -1, -1, -1])
        rv = O.quat_mul(O.quat_mul(q, np.concatenate([[0.0], v])), qc)
        R = O.quat_to_matrix(q)
        assert abs(rv[0]) < 1e-13
        assert np.allclose(R @ v, rv[1:], atol=1e-13)
        assert np.allclose(R @ R.T, np.eye(3), atol=1e-13)
        assert np.linalg.det(R) == pytest.approx(1.0)
        p = r.standard_normal(4)
        p /= np.linalg.norm(p)
        assert np.allclose(O.quat_to_matrix(O.quat_mul(p, q)), O.quat_to_matrix(p) @ R, atol=1e-13)
    # unit quaternion inner product is Re(y^-1 x) (Section 2, eq. producto2)
    x, y = r.standard_normal(4), r.standard_normal(4)
    x /= np.linalg.norm(x)
    y /= np.linalg.norm(y)
    yinv = y * np.array([1, -1, -1, -1])
    assert O.quat_mul(yinv, x)[0] == pytest.approx(float(np.dot(x, y)))


def test_rotation_about_axis0_is_numpy_rot90():
    L = 9                             # odd: the centre L//2 is the array centre
    t = _rng(6).standard_normal((L, L, L))
    q = np.array([math.cos(math.pi / 4), math.sin(math.pi / 4), 0, 0])
    got = O.rotate_trilinear(t, q)
    assert np.allclose(got, np.rot90(t, 1, axes=(1, 2)), atol=1e-12)


def test_rotation_composition_on_exact_grid_rotations():
    # t_{R1 R2} = (t_{R2})_{R1}  (Section 2, composition of rotations)
    L = 10
    t = _rng(7).standard_normal((L, L, L))
    g = synth.binary_octahedral()
    r = _rng(8)
    for _ in range(6):
        q1, q2 = g[r.integers(len(g))], g[r.integers(len(g))]
        lhs = O.rotate_trilinear(t, O.quat_mul(q1, q2))
        rhs = O.rotate_trilinear(O.rotate_trilinear(t, q2), q1)
        # a 90-degree rotation about the centre can move part of an even box out of it
        keep = (np.abs(O.rotate_trilinear(np.ones_like(t), O.quat_mul(q1, q2)) - 1) < 1e-12) & \
               (np.abs(O.rotate_trilinear(O.rotate_trilinear(np.ones_like(t), q2), q1) - 1) < 1e-12)
        assert keep.sum() > 0.5 * t.size
        assert np.allclose(lhs[keep], rhs[keep], atol=1e-12)


def test_trilinear_reproduces_linear_functions():
    # trilinear interpolation is exact for affine functions away from the border
    L = 12
    ax = np.arange(L, dtype=np.float64)
    g = np.meshgrid(ax, ax, ax, indexing="ij")
    coef = np.array([0.3, -1.1, 0.7])
    t = 2.0 + coef[0] * g[0] + coef[1] * g[1] + coef[2] * g[2]
    q = synth.random_quaternions(_rng(9), 1)[0]
    got = O.rotate_trilinear(t, q)
    c = L // 2
    R = O.quat_to_matrix(q)
    u = np.stack(g, axis=-1) - c
    p = u @ R + c                                  # c + R^-1 (u - c)
    inside = np.all((p >= 0) & (p <= L - 1), axis=-1)
    expect = 2.0 + p @ coef
    assert inside.sum() > 100
    assert np.allclose(got[inside], expect[inside], atol=1e-11)


# --------------------------------------------------------------------------
# correlation and local normalisation (Section 2)
# --------------------------------------------------------------------------

def _fft_correlation(f, g):
    """Circular correlation by the library FFT: the template is wrapped so
    that its centre sits at the origin, then F^-1(F(f) conj F(g))."""
    N = f.shape
    L = g.shape
    c = O.template_centre(L)
    big = np.zeros(N)
    for u0 in range(L[0]):
        for u1 in range(L[1]):
            for u2 in range(L[2]):
                big[(u0 - c[0]) % N[0], (u1 - c[1]) % N[1], (u2 - c[2]) % N[2]] += g[u0, u1, u2]
    return np.real(np.fft.ifftn(np.fft.fftn(f) * np.conj(np.fft.fftn(big))))


def test_direct_correlation_equals_fft_and_loops():
    r = _rng(11)
    f = r.standard_normal((12, 10, 14))
    g = r.standard_normal((5, 4, 6))
    xs = O.all_positions(f.shape)
    direct = O.correlate_at(f, g, xs).reshape(f.shape)
    assert np.allclose(direct, _fft_correlation(f, g), atol=1e-11)
    # a few by explicit loops
    c = O.template_centre(g.shape)
    for x in [(0, 0, 0), (5, 3, 7), (11, 9, 13)]:
        s = 0.0
        for u0 in range(5):
            for u1 in range(4):
                for u2 in range(6):
                    s += f[(x[0] + u0 - c[0]) % 12, (x[1] + u1 - c[1]) % 10, (x[2] + u2 - c[2]) % 14] * g[u0, u1, u2]
        assert direct[x] == pytest.approx(s, abs=1e-12)


def test_local_norm_two_pass_equals_one_pass_fft():
    # ||P_S tau_x f||_S^2 = <(tau_x f)^2, m> - <tau_x f, m>^2 / <1, m>   (Section 2)
    r = _rng(12)
    f = 3.0 + r.standard_normal((14, 12, 10))
    m = synth.ball_mask(7, 3.5)
    m1 = _fft_correlation(f, m)
    m2 = _fft_correlation(f * f, m)
    v = m2 - m1 ** 2 / m.sum()
    xs = O.all_positions(f.shape)
    w = O.local_norm_at(f, m, xs).reshape(f.shape)
    assert np.allclose(w, 1.0 / np.sqrt(v), rtol=1e-9)


def test_local_norm_constant_window_is_zero():
    f = np.ones((12, 12, 12))
    f[0, 0, 0] = 5.0
    m = synth.ball_mask(4, 2.0)
    w = O.local_norm_at(f, m, np.array([[6, 6, 6]]))
    assert w[0] == 0.0


# --------------------------------------------------------------------------
# classical NCC (Theorem "similar", Theorem "ThCTM")
# --------------------------------------------------------------------------

def _random_setup(seed, N=(14, 14, 14), L=8):
    r = _rng(seed)
    f = r.standard_normal(N)
    t = synth.make_blob_template(r, L, 3, L / 2).grid()
    m = synth.ball_mask(L, L / 2)
    return f, t, m


def test_ncc_bounded_by_cauchy_schwarz():
    f, t, m = _random_setup(13)
    # structured image too, to approach the bound
    f = f + 3 * np.roll(np.pad(t, 3), 2, axis=0)[:14, :14, :14]
    quats = synth.random_quaternions(_rng(14), 12)
    xs = O.all_positions(f.shape)
    c = O.classical_ncc_at(f, t, m, quats, xs)
    assert np.all(np.abs(c) <= 1.0 + 1e-12)
    assert np.abs(c).max() > 0.3


def test_ncc_is_one_at_noiseless_copy_and_affine_invariant():
    f, t, m = _random_setup(15)
    # radius 3 keeps every rotated sample inside the 8-box, where adding a
    # constant to t commutes with zero-filled resampling
    m = synth.ball_mask(t.shape[0], 3.0)
    q = synth.random_quaternions(_rng(16), 1)[0]
    s = O.rotated_template(t, m, q)
    L = t.shape[0]
    c = L // 2
    x0 = np.array([7, 6, 8])
    g = f.copy()
    sl = tuple(slice(x0[i] - c, x0[i] - c + L) for i in range(3))
    inside = m > 0
    win = g[sl]
    win[inside] = 2.5 * s[inside] - 1.25            # alpha s + beta inside the mask
    g[sl] = win
    val = O.classical_ncc_at(g, t, m, q[None], x0[None])[0, 0]
    assert val == pytest.approx(1.0, abs=1e-12)
    xs = O.all_positions(g.shape)[::7]
    base = O.classical_ncc_at(g, t, m, q[None], xs)
    # f -> a f + b, t -> d t + e: unchanged if a d > 0, negated if a d < 0
    same = O.classical_ncc_at(3.0 * g + 2.0, 0.5 * t - 7.0, m, q[None], xs)
    flip = O.classical_ncc_at(-3.0 * g + 2.0, 0.5 * t + 1.0, m, q[None], xs)
    assert np.allclose(same, base, atol=1e-10)
    assert np.allclose(flip, -base, atol=1e-10)


def test_classical_argmax_finds_planted_rotation():
    f, t, m = _random_setup(17)
    quats = synth.random_quaternions(_rng(18), 20)
    k = 13
    s = O.rotated_template(t, m, quats[k])
    L = t.shape[0]
    x0 = np.array([7, 7, 7])
    sl = tuple(slice(x0[i] - L // 2, x0[i] - L // 2 + L) for i in range(3))
    win = f[sl]
    win[m > 0] = s[m > 0]
    f[sl] = win
    best, idx = O.classical_best_at(f, t, m, quats, x0[None])
    assert idx[0] == k and best[0] == pytest.approx(1.0, abs=1e-12)


# --------------------------------------------------------------------------
# tensor template and tensor field (Sections 3.2-3.4)
# --------------------------------------------------------------------------

def test_rotation_invariant_template_gives_degenerate_tensor():
    # A template invariant under the cube rotations, integrated with the binary
    # octahedral group (a 7-design), gives T_alpha = E[Q^alpha] s exactly.
    L = 10
    c = L // 2
    ax = np.arange(L) - c
    g = np.meshgrid(ax, ax, ax, indexing="ij")
    rad2 = g[0] ** 2 + g[1] ** 2 + g[2] ** 2
    t = np.exp(-rad2 / 6.0) + 0.3 * np.cos(rad2 / 3.0)
    m = synth.ball_mask(L, 4.5)
    quats = synth.binary_octahedral()
    w = np.full(len(quats), 1.0 / len(quats))
    s = O.rotated_template(t, m, np.array([1.0, 0, 0, 0]))
    for n in (2, 4, 6):
        T = O.tensor_template(t, m, n, quats, w)
        M = np.array([_closed_form_moment(tuple(a)) for a in O.multi_indices(n)])
        assert np.allclose(T, M[:, None, None, None] * s[None], atol=1e-12)
        # then phi(Q) = C Q^n is the same for every unit Q
        A = M * 0.37
        vals = [O.tensor_apply(A, n, q) for q in synth.random_quaternions(_rng(n), 5)]
        assert np.allclose(vals, vals[0], atol=1e-14)


def test_tensor_field_is_integral_of_classical_ncc():
    # C_n(x) = int R^{(.)n} c(x,R) dR  (Section 3.2), exactly on any quadrature;
    # and phi(Q) = C_n(x) Q^n = int (Q.R)^n c(x,R) dR (proof of Theorem "main")
    f, t, m = _random_setup(19)
    n = 4
    quats = synth.random_quaternions(_rng(20), 30)
    wts = _rng(21).uniform(0.5, 1.5, len(quats))
    wts /= wts.sum()
    T = O.tensor_template(t, m, n, quats, wts)
    xs = np.array([[7, 7, 7], [5, 9, 6], [8, 4, 10]])
    C = O.tensor_field_at(f, T, m, xs)
    c = O.classical_ncc_at(f, t, m, quats, xs)
    ref = c @ (wts[:, None] * O.monomials(quats, n))
    assert np.allclose(C, ref, atol=1e-13)
    Q = synth.random_quaternions(_rng(22), 3)
    for p in range(len(xs)):
        for q in Q:
            lhs = O.tensor_apply(C[p], n, q)
            rhs = float(np.sum(wts * (quats @ q) ** n * c[p]))
            assert lhs == pytest.approx(rhs, abs=1e-13)


def test_spectral_norm_bound():
    # ||T||_sigma >= ||T||_F / 2^{n-1}, ||T||_sigma = max |T Q^n|  (Section 3.4)
    for n in (2, 4, 6):
        for seed in range(4):
            A = _rng(30 + seed).standard_normal(O.num_components(n))
            pts = O.oracle_sphere_points(20000)
            vals = O.monomials(pts, n) @ (O.multiplicities(n) * A)
            assert np.abs(vals).max() >= O.frobenius_norm(A, n) / 2 ** (n - 1)


def test_sshopm_reaches_brute_force_maximum():
    for n in (2, 4, 6):
        A = _rng(40 + n).standard_normal(O.num_components(n))
        q, lam, _ = O.dominant_z_eigenpair(A, n, n_brute=50000)
        pts = O.oracle_sphere_points(50000)
        vals = O.monomials(pts, n) @ (O.multiplicities(n) * A)
        assert lam >= vals.max() - 1e-12
        # a Z-eigenpair: A q^{n-1} = lambda q
        assert np.allclose(O.tensor_apply_nm1(A, n, q), lam * q, atol=1e-8)
        if n == 2:
            # order 2: the dominant Z-eigenvalue is the top matrix eigenvalue
            assert lam == pytest.approx(np.linalg.eigvalsh(O.unpack_symmetric(A, 2))[-1], abs=1e-10)


@pytest.fixture(scope="module")
def planted_setup():
    # the quadrature must resolve c(x, R) over SO(3): 10^4 rotations (~5 degree
    # spacing) bring the recovered pose within a fraction of a degree
    L, n = 12, 4
    tm = synth.make_blob_template(_rng(50), L, 5, L / 2)
    m = synth.ball_mask(L, L / 2)
    qs = synth.super_fibonacci(10000)
    wts = np.full(len(qs), 1.0 / len(qs))
    T = O.tensor_template(tm.grid(), m, n, qs, wts)
    return L, n, tm, m, T


def test_theorem_main_recovers_planted_rotation(planted_setup):
    # a noiseless analytic copy at x0 rotated by R*: phi peaks at R* (Theorem "main")
    L, n, tm, m, T = planted_setup
    errs = []
    for k, qtrue in enumerate(synth.random_quaternions(_rng(51), 3)):
        x0 = np.array([[12, 12, 12]])
        f = synth.render_copies((24, 24, 24), tm, x0, qtrue[None])
        C = O.tensor_field_at(f, T, m, x0)[0]
        q, lam, second = O.dominant_z_eigenpair(C, n, n_brute=60000)
        errs.append(O.rotation_angle_deg(q, qtrue))
    assert max(errs) < 1.0, errs


def test_rotation_map_at_planted_copies_flat_window_and_bound(planted_setup):
    # two noiseless copies with different rotations in one image: at each
    # copy's centre the map holds that copy's rotation, not the other's
    # (Theorem "main" position by position); a window in a flat region (w = 0)
    # holds the identity with lambda = 0; and |lambda| <= F = |C_n(x)|_F at
    # every voxel (Cauchy-Schwarz with |Q^{(.)n}|_F = 1)
    L, n, tm, m, T = planted_setup
    qtrue = synth.random_quaternions(_rng(52), 2)
    assert O.rotation_angle_deg(qtrue[0], qtrue[1]) > 20.0
    centres = np.array([[12, 12, 12], [12, 12, 30]])
    f = synth.render_copies((24, 24, 60), tm, centres, qtrue)
    xs = np.array([[12, 12, 12], [12, 12, 30], [12, 12, 48], [11, 13, 21]])
    q, lam, _ = O.rotation_map_at(f, T, m, n, xs, n_brute=60000)
    assert O.rotation_angle_deg(q[0], qtrue[0]) < 1.0
    assert O.rotation_angle_deg(q[1], qtrue[1]) < 1.0
    assert np.array_equal(q[2], [1.0, 0.0, 0.0, 0.0]) and lam[2] == 0.0
    F = O.score_from_field(O.tensor_field_at(f, T, m, xs), n)
    assert F[2] == 0.0
    assert np.all(np.abs(lam) <= F + 1e-12)
    assert lam[0] > 0.0 and lam[1] > 0.0


# --------------------------------------------------------------------------
# candidate positions
# --------------------------------------------------------------------------

def test_find_peaks_hand_made():
    F = np.zeros((12, 12, 12))
    F[4, 4, 4] = 5.0
    F[4, 4, 5] = 4.0          # neighbour of a larger value: not a local max
    F[8, 8, 8] = 3.0
    F[4, 8, 4] = 5.0          # tie with (4,4,4): lower linear index first
    F[5, 5, 7] = 2.0          # within distance 4 of (4,4,4): suppressed
    F[1, 1, 1] = 9.0          # outside the valid region for L=4
    got = O.find_peaks(F, (4, 4, 4), 0.5, 4.0, 10)
    assert [tuple(p) for p in got] == [(4, 4, 4), (4, 8, 4), (8, 8, 8)]
    got = O.find_peaks(F, (4, 4, 4), 3.5, 4.0, 10)
    assert [tuple(p) for p in got] == [(4, 4, 4), (4, 8, 4)]
    got = O.find_peaks(F, (4, 4, 4), 0.5, 4.0, 1)
    assert [tuple(p) for p in got] == [(4, 4, 4)]
    # plateaus (equal neighbours) are not strict maxima
    F2 = np.zeros((10, 10, 10))
    F2[5, 5, 5] = F2[5, 5, 6] = 1.0
    assert len(O.find_peaks(F2, (4, 4, 4), 0.1, 2.0, 10)) == 0


def test_find_peaks_fast_matches_loops():
    r = _rng(60)
    F = r.random((14, 13, 12))
    for thr, d in [(0.5, 3.0), (0.9, 5.0), (0.0, 1.0)]:
        a = O.find_peaks(F, (5, 4, 6), thr, d, 7)
        b = O.find_peaks_fast(F, (5, 4, 6), thr, d, 7)
        assert np.array_equal(a, b)


def test_refinement_returns_to_a_noiseless_copy():
    # a nearly noiseless analytic copy at x0 with a random pose: started one
    # voxel away along a corner diagonal, the NCC-verified refinement moves to
    # x0, where the NCC at the recovered rotation is near 1 (the copy is exact
    # up to the rotation's quadrature error: Section 2, NCC = 1 at an exact
    # copy; Theorem "main" for the rotation).  Choosing by the largest
    # eigenvalue instead stays off the copy here, so this pins the NCC rule.
    L, n = 12, 4
    tm = synth.make_blob_template(_rng(60), L, 5, L / 2)
    t = tm.grid()
    m = synth.ball_mask(L, L / 2)
    qs = synth.super_fibonacci(3000)
    T = O.tensor_template(t, m, n, qs, np.full(len(qs), 1.0 / len(qs)))
    qtrue = synth.random_quaternions(_rng(61), 1)[0]
    x0 = np.array([12, 12, 12])
    f = synth.render_copies((24, 24, 24), tm, x0[None], qtrue[None])
    f = f + 0.01 * _rng(62).standard_normal(f.shape)
    for start in (x0 + np.array([-1, 1, -1]),):
        pos, q, lam, ncc, nccs = O.refine_by_ncc(f, t, m, T, n, start, n_brute=20000)
        assert np.array_equal(pos, x0), (start, pos, nccs)
        assert ncc > 0.95, ncc
        assert O.rotation_angle_deg(q, qtrue) < 3.0
        # the neighbour values that exist are finite and below the chosen one
        fin = nccs[np.isfinite(nccs)]
        assert len(fin) == 27 and fin.max() == ncc


def _order2_matrix(C):
    """The 4 x 4 symmetric matrix M of a packed order-2 tensor, C Q^2 = Q^T M Q:
    at order 2 the dominant Z-eigenvalue is the largest eigenvalue of M (a
    textbook symmetric eigenproblem)."""
    M = np.zeros((4, 4))
    for c, a in zip(C, O.multi_indices(2)):
        i, j = [k for k in range(4) for _ in range(a[k])]
        M[i, j] = M[j, i] = c
    return M


def _rule_pick(lams):
    """The selection rule of the eigenvalue refinement, written out: the
    largest value; the centre (index 13) among equal values, then the lowest
    neighbour index."""
    best = max(lams)
    if lams[13] == best:
        return 13
    return min(k for k in range(27) if lams[k] == best)


def test_refine_by_eigenvalue_rule_and_ties():
    # Section 3.4 reading: the candidate moves to the voxel of its 3x3x3
    # neighbourhood with the largest dominant Z-eigenvalue; the centre first on
    # ties, then the lower neighbour index.  An image constant along axis 2
    # makes the three voxels of each (d0, d1) column of the neighbourhood see
    # bit-identical windows, hence bit-identical tensors and eigenvalues: exact
    # three-way ties in every column.  At order 2 the 27 eigenvalues are pinned
    # against numpy's symmetric eigensolver, and the chosen voxel against the
    # rule applied to them.  At (12, 8, 8) the centre column is largest (the
    # centre must win over its lower-index equal, 12); at (6, 11, 8) the column
    # (+1, +1) is (its d2 = -1 voxel, index 24, must win over 25 and 26).
    n, L = 2, 7
    rng = _rng(90)
    g = rng.standard_normal((20, 20))
    f = np.repeat(g[:, :, None], 16, axis=2)
    t = synth.make_blob_template(rng, L, 3, L / 2).grid()
    m = synth.ball_mask(L, L / 2)
    qs = synth.super_fibonacci(400)
    T = O.tensor_template(t, m, n, qs, np.full(len(qs), 1.0 / len(qs)))
    offs = O.neighbourhood_offsets()
    for x, want in (([12, 8, 8], 13), ([6, 11, 8], 24)):
        x = np.array(x)
        pos, q, lam, lams = O.refine_by_eigenvalue(f, T, m, n, x, n_brute=5000)
        for k in range(0, 27, 3):
            assert lams[k] == lams[k + 1] == lams[k + 2]
        C = O.tensor_field_at(f, T, m, x[None] + offs)
        for k in range(27):
            ev = np.linalg.eigvalsh(_order2_matrix(C[k]))[-1]
            assert abs(lams[k] - ev) <= 1e-10 * O.frobenius_norm(C[k], n), (k, lams[k], ev)
        k = _rule_pick(list(lams))
        assert k == want, (k, want)
        assert np.array_equal(pos, x + offs[k]) and lam == lams[k]
    # a flat neighbourhood: w = 0 and C = 0 at all 27 voxels, every eigenvalue
    # is 0, and the candidate stays where it is
    f0 = np.zeros((20, 20, 16))
    f0[0, 0, 0] = 1.0
    pos, q, lam, lams = O.refine_by_eigenvalue(f0, T, m, n, np.array([10, 10, 8]), n_brute=2000)
    assert np.all(lams == 0.0) and np.array_equal(pos, [10, 10, 8])


def test_iterated_refinement_climbs_to_a_noiseless_copy():
    # the same nearly noiseless copy, started two voxels away along a corner
    # diagonal: one NCC refinement step moves one voxel; repeated from its own
    # result it reaches the copy and stops there (the copy is a fixed point:
    # its NCC is the largest of its neighbourhood), in three rounds
    L, n = 12, 4
    tm = synth.make_blob_template(_rng(60), L, 5, L / 2)
    t = tm.grid()
    m = synth.ball_mask(L, L / 2)
    qs = synth.super_fibonacci(3000)
    T = O.tensor_template(t, m, n, qs, np.full(len(qs), 1.0 / len(qs)))
    qtrue = synth.random_quaternions(_rng(61), 1)[0]
    x0 = np.array([12, 12, 12])
    f = synth.render_copies((24, 24, 24), tm, x0[None], qtrue[None])
    f = f + 0.01 * _rng(62).standard_normal(f.shape)
    start = x0 + np.array([2, -2, 2])
    # a cap of one round is the single step
    one, _, _, _, r1 = O.refine_by_ncc_iterated(f, t, m, T, n, start, n_brute=4000, max_rounds=1)
    assert np.abs(one - x0).max() == 1 and r1 == 1, one
    pos, q, lam, ncc, rounds = O.refine_by_ncc_iterated(f, t, m, T, n, start, n_brute=4000)
    assert np.array_equal(pos, x0), pos
    assert rounds == 3, rounds
    assert ncc > 0.95 and O.rotation_angle_deg(q, qtrue) < 3.0


# --------------------------------------------------------------------------
# gradient of the score (adjoint) against central finite differences
# --------------------------------------------------------------------------

def test_rotation_adjoint_is_the_transpose():
    rng = _rng(70)
    L = (7, 6, 8)
    q = synth.random_quaternions(rng, 1)[0]
    t = rng.standard_normal(L)
    h = rng.standard_normal(L)
    lhs = float((O.rotate_trilinear(t, q) * h).sum())
    rhs = float((t * O.rotate_trilinear_adjoint(h, q, L)).sum())
    assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs))


def test_score_gradient_matches_central_differences():
    # L = sum_p g_p F(x_p) on a noisy image with a planted copy; central
    # differences (h = 1e-3) of the oracle's own forward pin the analytic
    # adjoint for template voxels (inside and outside the mask) and image
    # voxels (inside windows, in two overlapping windows, and outside all)
    rng = _rng(71)
    L, n = 8, 4
    tm = synth.make_blob_template(rng, L, 4, L / 2)
    t = tm.grid()
    m = synth.ball_mask(L, 3.6)
    qs = synth.random_quaternions(rng, 30)
    wts = rng.uniform(0.5, 1.5, 30)
    wts /= wts.sum()
    f = rng.standard_normal((20, 20, 20))
    f += 2.0 * synth.render_copies((20, 20, 20), tm, np.array([[10, 10, 10]]), qs[:1])
    # the last position is outside the valid region: F is 0 there by
    # definition and it must not contribute
    xs = np.array([[10, 10, 10], [11, 9, 10], [6, 13, 8], [1, 2, 18]])
    gF = np.array([1.0, -0.5, 0.7, 2.0])
    gt, gf = O.score_grad(f, t, m, n, qs, wts, xs, gF)

    def loss(tt, ff):
        return float(gF @ O.score_at(ff, tt, m, n, qs, wts, xs))

    h = 1e-3
    for idx in [(4, 4, 4), (1, 4, 5), (0, 0, 0), (6, 2, 3), (3, 7, 4)]:
        tp, tq = t.copy(), t.copy()
        tp[idx] += h
        tq[idx] -= h
        fd = (loss(tp, f) - loss(tq, f)) / (2 * h)
        assert abs(fd - gt[idx]) <= 1e-6 + 1e-5 * abs(fd), (idx, fd, gt[idx])
    for idx in [(10, 10, 10), (8, 11, 12), (11, 10, 9), (7, 12, 8), (1, 1, 18)]:
        fp, fq = f.copy(), f.copy()
        fp[idx] += h
        fq[idx] -= h
        fd = (loss(t, fp) - loss(t, fq)) / (2 * h)
        assert abs(fd - gf[idx]) <= 1e-6 + 1e-5 * abs(fd), (idx, fd, gf[idx])
    assert gf[1, 1, 18] == 0.0          # outside every valid window
    assert O.score_at(f, t, m, n, qs, wts, xs)[3] == 0.0


# --------------------------------------------------------------------------
# low-pass filter and soft mask
# --------------------------------------------------------------------------

def test_lowpass_pins():
    rng = _rng(90)
    # unit DC gain: a constant image is unchanged (h * 1 = 1)
    c = np.full((9, 10, 11), 3.25)
    assert np.allclose(O.lowpass(c, 1.3), c, atol=1e-13)
    # sigma 0 is the identity
    f = rng.standard_normal((12, 9, 10))
    assert np.array_equal(O.lowpass(f, 0.0), f)
    # separable filter = brute-force 3-D circular convolution with the outer product
    sigma = 0.8
    h = O.lowpass_kernel(sigma)
    R = (len(h) - 1) // 2
    g = rng.standard_normal((7, 8, 9))
    ref = np.zeros_like(g)
    N = g.shape
    for k0 in range(-R, R + 1):
        for k1 in range(-R, R + 1):
            for k2 in range(-R, R + 1):
                ref += h[k0 + R] * h[k1 + R] * h[k2 + R] * np.roll(g, (k0, k1, k2), axis=(0, 1, 2))
    assert np.allclose(O.lowpass(g, sigma), ref, atol=1e-12)
    # the same as multiplying the spectrum by the transfer function of h
    ker = np.zeros(N)
    for k0 in range(-R, R + 1):
        for k1 in range(-R, R + 1):
            for k2 in range(-R, R + 1):
                ker[k0 % N[0], k1 % N[1], k2 % N[2]] += h[k0 + R] * h[k1 + R] * h[k2 + R]
    fft = np.real(np.fft.ifftn(np.fft.fftn(g) * np.fft.fftn(ker)))
    assert np.allclose(O.lowpass(g, sigma), fft, atol=1e-12)
    # isotropic on the grid: commutes with a 90-degree turn
    cube = rng.standard_normal((8, 8, 8))
    assert np.allclose(O.lowpass(np.rot90(cube, axes=(1, 2)), 1.1), np.rot90(O.lowpass(cube, 1.1), axes=(1, 2)),
                       atol=1e-12)
    # zero extension = periodic filtering of the zero-padded box, cropped
    pad = np.pad(g, R + 1)
    crop = O.lowpass(pad, sigma)[R + 1:-R - 1, R + 1:-R - 1, R + 1:-R - 1]
    assert np.allclose(O.lowpass(g, sigma, periodic=False), crop, atol=1e-12)


def test_soft_mask_shape():
    m = O.soft_mask(16, 5.0, 7.0)
    c = O.template_centre((16, 16, 16))
    assert m[tuple(c)] == 1.0 and m[c[0], c[1], c[2] + 5] == 1.0
    assert m[c[0], c[1], c[2] + 7] == 0.0 and m[0, 0, 0] == 0.0
    assert abs(m[c[0], c[1], c[2] + 6] - 0.5) < 1e-12
    # rotationally symmetric on the grid (odd box: its centre is the array's)
    m15 = O.soft_mask(15, 4.5, 6.5)
    assert np.allclose(m15, np.rot90(m15, axes=(0, 2))) and np.allclose(m15, np.transpose(m15, (2, 0, 1)))


# --------------------------------------------------------------------------
# S'-consistent normalisation (Section 3.4, false positives; S' = S_2 S from
# the proof of Theorem "main")
# --------------------------------------------------------------------------

def _cube_rotations():
    """The 24 rotations of the cube, one quaternion per rotation."""
    g = synth.binary_octahedral()
    keep = [q for q in g if q[np.nonzero(q)[0][0]] > 0]
    assert len(keep) == 24
    return np.array(keep)


def _ball(L, radius):
    c = L // 2
    g = np.meshgrid(*[np.arange(L) - c] * 3, indexing="ij")
    r2 = g[0] ** 2 + g[1] ** 2 + g[2] ** 2
    return (np.sqrt(r2) < radius).astype(np.float64), r2


@pytest.mark.parametrize("n", [2, 4, 6, 8])
def test_s_prime_norm_closed_form_on_the_cube_group(n):
    """A window invariant under the cube's rotations, the 24 rotations as the
    quadrature (grid-exact, equal weights): every rotated copy is the window,
    so D = (1/24) sum_R a_R^n.  The classes of the group: the identity (a = 1),
    three half-turns about the axes and six about the edge diagonals (a = 0),
    six quarter-turns (a = 1/sqrt 2) and eight third-turns about the body
    diagonals (a = 1/2)."""
    m, r2 = _ball(11, 4.6)
    h = 3.0 + 2.0 * np.exp(-r2 / 8.0)          # radial, with an offset and a scale
    D = O.s_prime_norm2(h, m, n, _cube_rotations(), np.full(24, 1 / 24))
    closed = (1.0 + 6.0 * 2.0 ** (-n / 2) + 8.0 * 2.0 ** (-n)) / 24.0
    assert abs(D - closed) < 1e-12


def test_s_prime_score_bounded_and_one_at_a_copy_on_the_cube_group():
    """With the cube group as the quadrature the discrete S' form is a group
    convolution with the positive-definite kernel a^n, so the S'-normalised
    score obeys Cauchy-Schwarz at every position and every group rotation,
    with equality at a noiseless copy (affinely changed) rotated by a group
    element."""
    G, w, n = _cube_rotations(), np.full(24, 1 / 24), 4
    L, c = 11, 5
    m, _ = _ball(L, 4.6)
    rng = _rng(41)
    t = rng.standard_normal((L, L, L))
    f = rng.standard_normal((40, 40, 40))
    T = O.tensor_template(t, m, n, G, w)
    xs = np.array([[10, 12, 20], [20, 20, 20], [30, 15, 8], [7, 33, 25]])
    C = O.tensor_field_at(f, T, m, xs)
    Dx, Dt = O.s_prime_norms_at(f, t, m, n, G, w, xs)
    assert Dt > 0 and np.all(Dx > 0)
    for p in range(len(xs)):
        lam = np.array([O.tensor_apply(C[p], n, q) for q in G])
        rho = O.s_prime_score(lam, np.full(24, Dx[p]), Dt)
        assert np.all(np.abs(rho) <= 1.0 + 1e-12)
    # the copy: rotate by a group element with numpy index operations only
    # (a quarter-turn about axis 0 is rot90 over axes (1, 2))
    q0 = np.array([math.cos(math.pi / 4), math.sin(math.pi / 4), 0.0, 0.0])
    x0 = np.array([20, 20, 20])
    f2 = f.copy()
    f2[x0[0] - c:x0[0] - c + L, x0[1] - c:x0[1] - c + L, x0[2] - c:x0[2] - c + L] = \
        2.5 * np.rot90(t, 1, axes=(1, 2)) + 1.0
    C2 = O.tensor_field_at(f2, T, m, x0[None])
    Dx2, _ = O.s_prime_norms_at(f2, t, m, n, G, w, x0[None])
    assert abs(Dx2[0] - Dt) < 1e-12 * Dt
    rho = O.s_prime_score([O.tensor_apply(C2[0], n, q0)], Dx2, Dt)[0]
    assert abs(rho - 1.0) < 1e-12


def test_s_prime_norm_continuum_value_for_a_radial_window():
    """In the continuum, a rotation-invariant window is its own rotated copy,
    so ||h~||^2_{S'} = int_{SO(3)} a_P^n dP = E[a^n] over the unit sphere of
    R^4 = Gamma((n+1)/2) / (sqrt(pi) Gamma((n+4)/2)) (1/4, 1/8, 5/64 for
    n = 2, 4, 6).  A smooth radial blob with a dense quadrature reaches it to
    the quadrature and interpolation error."""
    q = synth.super_fibonacci(2000)
    w = np.full(len(q), 1.0 / len(q))
    m, r2 = _ball(15, 6.5)
    h = np.exp(-r2 / (2 * 3.0 ** 2))
    n = 4
    D = O.s_prime_norm2(h, m, n, q, w)
    E = math.gamma((n + 1) / 2) / (math.sqrt(math.pi) * math.gamma((n + 4) / 2))
    assert abs(E - 0.125) < 1e-15
    assert abs(D / E - 1.0) < 2e-3


def test_s_prime_norm_flat_window_and_zero_score():
    L = 9
    m, _ = _ball(L, 3.6)
    G = _cube_rotations()
    assert math.isnan(O.s_prime_norm2(np.full((L, L, L), 2.0), m, 4, G, np.full(24, 1 / 24)))
    rho = O.s_prime_score([0.5, 0.5, 0.5], [math.nan, -1.0, 0.04], 0.04)
    assert rho[0] == 0.0 and rho[1] == 0.0 and abs(rho[2] - 12.5) < 1e-12


# --------------------------------------------------------------------------
# two-dimensional TTM (Sections 2 and 3 with d = 2; rotations as unit complex
# numbers of half the rotation angle)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n", [2, 4, 8])
def test_planar_power_identity(n):
    """<z^(.)n, y^(.)n> = (z . y)^n with the packed planar storage (the
    identity of Section 3.1 in S^n(R^2))."""
    rng = _rng(50 + n)
    for _ in range(5):
        z, y = rng.standard_normal(2), rng.standard_normal(2)
        lhs = float(O.planar_monomials(z[None], n)[0] * O.planar_multiplicities(n)
                    @ O.planar_monomials(y[None], n)[0]) * (np.linalg.norm(z) * np.linalg.norm(y)) ** n
        assert abs(lhs - float(z @ y) ** n) < 1e-12 * max(1.0, abs(float(z @ y)) ** n)
    # the Frobenius norm over all 2^n entries, by brute force
    C = rng.standard_normal(n + 1)
    full = 0.0
    for idx in np.ndindex(*([2] * n)):
        full += C[int(sum(idx))] ** 2
    assert abs(O.score_from_field_2d(C[None], n)[0] ** 2 - full) < 1e-10 * full


def test_planar_rotation_is_rot90_and_the_half_angle_separates_half_turns():
    t = _rng(60).standard_normal((9, 9))
    z90 = np.array([math.cos(math.pi / 4), math.sin(math.pi / 4)])
    assert np.allclose(O.rotate_bilinear(t, z90), np.rot90(t, 1, axes=(0, 1)), atol=1e-12)
    z180 = np.array([0.0, 1.0])
    assert np.allclose(O.rotate_bilinear(t, z180), np.rot90(t, 2, axes=(0, 1)), atol=1e-12)
    assert np.allclose(O.rot2_matrix(z180), -np.eye(2), atol=1e-15)
    assert abs(O.rotation_angle_2d_deg([1.0, 0.0], z180) - 180.0) < 1e-12


def test_planar_tensor_field_is_the_integral_of_classical_ncc():
    """C_k(x) = sum_j omega_j a_j^(n-k) b_j^k c(x, R_j) (the defining integral
    of Section 3.2 in the plane), with c from the classical NCC."""
    rng = _rng(61)
    L, n = 11, 4
    t = rng.standard_normal((L, L))
    m = synth.disc_mask(L, 5.0)
    f = rng.standard_normal((40, 36))
    zs = synth.circle_quadrature(37)
    w = rng.uniform(0.5, 1.5, 37)
    w /= w.sum()
    xs = np.array([[10, 12], [20, 20], [29, 7]])
    C = O.tensor_field_at_2d(f, O.tensor_template_2d(t, m, n, zs, w), m, xs)
    c = O.classical_ncc_at_2d(f, t, m, zs, xs)
    ref = (c * w[None]) @ O.planar_monomials(zs, n)
    assert np.allclose(C, ref, atol=1e-12)


@pytest.mark.parametrize("n", [2, 4, 6])
def test_planar_rotation_invariant_template_gives_closed_form_moments(n):
    """A disc-symmetric template is its own rotated copy under grid-exact
    quarter-turns; with the four quarter-turns z = (cos psi, sin psi),
    psi = 0, 45, 90, 135 degrees, T_k = M_k s with M_k the mean of
    cos^(n-k) psi sin^k psi, which for an equispaced set of more than n/2
    points on [0, pi) equals the circle average (n-k-1)!! (k-1)!! / n!! for
    even k (0 for odd k)."""
    L = 11
    m = synth.disc_mask(L, 5.0)
    g = np.meshgrid(np.arange(L) - 5, np.arange(L) - 5, indexing="ij")
    t = np.exp(-(g[0] ** 2 + g[1] ** 2) / 6.0)
    psi = np.array([0.0, 0.25, 0.5, 0.75]) * math.pi
    zs = np.stack([np.cos(psi), np.sin(psi)], axis=1)
    T = O.tensor_template_2d(t, m, n, zs, np.full(4, 0.25))
    s = O.masked_normalize(t, m)

    def dfact(k):
        return 1 if k <= 0 else k * dfact(k - 2)

    for k in range(n + 1):
        M = dfact(n - k - 1) * dfact(k - 1) / dfact(n) if k % 2 == 0 else 0.0
        assert np.allclose(T[k], M * s, atol=1e-12), k


def test_planar_theorem_recovers_planted_rotations():
    """The planar analogue of Theorem "main", checked numerically: at the
    centre of a noiseless copy the dominant eigenvector of C_n(x) is the
    copy's rotation, for quarter, half and three-quarter turns (exact on the
    grid, through numpy) and for an analytically rendered copy at 37 degrees;
    a half turn is not confused with the identity."""
    n = 8
    L = 25
    rng = _rng(62)
    tm = synth.make_blob_template_2d(rng, L, 5, L / 2)
    c = L // 2
    ax = np.arange(L, dtype=np.float64) - c
    t = tm.evaluate(np.stack(np.meshgrid(ax, ax, indexing="ij"), axis=-1))
    m = synth.disc_mask(L, L / 2)
    zs = synth.circle_quadrature(720)
    T = O.tensor_template_2d(t, m, n, zs, np.full(720, 1 / 720))
    f = np.zeros((60, 120))
    cases = []
    for i, k in enumerate((1, 2, 3)):
        x = np.array([30, 20 + 35 * i])
        f[x[0] - c:x[0] - c + L, x[1] - c:x[1] - c + L] = np.rot90(t, k, axes=(0, 1))
        cases.append((x, 90.0 * k))
    C = O.tensor_field_at_2d(f + 0.0, T, m, np.array([x for x, _ in cases]))
    for (x, ang), Cx in zip(cases, C):
        z, lam, second = O.dominant_eigen_2d(Cx, n)
        zt = np.array([math.cos(math.radians(ang) / 2), math.sin(math.radians(ang) / 2)])
        assert O.rotation_angle_2d_deg(z, zt) < 1.0, (ang, z)
        assert lam > second
    # analytic copy at 37 degrees
    a = math.radians(37.0)
    rm = np.array([[math.cos(a), -math.sin(a)], [math.sin(a), math.cos(a)]])
    g = np.stack(np.meshgrid(np.arange(L) - c, np.arange(L) - c, indexing="ij"), axis=-1).astype(float)
    f2 = np.zeros((40, 40))
    f2[20 - c:20 - c + L, 20 - c:20 - c + L] = tm.evaluate(g @ rm)
    Cx = O.tensor_field_at_2d(f2, T, m, np.array([[20, 20]]))[0]
    z, lam, _ = O.dominant_eigen_2d(Cx, n)
    assert O.rotation_angle_2d_deg(z, [math.cos(a / 2), math.sin(a / 2)]) < 2.0


@pytest.mark.parametrize("n", [2, 4, 6, 8])
def test_planar_eigenpair_closed_forms(n):
    """The dominant eigenpair on the circle in two closed forms.  For the
    rank-one tensor z^n (C_k = a^(n-k) b^k) the eigenvalue on the circle is
    (a cos psi + b sin psi)^n = cos^n(psi - theta/2): lambda = 1 exactly, at
    z, and the best value more than 5 degrees of rotation away (2.5 degrees of
    half-angle) is cos^n(2.5 deg) up to one scan step.  The tensor of
    (x^2 + y^2)^(n/2) (C_k = C(n/2, k/2) / C(n, k) for even k, 0 for odd k)
    is 1 on the whole circle: lambda and that best value both equal 1."""
    step = 180.0 / 20000
    for deg in (0.0, 0.2, 37.0, 90.0, 179.9, 180.0, 270.0, 359.8):
        th = math.radians(deg)
        a, b = math.cos(th / 2), math.sin(th / 2)
        C = np.array([a ** (n - k) * b ** k for k in range(n + 1)])
        z, lam, second = O.dominant_eigen_2d(C, n)
        assert abs(lam - 1.0) <= 1e-12, (deg, lam)
        assert O.rotation_angle_2d_deg(z, [a, b]) <= 1e-5, (deg, z)
        assert z[0] > 0.0 or (z[0] == 0.0 and z[1] > 0.0)
        hi = math.cos(math.radians(2.5)) ** n
        lo = math.cos(math.radians(2.5 + step)) ** n
        assert lo - 1e-12 <= second <= hi + 1e-12, (deg, second, lo, hi)
    C = np.array([math.comb(n // 2, k // 2) / math.comb(n, k) if k % 2 == 0 else 0.0 for k in range(n + 1)])
    z, lam, second = O.dominant_eigen_2d(C, n)
    assert abs(lam - 1.0) <= 1e-12 and abs(second - 1.0) <= 1e-12


def test_planar_local_norm_two_pass_equals_one_pass_fft_and_loops():
    # ||P_S tau_x f||_S^2 = <(tau_x f)^2, m> - <tau_x f, m>^2 / <1, m> in the
    # plane (Section 2, with d = 2): the two-pass oracle against the one-pass
    # form evaluated with the library FFT, and against explicit loops for the
    # masked mean and variance; a constant window gives w = 0
    r = _rng(13)
    f = 3.0 + r.standard_normal((17, 14))
    L = (7, 6)
    m = r.uniform(0.2, 1.0, L)
    m[0, 0] = 0.0
    c = [l // 2 for l in L]
    big = np.zeros(f.shape)
    for u0 in range(L[0]):
        for u1 in range(L[1]):
            big[(u0 - c[0]) % f.shape[0], (u1 - c[1]) % f.shape[1]] += m[u0, u1]
    corr = lambda a: np.real(np.fft.ifft2(np.fft.fft2(a) * np.conj(np.fft.fft2(big))))
    v = corr(f * f) - corr(f) ** 2 / m.sum()
    g = np.meshgrid(np.arange(f.shape[0]), np.arange(f.shape[1]), indexing="ij")
    xs = np.stack([g[0].ravel(), g[1].ravel()], axis=1)
    w = O.local_norm_at_2d(f, m, xs).reshape(f.shape)
    assert np.allclose(w, 1.0 / np.sqrt(v), rtol=1e-9)
    for x in [(0, 0), (8, 5), (16, 13)]:
        vals, wts = [], []
        for u0 in range(L[0]):
            for u1 in range(L[1]):
                vals.append(f[(x[0] + u0 - c[0]) % 17, (x[1] + u1 - c[1]) % 14])
                wts.append(m[u0, u1])
        vals, wts = np.array(vals), np.array(wts)
        mu = sum(a * b for a, b in zip(vals, wts)) / wts.sum()
        var = sum(b * (a - mu) ** 2 for a, b in zip(vals, wts))
        assert w[x] == pytest.approx(1.0 / math.sqrt(var), rel=1e-12)
    f1 = np.full((17, 14), 2.5)
    f1[0, 0] = 9.0
    assert O.local_norm_at_2d(f1, m, np.array([[8, 7]]))[0] == 0.0


def test_planar_refinement_returns_to_a_copy():
    n, L = 6, 21
    rng = _rng(63)
    tm = synth.make_blob_template_2d(rng, L, 5, L / 2)
    c = L // 2
    ax = np.arange(L, dtype=np.float64) - c
    t = tm.evaluate(np.stack(np.meshgrid(ax, ax, indexing="ij"), axis=-1))
    m = synth.disc_mask(L, L / 2)
    zs = synth.circle_quadrature(360)
    T = O.tensor_template_2d(t, m, n, zs, np.full(360, 1 / 360))
    f = 0.01 * rng.standard_normal((50, 50))
    f[25 - c:25 - c + L, 25 - c:25 - c + L] += np.rot90(t, 1, axes=(0, 1))
    pos, z, lam, ncc = O.refine_by_ncc_2d(f, t, m, T, n, np.array([26, 24]))
    assert tuple(pos) == (25, 25) and ncc > 0.95
    assert O.rotation_angle_2d_deg(z, [math.cos(math.pi / 4), math.sin(math.pi / 4)]) < 2.0
