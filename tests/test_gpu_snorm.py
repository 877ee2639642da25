"""S'-consistent normalisation of peak scores (ttm_snorm) through the C ABI
against the float64 oracle.

Tolerances: D (the squared S'-norm of a window) within 1e-4 relative plus
1e-6 absolute (per-lane float32 sums of about L^3 / 128 terms per rotation,
float64 from the wave reduction on); rho' = lambda / sqrt(D Dt) within 1e-4
relative; flags bit-exact.  At the full 256^3 / 32^3 / 10^4-rotation size
the oracle evaluates the template and one peak window (its rotation sum split
over worker processes), and every peak is checked for the relation between
rho', lambda and the two norms.
"""
import concurrent.futures as cf
import multiprocessing as mp
import os

import numpy as np
import pytest
import torch

from oracle import ttm_oracle as O
from paper_2311_07561_amd import synth, ttm

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ttm.lib()


def dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def _ball(L, radius):
    c = np.array(L) // 2
    g = np.meshgrid(*[np.arange(l) - c[i] for i, l in enumerate(L)], indexing="ij")
    return (np.sqrt(g[0] ** 2 + g[1] ** 2 + g[2] ** 2) < radius).astype(np.float32)


def _smooth_template(rng, L):
    t = rng.standard_normal(L)
    # a little smoothing so that rotated copies stay correlated
    for ax in range(3):
        t = t + 0.5 * np.roll(t, 1, axis=ax) + 0.5 * np.roll(t, -1, axis=ax)
    return t.astype(np.float32)


def _check(img, tmpl, mask, n, q, w, pos, lam, rho, D, flags, expect_flags):
    Lsh = tmpl.shape
    P = len(pos)
    got_D = D.cpu().numpy()
    got_rho = rho.cpu().numpy()
    got_fl = flags.cpu().numpy()
    assert got_fl.tolist() == list(expect_flags)
    Dt = O.s_prime_norm2(tmpl.astype(np.float64), mask.astype(np.float64), n, q.astype(np.float64), w)
    assert abs(got_D[P] - Dt) <= 1e-6 + 1e-4 * abs(Dt)
    worst = 0.0
    for p in range(P):
        if expect_flags[p] & (ttm.SNORM_FLAT | ttm.SNORM_OUTSIDE):
            assert np.isnan(got_D[p]) and got_rho[p] == 0.0
            continue
        c = np.array(Lsh) // 2
        lo = pos[p] - c
        win = img[lo[0]:lo[0] + Lsh[0], lo[1]:lo[1] + Lsh[1], lo[2]:lo[2] + Lsh[2]].astype(np.float64)
        Dx = O.s_prime_norm2(win, mask.astype(np.float64), n, q.astype(np.float64), w)
        err = abs(got_D[p] - Dx)
        worst = max(worst, err / max(abs(Dx), 1e-12))
        assert err <= 1e-6 + 1e-4 * abs(Dx), (p, got_D[p], Dx)
        ref = O.s_prime_score([lam[p]], [Dx], Dt)[0]
        assert abs(got_rho[p] - ref) <= 1e-4 * max(1.0, abs(ref)), (p, got_rho[p], ref)
    return Dt, worst


@pytest.mark.parametrize("L,radius,n_rot,n", [
    ((16, 16, 16), 7.0, 301, 4),        # rotation count not a multiple of the group of 8
    ((13, 16, 11), 4.5, 64, 2),         # non-cubic box
    ((12, 12, 12), 6.0, 96, 6),         # mask reaching the box's last voxel: corners outside
    ((12, 12, 12), 8.0, 96, 4),         # mask past the inscribed ball: the sampler's bounds test runs
])
def test_snorm_matches_oracle(L, radius, n_rot, n):
    rng = np.random.default_rng(7 + n)
    Nsh = (48, 44, 40)
    img = rng.standard_normal(Nsh).astype(np.float32)
    tmpl = _smooth_template(rng, L)
    mask = _ball(L, radius)
    c = np.array(L) // 2
    # a noiseless copy (affinely changed) at x0, a flat patch at x1
    x0 = np.array([20, 22, 19])
    lo = x0 - c
    img[lo[0]:lo[0] + L[0], lo[1]:lo[1] + L[1], lo[2]:lo[2] + L[2]] = 1.5 * tmpl - 0.25
    x1 = np.array([36, 10, 30])
    lo1 = x1 - c
    img[lo1[0]:lo1[0] + L[0], lo1[1]:lo1[1] + L[1], lo1[2]:lo1[2] + L[2]] = 3.0
    q = synth.super_fibonacci(n_rot).astype(np.float32)
    w = np.full(n_rot, 1.0 / n_rot)
    lo_v, hi_v = O.valid_region(Nsh, L)
    rand = np.stack([rng.integers(lo_v[a], hi_v[a], 6) for a in range(3)], axis=1)
    outside = np.array([[2, 20, 20]])                 # the window leaves the image
    pos = np.concatenate([x0[None], rand, x1[None], outside]).astype(np.int32)
    expect = [0] * 7 + [ttm.SNORM_FLAT, ttm.SNORM_OUTSIDE]
    lam = rng.uniform(-0.2, 0.6, len(pos))
    rho, D, flags = ttm.snorm(dev(img), dev(tmpl), dev(mask), n, q, w, dev(pos, torch.int32),
                              dev(lam, torch.float64))
    torch.cuda.synchronize()
    Dt, worst = _check(img, tmpl, mask, n, q, w, pos, lam, rho, D, flags, expect)
    # the copy: D(window) = D(template) up to float32 rounding of the image
    d0 = float(D[0])
    print(f"\nL {L}, order {n}, {n_rot} rotations: D(template) {Dt:.5f}, D(copy) {d0:.5f}, "
          f"worst relative D error {worst:.2e}")
    assert abs(d0 - Dt) <= 1e-4 * Dt


def test_snorm_count_from_device_and_cube_group_copy():
    """The cube's 24 rotations as the quadrature (grid-exact, odd box): rho' of
    an exact quarter-turn copy is 1 with the oracle's lambda at that rotation;
    positions past the device count are not written."""
    G = synth.binary_octahedral()
    G = np.array([g for g in G if g[np.nonzero(g)[0][0]] > 0])
    w = np.full(24, 1.0 / 24)
    n, L = 4, (11, 11, 11)
    rng = np.random.default_rng(11)
    tmpl = rng.standard_normal(L).astype(np.float32)
    mask = _ball(L, 4.6)
    img = rng.standard_normal((40, 40, 40)).astype(np.float32)
    x0 = np.array([20, 20, 20])
    img[15:26, 15:26, 15:26] = 2.0 * np.rot90(tmpl, 1, axes=(1, 2)) + 1.0
    q0 = np.array([np.cos(np.pi / 4), np.sin(np.pi / 4), 0.0, 0.0])
    T = O.tensor_template(tmpl.astype(np.float64), mask.astype(np.float64), n, G, w)
    C = O.tensor_field_at(img.astype(np.float64), T, mask.astype(np.float64), x0[None])
    lam0 = O.tensor_apply(C[0], n, q0)
    pos = np.array([x0, [12, 30, 22], [25, 14, 9], [30, 30, 30]], dtype=np.int32)
    lam = np.array([lam0, 0.1, 0.2, 0.3])
    count = dev(np.array([3, 0]), torch.int32)
    rho, D, flags = ttm.snorm(dev(img), dev(tmpl), dev(mask), n, G.astype(np.float32), w,
                              dev(pos, torch.int32), dev(lam, torch.float64), count=count)
    torch.cuda.synchronize()
    r = rho.cpu().numpy()
    print(f"\ncube group, quarter-turn copy: rho' = {r[0]:.7f}")
    assert abs(r[0] - 1.0) <= 1e-5
    assert r[3] == 0.0 and float(D[3]) == 0.0 and int(flags[3]) == 0     # past the count
    _check(img, tmpl, mask, n, G.astype(np.float32), w, pos[:3], lam[:3], rho[:3],
           torch.cat([D[:3], D[4:]]), flags[:3], [0, 0, 0])


def test_snorm_box_beyond_lds_takes_the_global_path():
    """A 40^3 box does not fit the LDS layout: the rotations sample the
    window from global memory."""
    n, L, n_rot = 4, (40, 40, 40), 40
    rng = np.random.default_rng(12)
    tmpl = _smooth_template(rng, L)
    mask = _ball(L, 19.0)
    img = rng.standard_normal((64, 64, 64)).astype(np.float32)
    q = synth.super_fibonacci(n_rot).astype(np.float32)
    w = np.full(n_rot, 1.0 / n_rot)
    pos = np.array([[30, 31, 32], [25, 40, 22]], dtype=np.int32)
    lam = np.array([0.3, -0.1])
    rho, D, flags = ttm.snorm(dev(img), dev(tmpl), dev(mask), n, q, w, dev(pos, torch.int32),
                              dev(lam, torch.float64))
    torch.cuda.synchronize()
    _check(img, tmpl, mask, n, q, w, pos, lam, rho, D, flags, [0, 0])


def _partial_D(args):
    h, m, n, q, w = args
    return O.s_prime_norm2(h, m, n, q, w)


def _oracle_D_parallel(h, m, n, q, w, workers):
    """D is a sum over the quadrature: the oracle's partial sums over chunks
    of the rotation list, in worker processes, added in chunk order."""
    chunks = np.array_split(np.arange(len(q)), workers * 4)
    jobs = [(h, m, n, q[c], w[c]) for c in chunks]
    with cf.ProcessPoolExecutor(workers, mp_context=mp.get_context("spawn")) as ex:
        return float(sum(ex.map(_partial_D, jobs)))


def test_snorm_full_size_peaks():
    """256^3 tomogram, 32^3 template, order 4, 10^4 rotations: the peaks of
    ttm_match (iterated refinement) with the device count, as the benchmark
    calls it.  The template's D and the best peak's D against the oracle; for
    every peak rho' = lambda / sqrt(D Dt) and no flags."""
    wl = synth.workload_tomogram()
    n = 4
    q = synth.super_fibonacci(10000).astype(np.float32)
    w = np.full(len(q), 1.0 / len(q))
    img, tmpl, mask = dev(wl.image), dev(wl.template), dev(wl.mask)
    comps, bank = ttm.build_tensor_template(tmpl, mask, n, q, w, image_shape=wl.image.shape)
    opt = ttm.default_options(max_peaks=len(wl.positions), min_dist=16.0, threshold=0.0, refine=3)
    bufs = ttm.MatchBuffers(wl.image.shape, wl.template.shape, n, opt, "cuda")
    ttm.match(img, bank, mask, n, opt, bufs, tmpl=tmpl)
    rho, D, flags = ttm.snorm(img, tmpl, mask, n, q, w, bufs.pos, bufs.lam, count=bufs.count)
    torch.cuda.synchronize()
    res = bufs.result()
    cnt = res["count"]
    assert cnt > 0
    Dn = D.cpu().numpy()
    lam = bufs.lam.cpu().numpy()[:cnt]
    r = rho.cpu().numpy()[:cnt]
    assert np.all(flags.cpu().numpy()[:cnt] == 0)
    assert np.all(Dn[:cnt] > 0) and Dn[-1] > 0
    rel = np.abs(r - lam / np.sqrt(Dn[:cnt] * Dn[-1])) / np.abs(r)
    assert rel.max() <= 1e-6
    workers = max(1, min(16, os.cpu_count() or 1))
    m64 = wl.mask.astype(np.float64)
    Dt = _oracle_D_parallel(wl.template.astype(np.float64), m64, n, q.astype(np.float64), w, workers)
    x = res["pos"].cpu().numpy()[0]
    c = np.array(wl.template.shape) // 2
    lo = x - c
    win = wl.image[lo[0]:lo[0] + 32, lo[1]:lo[1] + 32, lo[2]:lo[2] + 32].astype(np.float64)
    Dx = _oracle_D_parallel(win, m64, n, q.astype(np.float64), w, workers)
    print(f"\n{cnt} peaks: D(template) GPU {Dn[-1]:.6f} oracle {Dt:.6f}; best peak D GPU {Dn[0]:.6f} "
          f"oracle {Dx:.6f}; rho' range [{r.min():.3f}, {r.max():.3f}]")
    assert abs(Dn[-1] - Dt) <= 1e-6 + 1e-4 * abs(Dt)
    assert abs(Dn[0] - Dx) <= 1e-6 + 1e-4 * abs(Dx)
