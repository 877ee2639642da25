"""The isotropic low-pass filter (ttm_lowpass) against the oracle, and the
whole path on filtered data under a soft (raised-cosine) mask: matching
applied to f * h and t * h with a rotationally symmetric mask that falls
from 1 to 0 between two radii (Section 2)."""
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


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda")


@pytest.mark.parametrize("shape,sigma,periodic", [((37, 48, 29), 1.3, True), ((37, 48, 29), 0.6, False),
                                                   ((16, 16, 16), 2.0, False), ((64, 32, 64), 1.0, True)])
def test_lowpass_matches_oracle(shape, sigma, periodic):
    rng = np.random.default_rng(int(sigma * 10) + shape[0])
    x = rng.standard_normal(shape).astype(np.float32)
    got = ttm.lowpass(dev(x), sigma, periodic).cpu().numpy()
    ref = O.lowpass(x.astype(np.float64), sigma, periodic)
    assert np.abs(got - ref).max() <= 1e-6 * np.abs(x).max()
    # in place
    y = dev(x)
    ttm.lowpass(y, sigma, periodic, out=y)
    assert np.abs(y.cpu().numpy() - ref).max() <= 1e-6 * np.abs(x).max()


def test_filtered_path_with_soft_mask():
    wl = synth.workload_small()
    n, sigma = 4, 1.0
    L = wl.template.shape
    m = O.soft_mask(L, 5.5, 7.5).astype(np.float32)
    q = synth.super_fibonacci(300).astype(np.float32)
    wts = np.full(len(q), 1.0 / len(q))
    f_h = ttm.lowpass(dev(wl.image), sigma, True)
    t_h = ttm.lowpass(dev(wl.template), sigma, False)
    comps, bank = ttm.build_tensor_template(t_h, dev(m), n, q, wts, image_shape=wl.image.shape)
    score, wv = ttm.correlate(f_h, bank, dev(m), n)
    # the oracle filters in float64 and matches with the same soft mask
    f64 = O.lowpass(wl.image.astype(np.float64), sigma, True)
    t64 = O.lowpass(wl.template.astype(np.float64), sigma, False)
    m64 = m.astype(np.float64)
    T = O.tensor_template(t64, m64, n, q.astype(np.float64), wts)
    rng = np.random.default_rng(4)
    lo, hi = O.valid_region(wl.image.shape, L)
    xs = np.concatenate([wl.positions, np.stack([rng.integers(lo[i], hi[i], 300) for i in range(3)], axis=1)])
    C = O.tensor_field_at(f64, T, m64, xs)
    F_ref = O.score_from_field(C, n)
    F = score.cpu().numpy()[xs[:, 0], xs[:, 1], xs[:, 2]]
    assert np.abs(F - F_ref).max() <= 1e-4, np.abs(F - F_ref).max()
    w_ref = O.local_norm_at(f64, m64, xs)
    assert np.allclose(wv.cpu().numpy()[xs[:, 0], xs[:, 1], xs[:, 2]], w_ref, rtol=1e-4)
    # peaks on the GPU map, poses at them, and the NCC refinement with the soft mask
    opt = ttm.default_options(max_peaks=3, min_dist=8.0)
    res = ttm.recover_pose(score, f_h, comps, dev(m), n, opt)
    cand = O.find_peaks_fast(score.cpu().numpy(), L, 0.0, 8.0, 3)
    pos = res["pos"].cpu().numpy()
    assert np.array_equal(pos, cand)
    Cp = O.tensor_field_at(f64, T, m64, pos)
    for i in range(len(pos)):
        qo, lo_, second = O.dominant_z_eigenpair(Cp[i], n, n_brute=60000)
        if second < lo_ - 1e-3 * abs(lo_):
            assert O.rotation_angle_deg(res["quat"].cpu().numpy()[i], qo) <= 1.0
    opt2 = ttm.default_options(max_peaks=3, min_dist=8.0, refine=2)
    r2 = ttm.recover_pose(score, f_h, comps, dev(m), n, opt2, tmpl=t_h)
    p2 = r2["pos"].cpu().numpy()
    assert np.all(np.abs(p2 - cand).max(axis=1) <= 1)
    i0 = 0
    _, _, _, ncc, nccs = O.refine_by_ncc(f64, t64, m64, T, n, cand[i0], n_brute=30000)
    k = int(np.argmax([(p2[i0] - cand[i0] == o).all() for o in O.neighbourhood_offsets()]))
    assert nccs[k] >= ncc - 1e-3
