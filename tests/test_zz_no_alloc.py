"""ttm_pose_at_noalloc (the pose at given positions with the library's static
device scratch, for callers that cannot allocate) against ttm_pose_at with a
caller workspace: the same outputs bit for bit, on two calls in a row, the
second with a smaller input; sizes beyond the static scratch are refused."""
import ctypes

import numpy as np
import pytest
import torch

from oracle import ttm_oracle as O
from paper_2311_07561_amd import synth, ttm

pytestmark = pytest.mark.gpu


def dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def _case(seed, N, L, n, nrot, npl):
    rng = np.random.default_rng(seed)
    img = (0.1 * rng.standard_normal(N)).astype(np.float32)
    tm = synth.make_blob_template(rng, L, 4, L / 2)
    tmpl = tm.grid().astype(np.float32)
    mask = synth.ball_mask(L, L / 2).astype(np.float32)
    q = synth.super_fibonacci(nrot).astype(np.float32)
    w = np.full(nrot, 1.0 / nrot)
    c = L // 2
    centres = []
    for k, qp in enumerate(synth.random_quaternions(rng, npl)):
        x = np.array([c + 2 + k * (L + 1), N[1] // 2, N[2] // 2])
        s = O.rotated_template(tmpl, mask, qp)
        sl = tuple(slice(x[i] - c, x[i] - c + L) for i in range(3))
        img[sl] += (2.0 * s).astype(np.float32)
        centres.append(x)
    comps, _ = ttm.build_tensor_template(dev(tmpl), dev(mask), n, q, w)
    starts = np.array([x + np.array([1, -1, 1]) for x in centres] + [[c + 1, c + 1, c + 1]], dtype=np.int32)
    return dev(img), comps, dev(mask), dev(tmpl), starts


def _outputs(P, K):
    return dict(pos=torch.full((P, 3), -7, dtype=torch.int32, device="cuda"),
                quat=torch.full((P, 4), -7.0, dtype=torch.float32, device="cuda"),
                lam=torch.full((P,), -7.0, dtype=torch.float64, device="cuda"),
                flags=torch.full((P,), -7, dtype=torch.int32, device="cuda"),
                C=torch.full((P, K), -7.0, dtype=torch.float64, device="cuda"))


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ttm.lib()


def test_noalloc_equals_workspace_call_twice():
    cases = [dict(seed=5, N=(48, 40, 44), L=10, n=4, nrot=600, npl=3, refine=3, max_peaks=8),
             dict(seed=6, N=(24, 28, 20), L=8, n=2, nrot=200, npl=1, refine=2, max_peaks=2)]
    for cs in cases:
        img, comps, mask, tmpl, starts = _case(cs["seed"], cs["N"], cs["L"], cs["n"], cs["nrot"], cs["npl"])
        opt = ttm.default_options(max_peaks=cs["max_peaks"], refine=cs["refine"])
        K = ttm.num_components(cs["n"])
        P = len(starts)
        pos = dev(starts, torch.int32)
        ref = ttm.pose_at(img, comps, mask, cs["n"], starts, opt, want_C=True, tmpl=tmpl)
        out = _outputs(P, K)
        ttm.pose_at_noalloc(img, comps, mask, cs["n"], pos, opt, out, tmpl=tmpl)
        torch.cuda.synchronize()
        for k in ("pos", "quat", "lam", "flags", "C"):
            assert torch.equal(out[k], ref[k]), (cs["seed"], k)
        print(f"\nno-alloc pose at {P} positions of {cs['N']} (order {cs['n']}, refine {cs['refine']}): "
              f"positions {out['pos'].cpu().numpy().tolist()}")


def test_noalloc_refuses_beyond_the_static_scratch():
    L = ttm.lib()
    fake = ctypes.c_void_p(256)
    big = ttm.default_options(max_peaks=4096, refine=3, n_seeds=65536)
    st = L.ttm_pose_at_noalloc(fake, fake, fake, fake, ttm.Dims(64, 64, 64), ttm.Dims(16, 16, 16), 8,
                               ctypes.byref(big), fake, 1, fake, fake, fake, fake, None, None)
    assert st == -3
