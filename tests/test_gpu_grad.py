"""The adjoint of correlate + normalise + score (ttm_score_backward, and the
TTMScore autograd function built on it) against the float64 oracle gradient
(oracle.score_grad, itself pinned by central finite differences in
test_oracle_pins.py), and a template refinement from detections that uses it.

Tolerance: the float32 rotation passes and atomics give gradients within
2e-3 of the largest oracle entry (template) and 1e-3 (image).
"""
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


def _compare(got, ref, rel):
    scale = np.abs(ref).max()
    err = np.abs(got - ref).max()
    assert err <= rel * scale, (err, scale)
    return err / scale


def test_score_backward_small_matches_oracle():
    rng = np.random.default_rng(81)
    L, n = 10, 4
    tm = synth.make_blob_template(rng, L, 4, L / 2)
    t = tm.grid().astype(np.float32)
    m = synth.ball_mask(L, 4.6).astype(np.float32)
    q = synth.random_quaternions(rng, 64).astype(np.float32)
    w = rng.uniform(0.5, 1.5, 64)
    w /= w.sum()
    f = rng.standard_normal((40, 40, 40)).astype(np.float32)
    f += (2.0 * synth.render_copies((40, 40, 40), tm, np.array([[20, 20, 20]]), q[:1])).astype(np.float32)
    xs = np.array([[20, 20, 20], [22, 19, 21], [10, 30, 12], [2, 2, 2]], dtype=np.int32)   # last: invalid
    gF = np.array([1.0, -0.4, 0.6, 3.0], dtype=np.float32)
    comps, _ = ttm.build_tensor_template(dev(t), dev(m), n, q, w)
    gt, gi = ttm.score_backward(dev(f), dev(t), dev(m), n, q, w, comps, xs, dev(gF))
    rt, ri = O.score_grad(f.astype(np.float64), t.astype(np.float64), m.astype(np.float64), n,
                          q.astype(np.float64), w, xs, gF.astype(np.float64))
    et = _compare(gt.cpu().numpy(), rt, 2e-3)
    ei = _compare(gi.cpu().numpy(), ri, 1e-3)
    print(f"\nsmall case: template gradient rel err {et:.2e}, image gradient rel err {ei:.2e}")
    # the invalid position contributes nothing
    assert np.all(gi.cpu().numpy()[:7, :7, :7] == 0.0)


def test_score_backward_gradient_workload_matches_oracle():
    """128^3 image, 24^3 template, order 4, the 20 planted peaks."""
    wl = synth.workload_grad()
    n = wl.order
    q = synth.super_fibonacci(200).astype(np.float32)
    w = np.full(len(q), 1.0 / len(q))
    comps, _ = ttm.build_tensor_template(dev(wl.template), dev(wl.mask), n, q, w)
    gF = np.ones(len(wl.positions), dtype=np.float32)
    gt, gi = ttm.score_backward(dev(wl.image), dev(wl.template), dev(wl.mask), n, q, w, comps,
                                wl.positions, dev(gF))
    rt, ri = O.score_grad(wl.image.astype(np.float64), wl.template.astype(np.float64),
                          wl.mask.astype(np.float64), n, q.astype(np.float64), w, wl.positions,
                          gF.astype(np.float64))
    et = _compare(gt.cpu().numpy(), rt, 2e-3)
    ei = _compare(gi.cpu().numpy(), ri, 1e-3)
    print(f"\n{wl.name}: template gradient rel err {et:.2e}, image gradient rel err {ei:.2e}")


def test_autograd_function_and_template_refinement():
    """TTMScore: the forward is the FFT correlation read at the positions, the
    backward the adjoint; 100 steps of normalised gradient ascent on
    sum_p F(x_p) from a noise-perturbed template raise the objective (the
    correlation with the planted template is reported: at SNR 0.1 the
    aligned average of 20 copies is itself noisier than the 20% perturbation,
    so the objective, not the correlation, is what ascent guarantees)."""
    wl = synth.workload_grad()
    n = wl.order
    q = synth.super_fibonacci(500).astype(np.float32)
    w = np.full(len(q), 1.0 / len(q))
    img = dev(wl.image)
    mask = dev(wl.mask)
    truth = dev(wl.template)
    rng = np.random.default_rng(5)
    t0 = wl.template + 0.2 * wl.template.std() * rng.standard_normal(wl.template.shape)
    t = dev(t0).requires_grad_(True)
    F = ttm.TTMScore.apply(t, img, mask, n, q, w, wl.positions)
    # the forward agrees with the direct float64 evaluation at the positions
    T = O.tensor_template(t0.astype(np.float32).astype(np.float64), wl.mask.astype(np.float64), n,
                          q.astype(np.float64), w)
    F_ref = O.score_from_field(O.tensor_field_at(wl.image.astype(np.float64), T, wl.mask.astype(np.float64),
                                                 wl.positions), n)
    assert np.abs(F.detach().cpu().numpy() - F_ref).max() <= 1e-4
    F.sum().backward()
    gt, _ = ttm.score_backward(img, t.detach(), mask, n, q, w,
                               ttm.build_tensor_template(t.detach(), mask, n, q, w)[0], wl.positions,
                               torch.ones(len(wl.positions), device="cuda"), want_image=False)
    assert torch.allclose(t.grad, gt, rtol=0, atol=1e-6 * float(gt.abs().max()))

    m = mask > 0

    def corr(a):
        a = a[m] - a[m].mean()
        b = truth[m] - truth[m].mean()
        return float((a * b).sum() / (a.norm() * b.norm()))

    x = dev(t0)
    obj0 = float(ttm.TTMScore.apply(x, img, mask, n, q, w, wl.positions).sum())
    c0 = corr(x)
    step = 0.003 * float(x.norm())
    for _ in range(100):
        xr = x.clone().requires_grad_(True)
        ttm.TTMScore.apply(xr, img, mask, n, q, w, wl.positions).sum().backward()
        g = xr.grad
        x = x + step * g / (g.norm() + 1e-30)
    obj1 = float(ttm.TTMScore.apply(x, img, mask, n, q, w, wl.positions).sum())
    c1 = corr(x)
    print(f"\nrefinement: objective {obj0:.4f} -> {obj1:.4f}, correlation with the planted template "
          f"{c0:.4f} -> {c1:.4f}")
    assert obj1 > obj0
