"""Seeded synthetic inputs shaped like cryo-electron tomography data.

This module only *generates inputs*: blob templates, tomograms with planted
rotated copies, additive noise, and rotation sets (quadratures) on the unit
quaternion sphere.  It holds none of the matching method's arithmetic (no
correlation, normalisation, tensor construction or pose recovery), so both the
FP64 oracle and the HIP path can consume what it produces.

Conventions shared by every consumer (each consumer implements them itself):

* arrays are C-order ``[n0][n1][n2]`` with ``n2`` fastest; voxel ``(i0,i1,i2)``
  sits at the point ``u = (i0, i1, i2)``;
* a unit quaternion is ``(a, b, c, d) = a + b i + c j + d k``, scalar first; it
  acts on 3-vectors as the active Hamilton rotation ``v -> q v q*`` with the
  vector part ``(b, c, d)`` on axes ``(0, 1, 2)``;
* a template of edge ``L`` is centred at the integer voxel ``L // 2``; a copy of
  the template rotated by ``R`` and placed at image voxel ``x`` means
  ``f(x + u - c) = t(c + R^-1 (u - c))``.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# Super-Fibonacci spiral constants (Alexa, "Super-Fibonacci Spirals", CVPR 2022):
# phi = sqrt(2) and psi the real root of psi^4 = psi + 4.
_SF_PHI = math.sqrt(2.0)
_SF_PSI = 1.533751168755204288118041


def super_fibonacci(n: int) -> np.ndarray:
    """``n`` near-uniform unit quaternions on S^3 (float64, shape (n, 4)),
    canonicalised to a non-negative scalar part."""
    s = np.arange(n, dtype=np.float64) + 0.5
    r = np.sqrt(s / n)
    big_r = np.sqrt(1.0 - s / n)
    alpha = 2.0 * np.pi * s / _SF_PHI
    beta = 2.0 * np.pi * s / _SF_PSI
    q = np.stack([r * np.sin(alpha), r * np.cos(alpha),
                  big_r * np.sin(beta), big_r * np.cos(beta)], axis=1)
    return _canon(q)


def _canon(q: np.ndarray) -> np.ndarray:
    q = np.array(q, dtype=np.float64, copy=True)
    q /= np.linalg.norm(q, axis=-1, keepdims=True)
    flip = q[..., 0] < 0
    q[flip] *= -1.0
    return q


def random_quaternions(rng: np.random.Generator, n: int) -> np.ndarray:
    """Uniform random rotations (normalised 4-D Gaussians), scalar part >= 0."""
    return _canon(rng.standard_normal((n, 4)))


def binary_tetrahedral() -> np.ndarray:
    """The 24 unit quaternions of the binary tetrahedral group."""
    out = []
    for i in range(4):
        for s in (1.0, -1.0):
            v = np.zeros(4)
            v[i] = s
            out.append(v)
    for sa in (1, -1):
        for sb in (1, -1):
            for sc in (1, -1):
                for sd in (1, -1):
                    out.append(0.5 * np.array([sa, sb, sc, sd], dtype=np.float64))
    return np.array(out)


def binary_octahedral() -> np.ndarray:
    """The 48 unit quaternions of the binary octahedral group (the 24 rotations
    of the cube, each with both signs)."""
    out = list(binary_tetrahedral())
    h = 1.0 / math.sqrt(2.0)
    for i in range(4):
        for j in range(i + 1, 4):
            for si in (1, -1):
                for sj in (1, -1):
                    v = np.zeros(4)
                    v[i] = si * h
                    v[j] = sj * h
                    out.append(v)
    return np.array(out)


def _rotmat(q: np.ndarray) -> np.ndarray:
    """Rotation matrix of a unit quaternion (used here only to render plants)."""
    a, b, c, d = q
    return np.array([
        [a * a + b * b - c * c - d * d, 2 * (b * c - a * d), 2 * (b * d + a * c)],
        [2 * (b * c + a * d), a * a - b * b + c * c - d * d, 2 * (c * d - a * b)],
        [2 * (b * d - a * c), 2 * (c * d + a * b), a * a - b * b - c * c + d * d],
    ])


@dataclasses.dataclass
class BlobTemplate:
    """A sum of anisotropic Gaussian blobs, defined in template-centred
    coordinates ``v = u - c``: ``t(v) = sum_b amp_b exp(-1/2 (v-mu_b)^T P_b (v-mu_b))``."""
    L: int
    centres: np.ndarray      # (B, 3)
    precisions: np.ndarray   # (B, 3, 3) inverse covariances
    amps: np.ndarray         # (B,)

    def evaluate(self, v: np.ndarray) -> np.ndarray:
        """Evaluate at template-centred points ``v`` of shape (..., 3)."""
        out = np.zeros(v.shape[:-1])
        for mu, prec, amp in zip(self.centres, self.precisions, self.amps):
            d = v - mu
            q = np.einsum("...i,ij,...j->...", d, prec, d)
            out += amp * np.exp(-0.5 * q)
        return out

    def grid(self) -> np.ndarray:
        """The template sampled on its own L^3 grid (float64)."""
        L = self.L
        c = L // 2
        ax = np.arange(L, dtype=np.float64) - c
        v = np.stack(np.meshgrid(ax, ax, ax, indexing="ij"), axis=-1)
        return self.evaluate(v)


def make_blob_template(rng: np.random.Generator, L: int, n_blobs: int,
                       radius: float) -> BlobTemplate:
    """Random blob template: covariance ``U diag(sigma^2) U^T`` with a random
    rotation ``U`` and ``sigma_i ~ U[L/16, L/8]``, centres uniform in the ball of
    radius ``0.55 radius`` (spread out, so that the template has no rotational
    symmetry and a well-defined pose), amplitudes ``~ U[0.5, 1.5]``."""
    sig_lo, sig_hi = L / 16.0, L / 8.0
    centres, precs, amps = [], [], []
    for _ in range(n_blobs):
        sig = rng.uniform(sig_lo, sig_hi, size=3)
        u = _rotmat(random_quaternions(rng, 1)[0])
        cov = u @ np.diag(sig ** 2) @ u.T
        rmax = 0.55 * radius
        while True:
            p = rng.uniform(-rmax, rmax, size=3)
            if np.linalg.norm(p) <= rmax:
                break
        centres.append(p)
        precs.append(np.linalg.inv(cov))
        amps.append(rng.uniform(0.5, 1.5))
    return BlobTemplate(L, np.array(centres), np.array(precs), np.array(amps))


def ball_mask(L: int, radius: float) -> np.ndarray:
    """Binary spherical mask on the L^3 template grid: 1 where the distance to
    the centre voxel ``L // 2`` is strictly below ``radius``."""
    c = L // 2
    ax = np.arange(L, dtype=np.float64) - c
    v = np.stack(np.meshgrid(ax, ax, ax, indexing="ij"), axis=-1)
    return (np.linalg.norm(v, axis=-1) < radius).astype(np.float64)


def plant_positions(rng: np.random.Generator, shape, L: int, count: int,
                    min_sep: float, max_tries: int = 200000) -> np.ndarray:
    """Integer centres uniform in the region where a whole L-box fits, with
    rejection so that centres are at least ``min_sep`` apart."""
    c = L // 2
    lo = np.array([c, c, c])
    hi = np.array(shape) - (L - c)          # inclusive upper bound
    pts = []
    tries = 0
    while len(pts) < count:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("could not place the requested number of copies")
        p = np.array([rng.integers(lo[i], hi[i] + 1) for i in range(3)])
        if all(np.linalg.norm(p - q) >= min_sep for q in pts):
            pts.append(p)
    return np.array(pts, dtype=np.int64)


def render_copies(shape, tmpl: BlobTemplate, positions: np.ndarray,
                  quats: np.ndarray, extent: int | None = None) -> np.ndarray:
    """Image (float64) holding the analytic blob template rotated by ``quats[p]``
    and centred at ``positions[p]``: value at voxel ``y`` is
    ``t(R^-1 (y - x_p))`` in template-centred coordinates (no interpolation)."""
    img = np.zeros(shape, dtype=np.float64)
    ext = tmpl.L if extent is None else extent
    for x, q in zip(positions, quats):
        r = _rotmat(q)
        lo = [max(int(x[i]) - ext, 0) for i in range(3)]
        hi = [min(int(x[i]) + ext + 1, shape[i]) for i in range(3)]
        ax = [np.arange(lo[i], hi[i], dtype=np.float64) - x[i] for i in range(3)]
        y = np.stack(np.meshgrid(*ax, indexing="ij"), axis=-1)
        v = y @ r               # row-vector form of R^T y = R^-1 y
        img[lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]] += tmpl.evaluate(v)
    return img


@dataclasses.dataclass
class Workload:
    """A seeded synthetic template-matching problem."""
    name: str
    image: np.ndarray          # float32 (n0, n1, n2)
    template: np.ndarray       # float32 (L, L, L)
    mask: np.ndarray           # float32 (L, L, L)
    order: int
    positions: np.ndarray      # (P, 3) int64 planted centres
    true_quats: np.ndarray     # (P, 4) planted rotations
    noise_sigma: float
    radius: float


def make_workload(name: str, shape, L: int, order: int, n_plants: int,
                  seed: int, n_blobs: int = 6, radius: float | None = None,
                  noise_sigma: float | None = None, snr: float | None = None,
                  min_sep: float | None = None) -> Workload:
    """Build a planted-template tomogram.  Sub-seeds: +0 template, +1 positions,
    +2 rotations, +3 noise.  Noise is additive Gaussian; with ``snr`` given its
    standard deviation is ``sqrt(var_signal / snr)`` where ``var_signal`` is the
    variance of the template over its mask."""
    r = L / 2.0 if radius is None else radius
    tmpl = make_blob_template(np.random.default_rng(seed), L, n_blobs, r)
    tgrid = tmpl.grid()
    mask = ball_mask(L, r)
    pos = plant_positions(np.random.default_rng(seed + 1), shape, L, n_plants,
                          float(L) if min_sep is None else min_sep)
    quats = random_quaternions(np.random.default_rng(seed + 2), n_plants)
    img = render_copies(tuple(shape), tmpl, pos, quats)
    if noise_sigma is None:
        if snr is None:
            noise_sigma = 0.0
        else:
            vals = tgrid[mask > 0]
            noise_sigma = math.sqrt(float(vals.var()) / snr)
    if noise_sigma > 0:
        img += noise_sigma * np.random.default_rng(seed + 3).standard_normal(img.shape)
    return Workload(name, img.astype(np.float32), tgrid.astype(np.float32),
                    mask.astype(np.float32), order, pos, quats, float(noise_sigma), r)


# Named workloads (sizes of the configurations this library is measured on).
def workload_small(seed: int = 1000) -> Workload:
    """64^3 image, N(0, 0.3^2) noise, 3 copies of a 16^3 four-blob template,
    mask radius 8, tensor order 2."""
    return make_workload("ttm-64c-L16-n2", (64, 64, 64), 16, 2, 3, seed,
                         n_blobs=4, radius=8.0, noise_sigma=0.3)


def workload_tomogram(seed: int = 2000) -> Workload:
    """256^3 tomogram, 50 copies of a 32^3 random-blob template, SNR 0.1,
    tensor order 4."""
    return make_workload("ttm-256c-L32-n4", (256, 256, 256), 32, 4, 50, seed,
                         n_blobs=6, snr=0.1)


def add_smooth_decoys(wl: Workload, seed: int, count: int, sigma: float = 5.0,
                      amplitude: float = 3.0) -> tuple:
    """The workload's image with ``count`` smooth radial decoys added:
    Gaussian bumps of width ``sigma`` voxels and peak height ``amplitude``
    times the noise standard deviation, centred in the region where a whole
    template box fits, at least one template extent from every copy and from
    each other.  Such windows are smooth where the copies are noisy: the
    situation in which an S-normalised tensor score can rank a non-match above
    a match.  Returns (Workload with the new image and name, decoy centres)."""
    L = wl.template.shape[0]
    rng = np.random.default_rng(seed)
    c = L // 2
    shape = wl.image.shape
    lo = np.array([c, c, c])
    hi = np.array(shape) - (L - c)
    taken = [np.asarray(p) for p in wl.positions]
    pts = []
    tries = 0
    while len(pts) < count:
        tries += 1
        if tries > 200000:
            raise RuntimeError("could not place the requested number of decoys")
        p = np.array([rng.integers(lo[i], hi[i] + 1) for i in range(3)])
        if all(np.linalg.norm(p - q) >= L for q in taken + pts):
            pts.append(p)
    img = wl.image.astype(np.float64)
    amp = amplitude * (wl.noise_sigma if wl.noise_sigma > 0 else 1.0)
    ext = int(math.ceil(4.0 * sigma))
    for x in pts:
        a = [max(int(x[i]) - ext, 0) for i in range(3)]
        b = [min(int(x[i]) + ext + 1, shape[i]) for i in range(3)]
        ax = [np.arange(a[i], b[i], dtype=np.float64) - x[i] for i in range(3)]
        r2 = ax[0][:, None, None] ** 2 + ax[1][None, :, None] ** 2 + ax[2][None, None, :] ** 2
        img[a[0]:b[0], a[1]:b[1], a[2]:b[2]] += amp * np.exp(-r2 / (2.0 * sigma * sigma))
    out = dataclasses.replace(wl, name=wl.name + f"-decoys{count}", image=img.astype(np.float32))
    return out, np.array(pts, dtype=np.int64)


def workload_precision(seed: int = 3000) -> Workload:
    """512x512x256 tomogram, 40^3 template, tensor order 6, SNR 0.1."""
    return make_workload("ttm-512x512x256-L40-n6", (512, 512, 256), 40, 6, 40,
                         seed, n_blobs=6, snr=0.1)


def workload_grad(seed: int = 5000) -> Workload:
    """128^3 image, 24^3 template, order 4, 20 copies, SNR 0.1."""
    return make_workload("ttm-128c-L24-n4", (128, 128, 128), 24, 4, 20, seed,
                         n_blobs=6, snr=0.1)


@dataclasses.dataclass
class BatchWorkload:
    """Uneven tomograms, each holding copies of several templates."""
    name: str
    templates: list            # float32 (L, L, L) per template
    masks: list                # float32 (L, L, L) per template
    images: list               # float32 cubic tomograms of uneven edges
    positions: list            # per tomogram, per template: (P, 3) int64 centres
    true_quats: list           # per tomogram, per template: (P, 4)
    noise_sigma: float
    order: int


def _batch_tomogram(args):
    """Tomogram i of workload_batch (independent sub-seeds, so tomograms can be
    generated in any order or in parallel)."""
    i, S, seed, tmpls, template_sizes, plants_per_template, sigma, sep = args
    prng = np.random.default_rng(seed + 10 + 3 * i)
    # the largest templates first; a placement that gets stuck restarts
    order_t = sorted(range(len(template_sizes)), key=lambda k: -template_sizes[k])
    for _ in range(1000):
        placed = []                          # (centre, L)
        per_t = [None] * len(template_sizes)
        ok = True
        for k in order_t:
            L = template_sizes[k]
            c = L // 2
            pts = []
            tries = 0
            while len(pts) < plants_per_template:
                tries += 1
                if tries > 2000:
                    ok = False
                    break
                p = np.array([prng.integers(c, S - (L - c) + 1) for _ in range(3)])
                if all(np.linalg.norm(p - q) >= sep * (L + Lq) / 2.0 for q, Lq in placed):
                    pts.append(p)
                    placed.append((p, L))
            if not ok:
                break
            per_t[k] = np.array(pts, dtype=np.int64)
        if ok:
            break
    else:
        raise RuntimeError("could not place the copies")
    qrng = np.random.default_rng(seed + 11 + 3 * i)
    qs = [random_quaternions(qrng, plants_per_template) for _ in template_sizes]
    img = np.zeros((S, S, S), dtype=np.float64)
    for t, p, q in zip(tmpls, per_t, qs):
        img += render_copies((S, S, S), t, p, q)
    img = img.astype(np.float32)
    if sigma > 0:
        img += np.float32(sigma) * np.random.default_rng(seed + 12 + 3 * i).standard_normal(
            img.shape, dtype=np.float32)
    return img, per_t, qs


def workload_batch(seed: int = 4000, count: int = 64, edges=(96, 320), template_sizes=(24, 32, 48),
                   plants_per_template: int = 3, snr: float = 0.1, order: int = 4,
                   n_blobs: int = 6, sep: float = 1.0, workers: int = 1) -> BatchWorkload:
    """``count`` cubic tomograms with edges uniform in ``edges`` (inclusive),
    each holding ``plants_per_template`` copies of every template (random-blob
    templates of the given edges, mask radius L/2).  Copies of templates a and
    b are at least sep (L_a + L_b)/2 apart (placed largest template first;
    with sep = 1 the template boxes do not overlap).
    Additive Gaussian noise with standard deviation sqrt(mean template
    variance over its mask / snr).  Sub-seeds: +0 templates, +1 edges, then
    per tomogram i: +10+3i positions, +11+3i rotations, +12+3i noise, so the
    result does not depend on ``workers`` (processes generating tomograms)."""
    trng = np.random.default_rng(seed)
    tmpls = [make_blob_template(trng, L, n_blobs, L / 2.0) for L in template_sizes]
    grids = [t.grid() for t in tmpls]
    masks = [ball_mask(L, L / 2.0) for L in template_sizes]
    var = float(np.mean([g[m > 0].var() for g, m in zip(grids, masks)]))
    sigma = math.sqrt(var / snr) if snr else 0.0
    sizes = np.random.default_rng(seed + 1).integers(edges[0], edges[1] + 1, count)
    jobs = [(i, int(S), seed, tmpls, tuple(template_sizes), plants_per_template, sigma, sep)
            for i, S in enumerate(sizes)]
    if workers > 1:
        import multiprocessing as mp
        with mp.get_context("spawn").Pool(workers) as pool:
            res = pool.map(_batch_tomogram, jobs, chunksize=1)
    else:
        res = [_batch_tomogram(j) for j in jobs]
    return BatchWorkload(f"ttm-batch{count}-e{edges[0]}-{edges[1]}-L{'-'.join(map(str, template_sizes))}-n{order}",
                         [g.astype(np.float32) for g in grids], [m.astype(np.float32) for m in masks],
                         [r[0] for r in res], [r[1] for r in res], [r[2] for r in res], sigma, order)


# --- two-dimensional workloads ------------------------------------------------

def make_blob_template_2d(rng: np.random.Generator, L: int, n_blobs: int, radius: float) -> BlobTemplate:
    """Planar blob template: as :func:`make_blob_template` in two dimensions
    (covariance ``U diag(sigma^2) U^T`` with a random plane rotation ``U``,
    ``sigma_i ~ U[L/16, L/8]``, centres in the disc of radius ``0.55 radius``)."""
    sig_lo, sig_hi = L / 16.0, L / 8.0
    centres, precs, amps = [], [], []
    for _ in range(n_blobs):
        sig = rng.uniform(sig_lo, sig_hi, size=2)
        a = rng.uniform(0.0, 2.0 * math.pi)
        u = np.array([[math.cos(a), -math.sin(a)], [math.sin(a), math.cos(a)]])
        cov = u @ np.diag(sig ** 2) @ u.T
        rmax = 0.55 * radius
        while True:
            p = rng.uniform(-rmax, rmax, size=2)
            if np.linalg.norm(p) <= rmax:
                break
        centres.append(p)
        precs.append(np.linalg.inv(cov))
        amps.append(rng.uniform(0.5, 1.5))
    return BlobTemplate(L, np.array(centres), np.array(precs), np.array(amps))


def disc_mask(L: int, radius: float) -> np.ndarray:
    """Binary disc on the L^2 grid: 1 where the distance to ``L // 2`` is
    strictly below ``radius``."""
    c = L // 2
    ax = np.arange(L, dtype=np.float64) - c
    v = np.stack(np.meshgrid(ax, ax, indexing="ij"), axis=-1)
    return (np.linalg.norm(v, axis=-1) < radius).astype(np.float64)


def circle_quadrature(n: int) -> np.ndarray:
    """``n`` unit complex numbers z = (cos psi, sin psi) with psi equispaced in
    [0, pi): plane rotations by theta = 2 psi, equispaced over the full turn."""
    psi = (np.arange(n, dtype=np.float64) + 0.5) * (math.pi / n)
    return np.stack([np.cos(psi), np.sin(psi)], axis=1)


@dataclasses.dataclass
class Workload2D:
    """A stack of seeded planar template-matching problems sharing one template."""
    name: str
    images: np.ndarray         # float32 (B, n1, n2)
    template: np.ndarray       # float32 (L, L)
    mask: np.ndarray           # float32 (L, L)
    order: int
    positions: list            # per image: (P, 2) int64 planted centres
    angles: list               # per image: (P,) planted rotation angles (radians)
    noise_sigma: float


def workload_2d(seed: int = 7000, count: int = 16, size: int = 512, L: int = 32, order: int = 8,
                plants: int = 12, snr: float = 0.5, n_blobs: int = 5) -> Workload2D:
    """``count`` images of ``size``^2, each with ``plants`` copies of one planar
    blob template (rendered analytically at ``R^-1 (y - x)``, uniform angles),
    at least L apart, plus Gaussian noise of variance ``var_signal / snr``.
    Sub-seeds: +0 template, then +1 + 3i, +2 + 3i, +3 + 3i for the positions,
    angles and noise of image i."""
    r = L / 2.0
    tmpl = make_blob_template_2d(np.random.default_rng(seed), L, n_blobs, r)
    c = L // 2
    ax = np.arange(L, dtype=np.float64) - c
    tgrid = tmpl.evaluate(np.stack(np.meshgrid(ax, ax, indexing="ij"), axis=-1))
    mask = disc_mask(L, r)
    sigma = math.sqrt(float(tgrid[mask > 0].var()) / snr)
    images, positions, angles = [], [], []
    for i in range(count):
        rng_p = np.random.default_rng(seed + 1 + 3 * i)
        pts = []
        tries = 0
        while len(pts) < plants:
            tries += 1
            if tries > 200000:
                raise RuntimeError("could not place the requested number of copies")
            p = np.array([rng_p.integers(c, size - (L - c) + 1) for _ in range(2)])
            if all(np.linalg.norm(p - q) >= L for q in pts):
                pts.append(p)
        ang = np.random.default_rng(seed + 2 + 3 * i).uniform(0.0, 2.0 * math.pi, plants)
        img = np.zeros((size, size))
        for x, a in zip(pts, ang):
            rm = np.array([[math.cos(a), -math.sin(a)], [math.sin(a), math.cos(a)]])
            lo = [max(int(x[k]) - L, 0) for k in range(2)]
            hi = [min(int(x[k]) + L + 1, size) for k in range(2)]
            g = np.stack(np.meshgrid(np.arange(lo[0], hi[0]) - x[0], np.arange(lo[1], hi[1]) - x[1],
                                     indexing="ij"), axis=-1).astype(np.float64)
            img[lo[0]:hi[0], lo[1]:hi[1]] += tmpl.evaluate(g @ rm)   # row-vector form of R^-1 y
        img += sigma * np.random.default_rng(seed + 3 + 3 * i).standard_normal(img.shape)
        images.append(img.astype(np.float32))
        positions.append(np.array(pts, dtype=np.int64))
        angles.append(ang)
    name = f"ttm2d-{count}x{size}sq-L{L}-n{order}"
    return Workload2D(name, np.stack(images), tgrid.astype(np.float32), mask.astype(np.float32), order,
                      positions, angles, sigma)
