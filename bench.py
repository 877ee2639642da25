"""Benchmark: tensorial template matching (TTM) on a 256^3 synthetic tomogram
with a 32^3 template at tensor order 4 (35 components), against classical
rotation-sampled NCC template matching at 10^4 rotations on the same GPU.

A step is one ttm_match call over the resident tomogram: image moments, R2C
of f and f^2, K+2 fanned-out spectral products, batched C2R inverses, local
normalisation and Frobenius score, then peak picking and the dominant
Z-eigenpair of the correlated tensor field at every peak and its 26
neighbours; the reported voxel is the one whose NCC at its own rotation is
largest, repeated from the moved peaks until none moves (--refine 3, the
default, at most 4 rounds; 2 stops after one round, 1 keeps the largest
eigenvalue, 0 the peak itself).  The tensor-template build (once per template) is timed separately.

    python bench.py [--gpus 1] [--steps 20] [--warmup 3]

Prints one JSON line on stdout (progress goes to stderr).
"""
from __future__ import annotations

import argparse
import faulthandler
import hashlib
import json
import os
import sys
import time

faulthandler.enable()

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "TTM tomogram voxels/s & HBM GB/s vs classical TM@10k rotations, same pose accuracy"
HBM_PEAK_GBPS = 8000.0
MFMA_F16_PEAK_TFLOPS = 2500.0     # dense fp16 matrix cores
CSRC = os.path.join(ROOT, "paper_2311_07561_amd", "csrc")
PROFILES = os.path.join(ROOT, "profiles")


def source_digest():
    """Digest of the HIP sources: counter summaries taken from other sources
    do not describe the kernels that run now."""
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        if name.endswith((".hip", ".h")):
            h.update(name.encode())
            with open(os.path.join(CSRC, name), "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()[:16]


def counter_traffic(kernel_class, workload):
    """HBM bytes per launch of a kernel class from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary of this workload (each counter scaled by
    its reading for a plain copy of known size), or None when there is no
    summary or the sources changed since it was taken."""
    path = os.path.join(PROFILES, f"{kernel_class}__{workload}__pmc.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("source_digest") != source_digest():
        return None
    try:
        return float(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--build-rotations", type=int, default=10000)
    p.add_argument("--classical-rotations", type=int, default=10000)
    p.add_argument("--refine", type=int, default=3,
                   help="0: pose at each peak; 1: best eigenvalue of the 3x3x3 neighbourhood; "
                        "2: best NCC at each neighbour's own rotation; 3: 2 repeated until no peak moves "
                        "(at most 4 rounds)")
    p.add_argument("--order6", type=int, default=1, help="also time and score tensor order 6")
    p.add_argument("--rmap-seeds", type=int, default=10016,
                   help="also time the all-voxel rotation map with this many seeds (0 = skip)")
    p.add_argument("--rmap-steps", type=int, default=3)
    p.add_argument("--batch", type=int, default=0,
                   help="tomograms of the batching leg (uneven edges 96..320, templates 24/32/48; 0 = skip). "
                        "Refused for now: runs of the 64-tomogram leg have ended with a host segmentation fault "
                        "after its graph replays, and its cause has not been shown")
    p.add_argument("--batch-replays", type=int, default=2)
    p.add_argument("--batch-streams", type=int, default=4, help="concurrent branches of the batch graph")
    p.add_argument("--batch-workers", type=int, default=16, help="processes generating the batch tomograms")
    p.add_argument("--rotations-2d", type=int, default=720,
                   help="rotations of the planar leg's tensor template and classical matching (0: skip the leg)")
    p.add_argument("--snorm-steps", type=int, default=3,
                   help="timed runs of the S'-normalisation of the peaks (0: skip)")
    p.add_argument("--legs", default="correlate,c1,c3,classical45k",
                   help="extra legs: correlate (ttm_correlate + ttm_recover_pose), c1 (64^3 workload, GPU and "
                        "oracle seconds), c3 (512x512x256, order 6), classical45k (classical TM at 45123 rotations)")
    p.add_argument("--cpu-seconds", type=float, default=15.0,
                   help="target CPU time of the oracle baseline sample (0 = skip)")
    p.add_argument("--seed", type=int, default=2000)
    p.add_argument("--profile-json", default="", help="also write the full result here")
    p.add_argument("--copy-calibration", type=int, default=0,
                   help="only copy this many MiB device-to-device (counter calibration) and exit")
    return p.parse_args()


def class_bytes(n0, n1, n2, L0, L1, K):
    """Algorithmic HBM bytes per step of each kernel class of ttm_match, from
    the units U_c (a half spectrum, complex64: 8 n0 n1 (n2/2+1) bytes), U_r (a
    real float32 field: 4 n0 n1 n2 bytes) and B_e (one bank entry: 8 L0 n1
    (n2/2+1) bytes).  Only outputs in the valid region (the window inside the
    image: v0 = n0 - L0 + 1 planes along axis 0, v1 = n1 - L1 + 1 rows along
    axis 1) are carried through the inverse passes, so those passes move the
    fractions r0 = v0 / n0 and r01 = v0 v1 / (n0 n1) of each array."""
    h2 = n2 // 2 + 1
    Uc = 8.0 * n0 * n1 * h2
    Ur = 4.0 * n0 * n1 * n2
    Be = 8.0 * L0 * n1 * h2
    r0 = (n0 - L0 + 1) / n0
    r01 = r0 * (n1 - L1 + 1) / n1
    E = K + 2                                             # K components, mask vs f, mask vs f^2
    return {
        "image_moments": 2 * Ur,                          # f read twice (mean, then variance)
        "r2c_rows": Ur + 2 * Uc,                          # read f; write F2(f), F2(f^2)
        "pencils_fwd": 2 * 2 * Uc,                        # two arrays, read + write
        "pass1_fanout": 2 * Uc + E * Be + E * r0 * Uc,    # F1(f), F1(f^2); E bank reads; E outputs
        "pencils_inv": E * r0 * Uc + E * r01 * Uc,        # E arrays: read v0 planes, write v0 x v1 rows
        "pass3_c2r_reduce": E * r01 * Uc + 2 * Ur,        # read v0 x v1 rows of E arrays; write F and w
        "peaks": Ur,                                      # one scan of F
        "pose": 0.0,
        "units": {"U_c": Uc, "U_r": Ur, "B_e": Be, "r0": r0, "r01": r01, "arrays": E},
    }


def path_model_bytes(n0, n1, n2, K):
    """Algorithmic HBM bytes of one correlation (image R2C, the K + 2 spectral
    products and inverses, local normalisation and score) on the fused
    two-pass model: every 3-D FFT reads and writes its array twice, the K
    template spectra are precomputed and read once, the product is fused into
    the first inverse pass and the score into the last, C is not stored:
    4 U_r + 14 U_c + 3 K U_c (8.32 GB at 256^3, K = 35)."""
    Uc = 8.0 * n0 * n1 * (n2 // 2 + 1)
    Ur = 4.0 * n0 * n1 * n2
    return 4 * Ur + 14 * Uc + 3 * K * Uc


def two_pass_class_bytes(n0, n1, n2, L0, L1, K):
    """Algorithmic HBM bytes of the kernel classes of ttm_correlate on the
    two-pass inverse (axes 1 and 2 of 256): pass A as pass 1 (axis 0 and the
    4-point digit of axis 1), pass B reading the v0 valid planes of the E
    arrays whole and writing F and w."""
    cb = class_bytes(n0, n1, n2, L0, L1, K)
    u = cb["units"]
    E, Uc, Ur, r0 = u["arrays"], u["U_c"], u["U_r"], u["r0"]
    cb["pass3_c2r_reduce"] = E * r0 * Uc + 2 * Ur
    cb.pop("pencils_inv")
    return cb


def time_steps(step, steps, warmup, ttm, torch):
    """Milliseconds per step over ``steps`` uninstrumented steps, then the
    per-kernel-class event timings of as many instrumented steps (the event
    pairs around each kernel group add their own gaps, so they are kept out
    of the step time)."""
    for _ in range(warmup):
        step()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for _ in range(steps):
        step()
    stop.record()
    torch.cuda.synchronize()
    total_ms = start.elapsed_time(stop)
    ttm.profile_enable(True)
    ttm.profile_read()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    prof = ttm.profile_read()
    ttm.profile_enable(False)
    return total_ms / steps, prof


def err_stats(errs):
    if not errs:
        return {"n": 0, "median_deg": None, "p90_deg": None}
    return {"n": len(errs), "median_deg": round(float(np.median(errs)), 3),
            "p90_deg": round(float(np.percentile(errs, 90)), 3)}


def angle_deg(q1, q2):
    """Angle of the rotation taking R(q1) to R(q2): 2 acos |<q1, q2>| (unit
    quaternions, either sign)."""
    q1 = np.asarray(q1, dtype=np.float64)
    q2 = np.asarray(q2, dtype=np.float64)
    d = abs(float(q1 @ q2)) / (np.linalg.norm(q1) * np.linalg.norm(q2))
    return float(np.degrees(2.0 * np.arccos(min(1.0, d))))


def angle2d_deg(z1, z2):
    """Angle between the plane rotations of the half-angle unit complex
    numbers z1 and z2, in [0, 180]."""
    t = 2.0 * (np.arctan2(z2[1], z2[0]) - np.arctan2(z1[1], z1[0]))
    return float(abs(np.degrees((t + np.pi) % (2.0 * np.pi) - np.pi)))


def run_2d(args, ttm, synth, torch, dev):
    """Planar TTM on a stack of 16 images of 512^2 (32^2 template, order 8,
    iterated refinement), against classical matching of the same stack with
    the same rotations on the same GPU."""
    wl = synth.workload_2d()
    B, n1, n2 = wl.images.shape
    L = wl.template.shape
    n = wl.order
    P = len(wl.positions[0])
    J = args.rotations_2d
    zs = synth.circle_quadrature(J).astype(np.float32)
    w = np.full(J, 1.0 / J)
    imgs = torch.as_tensor(wl.images, device=dev)
    tm2 = torch.as_tensor(wl.template, device=dev)
    mk2 = torch.as_tensor(wl.mask, device=dev)
    torch.cuda.synchronize()
    tb = time.time()
    comps, bank = ttm.build_tensor_template_2d(tm2, mk2, n, zs, w, stack_shape=(B, n1, n2))
    torch.cuda.synchronize()
    build_ms = (time.time() - tb) * 1e3
    opt = ttm.default_options(max_peaks=P, min_dist=float(L[0]) / 2, threshold=0.0, refine=args.refine)
    bufs = ttm.Match2DBuffers((B, n1, n2), L, n, opt, dev)
    ms, prof = time_steps(lambda: ttm.match_2d(imgs, bank, comps, mk2, n, opt, bufs, tmpl=tm2), args.steps,
                          args.warmup, ttm, torch)
    errs = []
    for b in range(B):
        res = bufs.result(b)
        pos, z = res["pos"].cpu().numpy(), res["z"].cpu().numpy()
        for x, a in zip(wl.positions[b], wl.angles[b]):
            if len(pos) == 0:
                break
            d = np.linalg.norm(pos - x[None], axis=1)
            i = int(np.argmin(d))
            if d[i] <= 2.0:
                errs.append(angle2d_deg(z[i], [np.cos(a / 2), np.sin(a / 2)]))
    V = B * n1 * n2
    out = {"workload": wl.name, "images": B, "size": [n1, n2], "template": list(L), "order": n,
           "components": n + 1, "rotations": J, "build_ms": round(build_ms, 1), "ms": round(ms, 4),
           "pixels_per_s": V / (ms / 1e3), "refine": args.refine,
           "pose_detected": dict(err_stats(errs), recall=len(errs) / (B * P)),
           "kernels_ms": {k: round(v[0] / args.steps, 4) for k, v in prof.items() if v[1]}}
    log(f"2-D: {B} x {n1}x{n2}, template {L}, order {n}: {ms:.3f} ms per stack "
        f"({V / (ms / 1e3):.3g} pixels/s), recall {len(errs) / (B * P):.2f}, {err_stats(errs)}")
    if args.classical_rotations > 0:
        q3 = np.stack([zs[:, 0], zs[:, 1], np.zeros(J), np.zeros(J)], axis=1).astype(np.float32)
        tm3, mk3 = tm2[None].contiguous(), mk2[None].contiguous()
        ttm.tm_classical(imgs, tm3, mk3, q3[:64])
        torch.cuda.synchronize()
        c0 = torch.cuda.Event(enable_timing=True)
        c1 = torch.cuda.Event(enable_timing=True)
        c0.record()
        best, idx = ttm.tm_classical(imgs, tm3, mk3, q3)
        c1.record()
        torch.cuda.synchronize()
        cms = c0.elapsed_time(c1)
        idx_np = idx.cpu().numpy()
        at = [angle2d_deg(zs[idx_np[b, x[0], x[1]]], [np.cos(a / 2), np.sin(a / 2)])
              for b in range(B) for x, a in zip(wl.positions[b], wl.angles[b])]
        # classical peaks: the same picker, plane by plane, on the best-NCC map
        comps3, _ = ttm.build_tensor_template(tm3, mk3, n, q3, w)
        opt0 = ttm.default_options(max_peaks=P, min_dist=float(L[0]) / 2, threshold=0.0)
        cerr = []
        for b in range(B):
            rc = ttm.recover_pose(best[b:b + 1], imgs[b:b + 1], comps3, mk3, n, opt0, want_C=False)
            cpos = rc["pos"].cpu().numpy()[:, 1:]
            for x, a in zip(wl.positions[b], wl.angles[b]):
                if len(cpos) == 0:
                    break
                d = np.linalg.norm(cpos - x[None], axis=1)
                i = int(np.argmin(d))
                if d[i] <= 2.0:
                    cerr.append(angle2d_deg(zs[idx_np[b, cpos[i, 0], cpos[i, 1]]], [np.cos(a / 2), np.sin(a / 2)]))
        out["classical"] = {"rotations": J, "ms": round(cms, 2), "pixels_per_s": V / (cms / 1e3),
                            "speedup_ttm_vs_classical": round(cms / ms, 1),
                            "pose_at_planted": err_stats(at),
                            "pose_detected": dict(err_stats(cerr), recall=len(cerr) / (B * P))}
        log(f"2-D classical, {J} rotations: {cms:.1f} ms ({cms / ms:.1f}x the TTM stack), detected {err_stats(cerr)}")
        del best, idx
    del bufs
    return out


def match_errors(pos, quats, planted, truth, angle, radius=2.0):
    errs = []
    for p, q in zip(planted, truth):
        if len(pos) == 0:
            break
        d = np.linalg.norm(pos - p[None], axis=1)
        i = int(np.argmin(d))
        if d[i] <= radius:
            errs.append(angle(quats[i], q))
    return errs


def run_snorm(wl, img, tmpl, mask, order, qb, wb, bank, bufs, opt, args, ttm, synth, torch):
    """S'-normalised scores (ttm_snorm, with the device count): the time per
    call on the match's peaks, then how the Frobenius score F, the eigenvalue
    lambda and rho' rank copies against smooth decoys: the same tomogram with
    25 smooth radial bumps added, matched with room for 75 peaks."""
    def call(b):
        return ttm.snorm(img if b is bufs else dimg, tmpl, mask, order, qb, wb, b.pos, b.lam, count=b.count)

    ms, prof = time_steps(lambda: call(bufs), args.snorm_steps, 1, ttm, torch)
    kern = prof.get("snorm", (0.0, 0))
    cnt = int(bufs.count[0])
    nm = int((wl.mask != 0).sum())
    out = {"ms": round(ms, 4), "windows": cnt + 1, "rotations": len(qb), "mask_voxels": nm,
           "voxel_rotations_per_s": (cnt + 1) * len(qb) * nm / (ms / 1e3),
           "kernel_ms": round(kern[0] / args.snorm_steps, 4)}

    dwl, decoys = synth.add_smooth_decoys(wl, args.seed + 4, 25)
    dimg = torch.as_tensor(dwl.image, device=img.device)
    P = len(wl.positions) + len(decoys)
    dopt = ttm.default_options(max_peaks=P, min_dist=opt.min_dist, threshold=0.0, refine=opt.refine)
    dbufs = ttm.MatchBuffers(dwl.image.shape, dwl.template.shape, order, dopt, img.device)
    ttm.match(dimg, bank, mask, order, dopt, dbufs, tmpl=tmpl)
    rho, D, flags = call(dbufs)
    torch.cuda.synchronize()
    n = int(dbufs.count[0])
    pos = dbufs.pos[:n].cpu().numpy()
    near = lambda pts: np.array([np.min(np.linalg.norm(pts - x[None], axis=1)) <= 2.0 for x in pos])
    on_copy, on_decoy = near(wl.positions), near(decoys)
    keys = {"F": dbufs.peak_score[:n].cpu().numpy(), "lambda": dbufs.lam[:n].cpu().numpy(),
            "rho": rho[:n].cpu().numpy(), "D": D[:n].cpu().numpy()}
    k = len(wl.positions)
    ranks = {}
    for name, v in keys.items():
        if name == "D":
            continue
        top = np.argsort(-v, kind="stable")[:k]
        ranks[name] = {"copies": int(on_copy[top].sum()), "decoys": int(on_decoy[top].sum())}

    def med(v):
        return round(float(np.median(v)), 4) if v.size else None

    out["decoys"] = {"workload": dwl.name, "peaks": n, "copies_found": int(on_copy.sum()),
                     "decoys_found": int(on_decoy.sum()), "flags": int(np.count_nonzero(flags[:n].cpu().numpy())),
                     f"top{k}": ranks,
                     "median_on_copies": {nm_: med(v[on_copy]) for nm_, v in keys.items()},
                     "median_on_decoys": {nm_: med(v[on_decoy]) for nm_, v in keys.items()}}
    log(f"S'-normalisation: {ms:.3f} ms for {cnt} peaks + template, {len(qb)} rotations; decoys: "
        f"{n} peaks ({int(on_copy.sum())} copies, {int(on_decoy.sum())} decoys), top {k} by F / lambda / rho': "
        f"{ranks['F']} / {ranks['lambda']} / {ranks['rho']}")
    del dbufs, dimg
    return out


def run_order(order, wl, img, tmpl, mask, args, ttm, synth, torch, dev, angle, with_profile):
    N = wl.image.shape
    L = wl.template.shape
    K = ttm.num_components(order)
    qb = synth.super_fibonacci(args.build_rotations).astype(np.float32)
    wb = np.full(len(qb), 1.0 / len(qb))
    torch.cuda.synchronize()
    tb = time.time()
    comps, bank = ttm.build_tensor_template(tmpl, mask, order, qb, wb, image_shape=N)
    torch.cuda.synchronize()
    build_ms = (time.time() - tb) * 1e3
    log(f"order {order}: tensor template build ({args.build_rotations} rotations) {build_ms:.1f} ms")
    opt = ttm.default_options(max_peaks=len(wl.positions), min_dist=float(L[0]) / 2, threshold=0.0,
                              refine=args.refine)
    bufs = ttm.MatchBuffers(N, L, order, opt, dev)
    score = bufs.score

    def step():
        ttm.match(img, bank, mask, order, opt, bufs, tmpl=tmpl)

    ms, prof = time_steps(step, args.steps, args.warmup, ttm, torch)
    log(f"order {order}: step {ms:.3f} ms")
    res = bufs.result()
    det = match_errors(res["pos"].cpu().numpy(), res["quat"].cpu().numpy(), wl.positions, wl.true_quats, angle)
    out = {"order": order, "components": K, "ms_per_step": ms, "build_ms": round(build_ms, 1),
           "pose_detected": dict(err_stats(det), recall=len(det) / len(wl.positions), refine=args.refine)}
    if args.snorm_steps > 0:
        out["snorm"] = run_snorm(wl, img, tmpl, mask, order, qb, wb, bank, bufs, opt, args, ttm, synth, torch)
    if args.refine == 3:
        # the single-round refinement's step time, for comparison
        opt2 = ttm.default_options(max_peaks=len(wl.positions), min_dist=float(L[0]) / 2, threshold=0.0, refine=2)
        bufs2 = ttm.MatchBuffers(N, L, order, opt2, dev)
        ms2, _ = time_steps(lambda: ttm.match(img, bank, mask, order, opt2, bufs2, tmpl=tmpl), args.steps,
                            args.warmup, ttm, torch)
        out["ms_per_step_refine2"] = round(ms2, 4)
        del bufs2
    for rf in (0, 1, 2, 3):
        if rf == args.refine:
            continue
        opt0 = ttm.default_options(max_peaks=len(wl.positions), min_dist=float(L[0]) / 2, threshold=0.0,
                                   refine=rf)
        r0 = ttm.recover_pose(score, img, comps, mask, order, opt0, want_C=False, tmpl=tmpl)
        d0 = match_errors(r0["pos"].cpu().numpy(), r0["quat"].cpu().numpy(), wl.positions, wl.true_quats, angle)
        out[f"pose_detected_refine{rf}"] = dict(err_stats(d0), recall=len(d0) / len(wl.positions))
    pa = ttm.pose_at(img, comps, mask, order, wl.positions,
                     ttm.default_options(max_peaks=len(wl.positions)), want_C=False)
    at = [angle(q, t) for q, t in zip(pa["quat"].cpu().numpy(), wl.true_quats)]
    out["pose_at_planted"] = err_stats(at)
    out["_prof"] = prof
    out["_score"] = score
    out["_comps"] = comps
    out["_bank"] = bank
    return out


def run_correlate(wl, img, mask, bank, K, comps, tmpl, args, ttm, torch):
    """ttm_correlate alone (the two-pass inverse at this size: pass A = axis 0
    with the 4-point digit of axis 1, pass B = the 64-point digit, axis-2 C2R
    and the score), then ttm_recover_pose (direct float64 tensors) on its
    score at refine 0 / 2 / 3: the boundary's call sequence."""
    N = wl.image.shape
    L = wl.template.shape
    ws = ttm.correlate_workspace(N, L, 4, img.device)
    out = (torch.empty_like(img), torch.empty_like(img))
    ms, prof = time_steps(lambda: ttm.correlate(img, bank, mask, 4, workspace=ws, out=out), args.steps,
                          args.warmup, ttm, torch)
    cb = two_pass_class_bytes(N[0], N[1], N[2], L[0], L[1], K)
    kernels = {}
    for name, (kms, cnt) in prof.items():
        if cnt == 0:
            continue
        ms_step = kms / args.steps
        byts = cb.get(name) or 0.0
        kernels[name] = {"ms_per_step": round(ms_step, 4), "model_bytes_per_step": byts,
                         "model_GBps": round(byts / (ms_step / 1e3) / 1e9, 1) if byts else None}
    pb = path_model_bytes(N[0], N[1], N[2], K)
    gbps = pb / (ms / 1e3) / 1e9
    res = {"ms": round(ms, 4), "voxels_per_s": float(np.prod(N)) / (ms / 1e3),
           "path_model_GB": round(pb / 1e9, 3), "path_GBps": round(gbps, 1),
           "path_frac": round(gbps / HBM_PEAK_GBPS, 4), "kernels": kernels}
    log(f"ttm_correlate: {ms:.3f} ms, {pb / 1e9:.2f} GB model at {gbps:.0f} GB/s = {gbps / HBM_PEAK_GBPS:.3f} of peak")
    pose = {}
    score = out[0]
    for rf in (0, 2, 3):
        opt = ttm.default_options(max_peaks=len(wl.positions), min_dist=float(L[0]) / 2, threshold=0.0, refine=rf)
        call = lambda: ttm.recover_pose(score, img, comps, mask, 4, opt, want_C=False, tmpl=tmpl)
        pms, pprof = time_steps(call, max(2, args.steps // 4), 1, ttm, torch)
        pose[f"refine{rf}_ms"] = round(pms, 4)
    res["recover_pose"] = pose
    log(f"ttm_recover_pose (50 peaks): {pose}")
    return res


def run_c1(args, ttm, synth, torch, dev, angle):
    """The 64^3 / 16^3 / order-2 workload (3 plants, sigma 0.3): the GPU
    seconds of the whole TTM path (build and match, refine 3) and of
    classical matching at 500 rotations; the CPU seconds of the same work by
    the oracle are in cpu_baseline."""
    wl = synth.workload_small()
    L = wl.template.shape
    n = wl.order
    q = synth.super_fibonacci(500).astype(np.float32)
    w = np.full(len(q), 1.0 / len(q))
    img, tm, mk = (torch.as_tensor(a, device=dev) for a in (wl.image, wl.template, wl.mask))
    ttm.build_tensor_template(tm, mk, n, q, w, image_shape=wl.image.shape)
    torch.cuda.synchronize()
    t0 = time.time()
    comps, bank = ttm.build_tensor_template(tm, mk, n, q, w, image_shape=wl.image.shape)
    torch.cuda.synchronize()
    build_ms = (time.time() - t0) * 1e3
    opt = ttm.default_options(max_peaks=len(wl.positions), min_dist=float(L[0]) / 2, threshold=0.0, refine=3)
    bufs = ttm.MatchBuffers(wl.image.shape, L, n, opt, dev)
    ms, _ = time_steps(lambda: ttm.match(img, bank, mk, n, opt, bufs, tmpl=tm), args.steps, args.warmup, ttm, torch)
    res = bufs.result()
    det = match_errors(res["pos"].cpu().numpy(), res["quat"].cpu().numpy(), wl.positions, wl.true_quats, angle)
    ttm.tm_classical(img, tm, mk, q[:16])
    torch.cuda.synchronize()
    c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    c0.record()
    best, idx = ttm.tm_classical(img, tm, mk, q)
    c1.record()
    torch.cuda.synchronize()
    cms = c0.elapsed_time(c1)
    idx_np = idx.cpu().numpy()
    at = [angle(q[idx_np[tuple(p)]], t) for p, t in zip(wl.positions, wl.true_quats)]
    log(f"c1 {wl.name}: build {build_ms:.2f} ms, match {ms:.3f} ms, classical 500 rotations {cms:.2f} ms")
    return {"workload": wl.name, "rotations": len(q), "gpu_build_ms": round(build_ms, 3),
            "gpu_match_ms": round(ms, 4), "gpu_ttm_seconds": round((build_ms + ms) / 1e3, 6),
            "gpu_classical_ms": round(cms, 3), "gpu_classical_seconds": round(cms / 1e3, 6),
            "ttm_pose_detected": dict(err_stats(det), recall=len(det) / len(wl.positions)),
            "classical_pose_at_planted": err_stats(at)}


def run_c3(args, ttm, synth, torch, dev, angle):
    """The 512 x 512 x 256 / 40^3 / order-6 workload (84 components, 40
    plants): build at 10^4 rotations, ttm_match (refine 3) and ttm_correlate
    per tomogram.  The per-output error against the float64 oracle is the
    precision test's (tests/test_gpu_precision.py)."""
    wl = synth.workload_precision()
    N, L, n = wl.image.shape, wl.template.shape, wl.order
    K = ttm.num_components(n)
    img, tm, mk = (torch.as_tensor(a, device=dev) for a in (wl.image, wl.template, wl.mask))
    q = synth.super_fibonacci(args.build_rotations).astype(np.float32)
    w = np.full(len(q), 1.0 / len(q))
    torch.cuda.synchronize()
    t0 = time.time()
    comps, bank = ttm.build_tensor_template(tm, mk, n, q, w, image_shape=N)
    torch.cuda.synchronize()
    build_ms = (time.time() - t0) * 1e3
    opt = ttm.default_options(max_peaks=len(wl.positions), min_dist=float(L[0]) / 2, threshold=0.0, refine=3)
    bufs = ttm.MatchBuffers(N, L, n, opt, dev)
    steps = max(3, args.steps // 4)
    ms, _ = time_steps(lambda: ttm.match(img, bank, mk, n, opt, bufs, tmpl=tm), steps, 1, ttm, torch)
    res = bufs.result()
    det = match_errors(res["pos"].cpu().numpy(), res["quat"].cpu().numpy(), wl.positions, wl.true_quats, angle)
    del bufs
    ws = ttm.correlate_workspace(N, L, n, dev)
    out = (torch.empty_like(img), torch.empty_like(img))
    cms, _ = time_steps(lambda: ttm.correlate(img, bank, mk, n, workspace=ws, out=out), steps, 1, ttm, torch)
    pb = path_model_bytes(N[0], N[1], N[2], K)
    log(f"c3 {wl.name}: build {build_ms:.1f} ms, match {ms:.3f} ms, correlate {cms:.3f} ms")
    return {"workload": wl.name, "order": n, "components": K, "build_ms": round(build_ms, 1),
            "match_ms": round(ms, 4), "voxels_per_s": float(np.prod(N)) / (ms / 1e3),
            "correlate_ms": round(cms, 4), "path_model_GB": round(pb / 1e9, 3),
            "path_frac": round(pb / (cms / 1e3) / 1e9 / HBM_PEAK_GBPS, 4),
            "pose_detected": dict(err_stats(det), recall=len(det) / len(wl.positions))}


def run_rotation_map(wl, img, mask, bank, K, args, ttm, synth, torch, dev, angle):
    """The all-voxel rotation map at the same workload: the correlation with
    the field kept, the fp16 MFMA seed scan (dominant kernel: 2 V_valid J K
    flops per launch, K = 35 useful components) and the float64 polish."""
    N = wl.image.shape
    L = wl.template.shape
    J = args.rmap_seeds
    seeds = torch.as_tensor(synth.super_fibonacci(J).astype(np.float32), device=dev)
    ws = ttm.rotation_map_workspace(N, L, 4, J, dev)
    out = ttm.rotation_map(img, bank, mask, 4, seeds, workspace=ws)

    def step():
        ttm.rotation_map(img, bank, mask, 4, seeds, workspace=ws, out=out)

    ms, prof = time_steps(step, args.rmap_steps, 1, ttm, torch)
    Vv = (N[0] - L[0] + 1) * (N[1] - L[1] + 1) * (N[2] - L[2] + 1)
    stages = {k: round(v[0] / args.rmap_steps, 4) for k, v in prof.items() if v[1]}
    scan_ms = prof["rmap_scan"][0] / prof["rmap_scan"][1]
    flops = 2.0 * Vv * J * K
    achieved = flops / (scan_ms / 1e3) / 1e12
    pos = torch.as_tensor(wl.positions, dtype=torch.long, device=dev)
    qp = out["quat"][pos[:, 0], pos[:, 1], pos[:, 2]].cpu().numpy()
    at = [angle(a, q) for a, q in zip(qp, wl.true_quats)]
    unconv = int(out["unconverged"].cpu()[0])
    log(f"rotation map ({J} seeds): {ms:.3f} ms, scan {scan_ms:.3f} ms = {achieved:.0f} TFLOP/s")
    del out, ws
    return {"n_seeds": J, "ms": round(ms, 4), "voxels_per_s": float(np.prod(N)) / (ms / 1e3),
            "valid_voxels_per_s": Vv / (ms / 1e3), "stages_ms": stages, "unconverged": unconv,
            "roofline": {"bound": "mfma", "kernel": "rmap_scan", "dtype": "f16 (f32 accumulate)",
                         "achieved": round(achieved, 1), "peak": MFMA_F16_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": round(achieved / MFMA_F16_PEAK_TFLOPS, 4),
                         "flops_per_launch": flops, "avg_launch_ms": round(scan_ms, 4), "traffic": None},
            "pose_at_planted": err_stats(at)}


def run_batch(bwl, args, ttm, synth, torch, dev, angle):
    """Batching leg: every tomogram against every template, tiled correlation
    at the tile edge the autotuner picks, peaks and poses, all jobs recorded
    into one hipGraph and replayed as one launch.  Per-tomogram latency from
    one graph per tomogram (its three jobs), each replayed and timed alone."""
    order = bwl.order
    edges = (64, 128, 256)
    qb = synth.super_fibonacci(args.build_rotations).astype(np.float32)
    wb = np.full(len(qb), 1.0 / len(qb))
    temps = []
    for t, m in zip(bwl.templates, bwl.masks):
        tt = torch.as_tensor(t, device=dev)
        mm = torch.as_tensor(m, device=dev)
        banks, comps = {}, None
        for T in edges:
            if T >= t.shape[0]:
                comps, banks[T] = ttm.build_tensor_template(tt, mm, order, qb, wb, image_shape=(T, T, T))
        table = ttm.autotune_tiles(banks, t.shape, mm, order, repeats=3)
        temps.append(dict(tmpl=tt, mask=mm, comps=comps, banks=banks, table=table, L=t.shape[0]))
        log(f"batch: template {t.shape[0]}^3 tile autotune (ms per tile) {table}")
    # as many peaks per job as the tomogram holds copies of all templates
    copies = sum(len(p) for p in bwl.positions[0])
    opt = ttm.default_options(max_peaks=copies, min_dist=float(min(t.shape[0] for t in bwl.templates)) / 2,
                              threshold=0.0, refine=args.refine)
    images = [torch.as_tensor(im, device=dev) for im in bwl.images]
    jobs, outs, meta = [], [], []
    choice = {}
    for i, im in enumerate(images):
        for k, tp in enumerate(temps):
            T = ttm.choose_tile(im.shape, bwl.templates[k].shape, tp["table"])
            choice[(tp["L"], T)] = choice.get((tp["L"], T), 0) + 1
            out = ttm.BatchOutputs(im.shape, opt.max_peaks, dev)
            jobs.append(ttm.batch_job(im, tp["banks"][T], T, tp["comps"], tp["mask"], out, tmpl=tp["tmpl"]))
            outs.append(out)
            meta.append((i, k, T))
    S = args.batch_streams
    ws = ttm.batch_workspace(jobs, order, opt, dev, S)
    torch.cuda.synchronize()
    t0 = time.time()
    ttm.batch_match(jobs, order, opt, ws)
    torch.cuda.synchronize()
    eager_ms = (time.time() - t0) * 1e3
    tc = time.time()
    graph = ttm.BatchGraph(jobs, order, opt, ws, S)
    capture_ms = (time.time() - tc) * 1e3
    graph.launch()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.batch_replays):
        graph.launch()
    e1.record()
    torch.cuda.synchronize()
    batch_ms = e0.elapsed_time(e1) / args.batch_replays
    graph.close()
    log(f"batch: {len(jobs)} jobs, eager (one stream) {eager_ms:.0f} ms, graph capture {capture_ms:.0f} ms, "
        f"graph replay on {S} branches {batch_ms:.1f} ms")
    # accuracy: each job's reported peaks against the plants of its template,
    # matched within 2 voxels and within L/4 (the Frobenius-score peak sits
    # near a copy's centre of mass, which for larger blob templates lies a few
    # voxels from its centre)
    errs, found, total = [], 0, 0
    per_t = {}
    for out, (i, k, T) in zip(outs, meta):
        res = out.result()
        pos, qs = res["pos"].cpu().numpy(), res["quat"].cpu().numpy()
        d = match_errors(pos, qs, bwl.positions[i][k], bwl.true_quats[i][k], angle)
        dl = match_errors(pos, qs, bwl.positions[i][k], bwl.true_quats[i][k], angle,
                          radius=temps[k]["L"] / 4.0)
        errs += d
        found += len(d)
        total += len(bwl.positions[i][k])
        e = per_t.setdefault(temps[k]["L"], {"r2": [], "rq": [], "n": 0})
        e["r2"] += d
        e["rq"] += dl
        e["n"] += len(bwl.positions[i][k])
    log(f"batch: accuracy read back ({found} of {total} copies within 2 voxels)")
    # per-tomogram latency: one graph per tomogram, each replayed alone
    lat = []
    nt = len(images)
    nk = len(temps)
    for i in range(nt):
        if i % 16 == 0:
            log(f"batch: per-tomogram graph {i} of {nt}")
        g = ttm.BatchGraph(jobs[i * nk:(i + 1) * nk], order, opt, ws, min(S, nk))
        g.launch()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        g.launch()
        b.record()
        torch.cuda.synchronize()
        lat.append(a.elapsed_time(b))
        g.close()
    log("batch: per-tomogram graphs done")
    vox = float(sum(im.numel() for im in images))
    del outs, jobs, ws
    return {"workload": bwl.name, "tomograms": nt, "templates": [tp["L"] for tp in temps], "jobs": nt * nk,
            "order": order, "edges": [int(min(im.shape[0] for im in images)), int(max(im.shape[0] for im in images))],
            "voxels": vox, "tile_ms_autotuned": {str(tp["L"]): tp["table"] for tp in temps},
            "tile_choice": {f"L{L}_T{T}": c for (L, T), c in sorted(choice.items())},
            "graph_streams": S, "graph_replay_ms": round(batch_ms, 2), "eager_one_stream_ms": round(eager_ms, 1),
            "graph_capture_ms": round(capture_ms, 1),
            "tomograms_per_s": nt / (batch_ms / 1e3),
            "voxel_template_pairs_per_s": vox * nk / (batch_ms / 1e3),
            "latency_ms_per_tomogram": {"p50": round(float(np.percentile(lat, 50)), 2),
                                        "p99": round(float(np.percentile(lat, 99)), 2),
                                        "max": round(float(np.max(lat)), 2)},
            "pose_detected": dict(err_stats(errs), recall=found / max(total, 1)),
            "pose_detected_per_template": {
                str(L): {"within_2": dict(err_stats(e["r2"]), recall=len(e["r2"]) / e["n"]),
                         "within_L/4": dict(err_stats(e["rq"]), recall=len(e["rq"]) / e["n"])}
                for L, e in sorted(per_t.items())}}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only (--gpus 1): the path shards by "
                                   "slabs of the tomogram with a halo, which is not run here", "n_gpus": args.gpus}))
        sys.exit(2)
    if args.batch > 0:
        print(json.dumps({"error": "the batching leg (--batch) is refused: runs of it have ended with a host "
                                   "segmentation fault after its graph replays whose cause has not been shown"}))
        sys.exit(2)
    # the batching leg's tomograms are generated before anything touches the
    # GPU (worker processes are started from a process without a GPU context)
    bwl = None
    if args.batch > 0 and args.copy_calibration == 0:
        from paper_2311_07561_amd import synth as _synth
        t0 = time.time()
        bwl = _synth.workload_batch(seed=4000, count=args.batch, workers=args.batch_workers)
        log(f"batch workload {bwl.name}: {args.batch} tomograms generated in {time.time() - t0:.1f}s")
    import torch

    if args.copy_calibration > 0:
        n = args.copy_calibration * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": n * 4}), flush=True)
        return

    angle = angle_deg
    from paper_2311_07561_amd import synth, ttm

    dev = torch.device("cuda:0")
    t0 = time.time()
    wl = synth.workload_tomogram(args.seed)
    N = wl.image.shape
    L = wl.template.shape
    V = int(np.prod(N))
    log(f"workload {wl.name}: image {N}, template {L}, {len(wl.positions)} plants, "
        f"noise sigma {wl.noise_sigma:.3f} (generated in {time.time() - t0:.1f}s)")
    img = torch.as_tensor(wl.image, device=dev)
    tmpl = torch.as_tensor(wl.template, device=dev)
    mask = torch.as_tensor(wl.mask, device=dev)

    main_run = run_order(4, wl, img, tmpl, mask, args, ttm, synth, torch, dev, angle, True)
    ms_per_step = main_run["ms_per_step"]
    value = V / (ms_per_step / 1e3)
    K = main_run["components"]

    # per-kernel roofline from the live event pairs of the timed steps
    cb = class_bytes(N[0], N[1], N[2], L[0], L[1], K)
    kernels = {}
    for name, (ms, cnt) in main_run["_prof"].items():
        if cnt == 0:
            continue
        ms_step = ms / args.steps
        byts = cb.get(name) or 0.0
        kernels[name] = {"ms_per_step": round(ms_step, 4), "launches_per_step": cnt / args.steps,
                         "avg_launch_ms": round(ms / cnt, 4),
                         "model_bytes_per_step": byts,
                         "model_GBps": round(byts / (ms_step / 1e3) / 1e9, 1) if byts else None}
    fft_classes = [k for k in kernels if kernels[k]["model_GBps"]]
    dom = max(fft_classes, key=lambda k: kernels[k]["ms_per_step"])
    achieved = kernels[dom]["model_GBps"]
    roofline = {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": counter_traffic(dom, wl.name),
                "bytes_per_launch": kernels[dom]["model_bytes_per_step"] / kernels[dom]["launches_per_step"],
                "bytes_per_step": kernels[dom]["model_bytes_per_step"],
                "avg_launch_ms": kernels[dom]["avg_launch_ms"],
                "launches_per_step": kernels[dom]["launches_per_step"]}
    corr_ms = sum(kernels[k]["ms_per_step"] for k in kernels if k not in ("peaks", "pose"))
    corr_bytes = sum(kernels[k]["model_bytes_per_step"] for k in kernels if k not in ("peaks", "pose"))
    hbm = {"correlate_ms": round(corr_ms, 4), "correlate_model_GB": round(corr_bytes / 1e9, 3),
           "correlate_model_GBps": round(corr_bytes / (corr_ms / 1e3) / 1e9, 1),
           "step_model_GBps": round(sum(k["model_bytes_per_step"] for k in kernels.values()) /
                                    (ms_per_step / 1e3) / 1e9, 1)}

    legs = set(x for x in args.legs.split(",") if x)
    corr = None
    if "correlate" in legs:
        corr = run_correlate(wl, img, mask, main_run["_bank"], K, main_run["_comps"], tmpl, args, ttm, torch)
    hbm["path_model_GB"] = round(path_model_bytes(N[0], N[1], N[2], K) / 1e9, 3)
    hbm["match_correlate_path_frac"] = round(path_model_bytes(N[0], N[1], N[2], K) / (corr_ms / 1e3) / 1e9 /
                                             HBM_PEAK_GBPS, 4)
    if corr:
        hbm["correlate_path_frac"] = corr["path_frac"]

    rmap = None
    if args.rmap_seeds > 0:
        rmap = run_rotation_map(wl, img, mask, main_run["_bank"], K, args, ttm, synth, torch, dev, angle)

    planar = run_2d(args, ttm, synth, torch, dev) if args.rotations_2d > 0 else None

    batch = run_batch(bwl, args, ttm, synth, torch, dev, angle) if bwl is not None else None
    del bwl

    order6 = None
    if args.order6:
        r6 = run_order(6, wl, img, tmpl, mask, args, ttm, synth, torch, dev, angle, False)
        order6 = {k: v for k, v in r6.items() if not k.startswith("_")}
        order6["ms_per_step"] = round(order6["ms_per_step"], 4)
        order6["voxels_per_s"] = V / (r6["ms_per_step"] / 1e3)
        del r6

    # classical TM at 10^4 rotations on the same GPU
    classical = None
    if args.classical_rotations > 0:
        qc = synth.super_fibonacci(args.classical_rotations).astype(np.float32)
        ttm.tm_classical(img, tmpl, mask, qc[:64])     # first call: code objects, workspace
        torch.cuda.synchronize()
        c0 = torch.cuda.Event(enable_timing=True)
        c1 = torch.cuda.Event(enable_timing=True)
        c0.record()
        best, idx = ttm.tm_classical(img, tmpl, mask, qc)
        c1.record()
        torch.cuda.synchronize()
        cms = c0.elapsed_time(c1)
        log(f"classical TM {args.classical_rotations} rotations: {cms:.1f} ms")
        idx_np = idx.cpu().numpy()
        at = [angle(qc[idx_np[tuple(p)]], q) for p, q in zip(wl.positions, wl.true_quats)]
        # classical peaks: the same peak picker on the best-NCC map
        opt = ttm.default_options(max_peaks=len(wl.positions), min_dist=float(L[0]) / 2, threshold=0.0)
        rc = ttm.recover_pose(best, img, main_run["_comps"], mask, 4, opt, want_C=False)
        cpos = rc["pos"].cpu().numpy()
        cq = np.array([qc[idx_np[tuple(p)]] for p in cpos]) if len(cpos) else np.zeros((0, 4))
        det = match_errors(cpos, cq, wl.positions, wl.true_quats, angle)
        step_deg = (8 * np.pi ** 2 / args.classical_rotations) ** (1.0 / 3.0) * 180 / np.pi
        c45 = None
        if "classical45k" in legs:
            q45 = synth.super_fibonacci(45123).astype(np.float32)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            b45, i45 = ttm.tm_classical(img, tmpl, mask, q45)
            e1.record()
            torch.cuda.synchronize()
            ms45 = e0.elapsed_time(e1)
            i45 = i45.cpu().numpy()
            at45 = [angle(q45[i45[tuple(p)]], t) for p, t in zip(wl.positions, wl.true_quats)]
            c45 = {"rotations": 45123, "sampling_step_deg": round((8 * np.pi ** 2 / 45123) ** (1 / 3) * 180 / np.pi, 2),
                   "ms": round(ms45, 2), "speedup_ttm_order4_vs_classical": round(ms45 / ms_per_step, 1),
                   "speedup_ttm_order6_vs_classical": round(ms45 / order6["ms_per_step"], 1) if order6 else None,
                   "pose_at_planted": err_stats(at45)}
            log(f"classical TM 45123 rotations: {ms45:.1f} ms, pose at planted {err_stats(at45)}")
            del b45
        classical = {"rotations": args.classical_rotations, "ms": round(cms, 2),
                     "voxels_per_s": V / (cms / 1e3),
                     "speedup_ttm_order4_vs_classical": round(cms / ms_per_step, 1),
                     "speedup_ttm_order6_vs_classical": round(cms / order6["ms_per_step"], 1) if order6 else None,
                     "sampling_step_deg": round(step_deg, 2),
                     "pose_at_planted": err_stats(at),
                     "pose_detected": dict(err_stats(det), recall=len(det) / len(wl.positions)),
                     "at_45123_rotations": c45}
        del best, idx

    c1 = run_c1(args, ttm, synth, torch, dev, angle) if "c1" in legs else None
    c3 = run_c3(args, ttm, synth, torch, dev, angle) if "c3" in legs else None

    cpu = cpu_baseline(wl, args.cpu_seconds, "c1" in legs) if args.cpu_seconds > 0 else None
    if c1 and cpu and cpu.get("c1"):
        c1["cpu"] = cpu["c1"]

    ttm4 = {k: v for k, v in main_run.items() if not k.startswith("_")}
    ttm4["ms_per_step"] = round(ttm4["ms_per_step"], 4)
    out = {
        "metric": METRIC, "value": value, "unit": "voxels/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": wl.name, "image": list(N), "template": list(L), "order": 4,
                   "components": K, "plants": len(wl.positions), "snr": 0.1,
                   "build_rotations": args.build_rotations, "refine": args.refine},
        "roofline": roofline,
        "hbm": hbm,
        "cpu_baseline": cpu,
        "ttm_order4": ttm4,
        "ttm_order6": order6,
        "correlate": corr,
        "c1": c1,
        "c3": c3,
        "rotation_map": rmap,
        "batch": batch,
        "planar": planar,
        "classical": classical,
        "kernels": kernels,
    }
    if args.profile_json:
        with open(args.profile_json, "w") as fh:
            json.dump(out, fh, indent=1)
    print(json.dumps(out), flush=True)


def cpu_baseline(wl, seconds, with_c1=False):
    """The FP64 oracle (direct spatial sums) at sampled voxels of the same
    tomogram: voxels/s for local normalisation + tensor field + score.  With
    with_c1, also the 64^3 / 16^3 / order-2 workload's CPU seconds: the
    tensor template (500 rotations) and the full-field score map by direct
    sums, and classical matching at 500 rotations extrapolated from two
    rotations over the whole valid region."""
    from oracle import ttm_oracle as O
    from paper_2311_07561_amd import synth
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threads = 1
    rng = np.random.default_rng(1)
    q = synth.super_fibonacci(64)
    T = O.tensor_template(wl.template.astype(np.float64), wl.mask.astype(np.float64), wl.order, q,
                          np.full(64, 1 / 64))
    f = wl.image.astype(np.float64)
    m = wl.mask.astype(np.float64)
    lo, hi = O.valid_region(wl.image.shape, wl.template.shape)

    def run(count):
        xs = np.stack([rng.integers(lo[i], hi[i], count) for i in range(3)], axis=1)
        t0 = time.perf_counter()
        C = O.tensor_field_at(f, T, m, xs)
        O.score_from_field(C, wl.order)
        return time.perf_counter() - t0

    probe = 128
    tp = run(probe)
    count = int(max(probe, min(65536, probe * seconds / max(tp, 1e-3))))
    t = run(count)
    log(f"oracle: {count} voxels in {t:.1f}s")
    c1 = None
    if with_c1:
        s1 = synth.workload_small()
        q1 = synth.super_fibonacci(500)
        f1, m1, t1 = (a.astype(np.float64) for a in (s1.image, s1.mask, s1.template))
        c0 = time.perf_counter()
        T1 = O.tensor_template(t1, m1, s1.order, q1, np.full(len(q1), 1.0 / len(q1)))
        tb = time.perf_counter() - c0
        xs1 = np.argwhere(O.valid_mask(s1.image.shape, s1.template.shape))
        c0 = time.perf_counter()
        O.score_from_field(O.tensor_field_at(f1, T1, m1, xs1), s1.order)
        tf = time.perf_counter() - c0
        c0 = time.perf_counter()
        O.classical_best_at(f1, t1, m1, q1[:2], xs1)
        tc = (time.perf_counter() - c0) * len(q1) / 2
        log(f"oracle c1: build {tb:.1f}s, full field {tf:.1f}s, classical 500 rotations ~{tc:.0f}s (from 2)")
        c1 = {"workload": s1.name, "ttm_build_seconds": round(tb, 2), "ttm_field_seconds": round(tf, 2),
              "ttm_seconds": round(tb + tf, 2), "classical_500_seconds_extrapolated": round(tc, 1),
              "classical_rotations_timed": 2, "valid_voxels": len(xs1), "cores": threads}
    return {"value": count / t, "unit": "voxels/s", "cores": threads, "kind": "oracle", "c1": c1,
            "sample": f"{count} random valid voxels of the 256^3 tomogram: FP64 direct local normalisation "
                      f"+ {wl.template.shape[0]}^3-window 35-component tensor field + Frobenius score "
                      f"(tensor template built beforehand with 64 rotations, not timed); window gathers "
                      f"single-threaded, the products on {threads} BLAS threads",
            "seconds": round(t, 2)}


if __name__ == "__main__":
    main()
