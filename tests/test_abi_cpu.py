"""The C-ABI library loads on a machine without a GPU, exports every function
include/ttm.h declares, and validates arguments on the host (no compute call
reaches the GPU: invalid arguments return before anything is enqueued)."""
import ctypes
import os

import numpy as np

import pytest

from paper_2311_07561_amd import ttm

pytestmark = pytest.mark.skipif(not os.path.exists(ttm.LIB_PATH), reason="libttm.so not built")


def test_exports_every_declared_symbol():
    names = ttm.declared_functions()
    assert len(names) >= 13
    L = ctypes.CDLL(ttm.LIB_PATH)
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(ttm._SIGS)


def test_host_only_functions():
    L = ttm.lib()
    assert [L.ttm_num_components(n) for n in (2, 4, 6, 8)] == [10, 35, 84, 165]
    for bad in (0, 1, 3, 5, 10, -2):
        assert L.ttm_num_components(bad) == -1
    assert [L.ttm_supported_length(n) for n in (16, 32, 64, 128, 256, 512)] == [1] * 6
    assert [L.ttm_supported_length(n) for n in (8, 24, 96, 1024, 0)] == [0] * 5
    assert L.ttm_status_string(0) == b"TTM_OK"
    assert L.ttm_status_string(-3).startswith(b"TTM_E_WORKSPACE")
    o = ttm.default_options()
    assert o.max_peaks == 64 and o.n_seeds == 4096 and o.hopm_max_iter == 1000
    assert abs(o.eps_v - 1e-5) < 1e-12 and o.hopm_tol == 1e-12
    assert o.refine == 0 and o.check_finite == 0
    # ttm_options's layout: natural alignment of its C declaration
    assert ctypes.sizeof(ttm.Options) == 40
    assert (ttm.Options.hopm_tol.offset, ttm.Options.refine.offset, ttm.Options.check_finite.offset) == (24, 32, 36)
    assert L.ttm_status_string(-5).startswith(b"TTM_E_NONFINITE")


def test_sizes():
    L = ttm.lib()
    N, T = ttm.Dims(256, 256, 256), ttm.Dims(32, 32, 32)
    assert L.ttm_bank_bytes(N, T, 35) == 36 * 32 * 256 * 129 * 8
    half = 256 * 256 * 129 * 8
    ws = L.ttm_correlate_workspace_bytes(N, T, 35)
    # two image spectra, 37 arrays, and (the two-pass inverse) one float32 w field
    assert ws >= (2 + 37) * half + 4 * 256 ** 3 and ws < (2 + 37) * half + 4 * 256 ** 3 + (1 << 20)
    n64 = ttm.Dims(64, 64, 64)
    h64 = 64 * 64 * 33 * 8
    ws = L.ttm_correlate_workspace_bytes(n64, T, 35)
    assert ws >= (2 + 37) * h64 and ws < (2 + 37) * h64 + (1 << 20)
    assert L.ttm_correlate_workspace_bytes(ttm.Dims(0, 1, 1), T, 35) == 0
    assert L.ttm_build_workspace_bytes(T, 4, 100, N) >= 100 * (16 + 8 + 16 + 35 * 8)
    assert L.ttm_build_workspace_bytes(T, 3, 100, N) == 0
    assert L.tm_classical_workspace_bytes(N, T, 10000) > 0


def _opt(**kw):
    return ttm.default_options(**kw)


def test_argument_validation_without_gpu():
    L = ttm.lib()
    N, T = ttm.Dims(64, 64, 64), ttm.Dims(16, 16, 16)
    o = _opt()
    fake = ctypes.c_void_p(256)          # never dereferenced: validation fails first
    big = 1 << 40
    # NULL pointers
    assert L.ttm_correlate(None, N, fake, T, 2, fake, ctypes.byref(o), fake, None, fake, big, None) == -1
    # odd order
    assert L.ttm_correlate(fake, N, fake, T, 3, fake, ctypes.byref(o), fake, None, fake, big, None) == -1
    # unsupported image size, template larger than image
    assert L.ttm_correlate(fake, ttm.Dims(64, 64, 96), fake, T, 2, fake, ctypes.byref(o), fake, None, fake,
                           big, None) == -2
    assert L.ttm_correlate(fake, ttm.Dims(16, 16, 16), fake, ttm.Dims(17, 4, 4), 2, fake, ctypes.byref(o),
                           fake, None, fake, big, None) == -2
    # workspace too small
    assert L.ttm_correlate(fake, N, fake, T, 2, fake, ctypes.byref(o), fake, None, fake, 1024, None) == -3
    # build: weights must sum to one, quaternions nonzero
    q = (ctypes.c_float * 8)(1, 0, 0, 0, 0, 1, 0, 0)
    w = (ctypes.c_double * 2)(0.5, 0.4)
    assert L.ttm_build_tensor_template(fake, fake, T, 2, q, w, 2, fake, N, None, fake, big, None) == -1
    w2 = (ctypes.c_double * 2)(0.5, 0.5)
    q0 = (ctypes.c_float * 8)(1, 0, 0, 0, 0, 0, 0, 0)
    assert L.ttm_build_tensor_template(fake, fake, T, 2, q0, w2, 2, fake, N, None, fake, big, None) == -1
    assert L.ttm_build_tensor_template(fake, fake, T, 2, q, w2, 0, fake, N, None, fake, big, None) == -1
    assert L.ttm_build_tensor_template(fake, fake, T, 2, q, w2, 2, fake, N, None, None, 0, None) == -3
    # pose options
    bad = _opt(max_peaks=0)
    args = [fake] * 5 + [N, T, 4, ctypes.byref(bad)] + [fake] * 7 + [fake, big, None]
    assert L.ttm_recover_pose(*args) == -1
    bad = _opt(n_seeds=8)
    args[8] = ctypes.byref(bad)
    assert L.ttm_recover_pose(*args) == -1
    bad = _opt(threshold=-1.0)
    args[8] = ctypes.byref(bad)
    assert L.ttm_recover_pose(*args) == -1
    bad = _opt(refine=4)
    args[8] = ctypes.byref(bad)
    assert L.ttm_recover_pose(*args) == -1
    bad = _opt(refine=3)        # refine 3 needs the raw template like 2
    args[8] = ctypes.byref(bad)
    args[4] = None
    assert L.ttm_recover_pose(*args) == -1
    args[4] = fake
    # refine 2 needs the raw template
    bad = _opt(refine=2)
    args[8] = ctypes.byref(bad)
    args[4] = None
    assert L.ttm_recover_pose(*args) == -1
    # pose at given positions: more positions than max_peaks
    ok = _opt(max_peaks=2)
    assert L.ttm_pose_at(fake, fake, fake, None, N, T, 4, ctypes.byref(ok), fake, 3, fake, fake, fake, fake,
                         None, fake, big, None) == -1
    assert L.ttm_pose_at(fake, fake, fake, None, N, T, 4, ctypes.byref(ok), fake, 2, fake, fake, fake, fake,
                         None, fake, 16, None) == -3
    r2 = _opt(max_peaks=2, refine=2)
    assert L.ttm_pose_at(fake, fake, fake, None, N, T, 4, ctypes.byref(r2), fake, 2, fake, fake, fake, fake,
                         None, fake, big, None) == -1
    # match: refine 2 without the template
    assert L.ttm_match(fake, N, fake, T, 4, fake, None, ctypes.byref(r2), fake, None, fake, fake, fake, fake,
                       fake, None, fake, fake, big, None) == -1
    # classical
    assert L.tm_classical(fake, N, fake, fake, T, q, 0, ctypes.byref(o), fake, fake, fake, big, None) == -1
    assert L.tm_classical(fake, N, fake, fake, T, q0, 2, ctypes.byref(o), fake, fake, fake, big, None) == -1


def test_binding_refuses_cpu_tensors():
    import torch
    t = torch.zeros((16, 16, 16))
    with pytest.raises(ValueError):
        ttm.correlate(t, t, t, 2)


def test_lowpass_validation_without_gpu():
    L = ttm.lib()
    N = ttm.Dims(16, 16, 16)
    fake = ctypes.c_void_p(256)
    big = 1 << 40
    assert L.ttm_lowpass(None, N, 1.0, 1, fake, fake, big, None) == -1
    assert L.ttm_lowpass(fake, N, -0.5, 1, fake, fake, big, None) == -1
    assert L.ttm_lowpass(fake, N, 11.0, 1, fake, fake, big, None) == -1     # radius 33 > 32
    assert L.ttm_lowpass(fake, N, 1.0, 2, fake, fake, big, None) == -1
    assert L.ttm_lowpass(fake, ttm.Dims(0, 4, 4), 1.0, 1, fake, fake, big, None) == -2
    assert L.ttm_lowpass(fake, N, 1.0, 1, fake, fake, 16, None) == -3
    assert L.ttm_lowpass_workspace_bytes(N) >= 2 * 4 * 16 ** 3



def test_rotation_map_validation_without_gpu():
    L = ttm.lib()
    N, T = ttm.Dims(64, 64, 64), ttm.Dims(16, 16, 16)
    o = _opt()
    fake = ctypes.c_void_p(256)
    big = 1 << 40

    def call(n_seeds=64, order=4, opt=o, seeds=fake, ws=big, dims=N):
        return L.ttm_rotation_map(fake, dims, fake, T, order, fake, ctypes.byref(opt), seeds, n_seeds, fake,
                                  None, fake, fake, None, fake, ws, None)

    assert call(n_seeds=48) == -1            # not a multiple of 32
    assert call(n_seeds=0) == -1
    assert call(n_seeds=131072 + 32) == -1
    assert call(order=3) == -1
    assert call(seeds=None) == -1
    assert call(opt=_opt(hopm_max_iter=0)) == -1
    assert call(dims=ttm.Dims(64, 64, 96)) == -2
    assert call(ws=1024) == -3
    assert L.ttm_rotation_map_workspace_bytes(N, T, 4, 48) == 0
    # workspace: the correlation's, plus K float32 planes over the valid box
    # (49^3 voxels), the fp16 seed table and one group index per valid voxel
    V = 49 ** 3
    need = L.ttm_rotation_map_workspace_bytes(N, T, 4, 64)
    assert need >= L.ttm_correlate_workspace_bytes(N, T, 35) + 35 * 4 * V + 4 * V + 64 * 48 * 2


def test_tile_schedule_host_logic():
    """Tile counts from an independent enumeration of tile origins, and the
    choice that minimises tiles x ms (ties: the larger edge)."""
    import itertools

    def count(N, L, T):
        total = 1
        for n, l in zip(N, L):
            W, WT = n - l + 1, T - l + 1
            origins = list(range(0, W, WT))
            covered = sorted(o + i for o in origins for i in range(WT) if o + i < W)
            assert covered == list(range(W))          # the tiles partition the valid positions
            total *= len(origins)
        return total

    for N, L, T in itertools.product([(96, 96, 96), (40, 52, 37), (320, 201, 97), (24, 24, 24)],
                                     [(24, 24, 24), (12, 9, 16)], [32, 64, 128, 256]):
        if any(l > n for l, n in zip(L, N)) or T < max(L):
            assert ttm.lib().ttm_tile_count(ttm.Dims(*N), ttm.Dims(*L), T) < 0
            continue
        assert ttm.tile_count(N, L, T) == count(N, L, T)
    assert ttm.lib().ttm_tile_count(ttm.Dims(64, 64, 64), ttm.Dims(8, 8, 8), 48) < 0      # not a supported length
    table = {64: 0.05, 128: 0.35, 256: 2.6}
    for N, L in [((96,) * 3, (24,) * 3), ((320,) * 3, (48,) * 3), ((200, 120, 300), (32,) * 3)]:
        cost = {T: ttm.tile_count(N, L, T) * ms for T, ms in table.items() if T >= max(L)}
        best = min(cost.values())
        assert ttm.choose_tile(N, L, table) == max(T for T, c in cost.items() if c == best)
    assert ttm.choose_tile((100,) * 3, (10,) * 3, {64: 1.0, 128: 8.0}) == 128   # 8 tiles of 64 = 1 of 128: tie


def test_batch_and_tiled_validation_without_gpu():
    L = ttm.lib()
    fake = ctypes.c_void_p(256)
    big = 1 << 40
    o = _opt()
    N, T = ttm.Dims(100, 90, 80), ttm.Dims(16, 16, 16)
    assert L.ttm_correlate_tiled(None, N, fake, T, 4, 32, fake, ctypes.byref(o), fake, None, fake, big, None) == -1
    assert L.ttm_correlate_tiled(fake, N, fake, T, 4, 48, fake, ctypes.byref(o), fake, None, fake, big, None) == -2
    assert L.ttm_correlate_tiled(fake, N, fake, T, 4, 8, fake, ctypes.byref(o), fake, None, fake, big, None) == -2
    assert L.ttm_correlate_tiled(fake, ttm.Dims(10, 90, 80), fake, T, 4, 32, fake, ctypes.byref(o), fake, None,
                                 fake, big, None) == -2
    assert L.ttm_correlate_tiled(fake, N, fake, T, 4, 32, fake, ctypes.byref(o), fake, None, fake, 64, None) == -3
    # the tiled workspace does not depend on the image extent
    assert L.ttm_correlate_tiled_workspace_bytes(T, 4, 32) >= 3 * 4 * 32 ** 3
    # a batch job with a missing output, with refine 2 and no template
    job = ttm.BatchJob()
    for f in ("image", "bank", "components", "mask", "tmpl", "out_score", "out_pos", "out_quat", "out_lambda",
              "out_peak_score", "out_flags", "out_count"):
        setattr(job, f, 256)
    job.N, job.L, job.tile = N, T, 32
    arr = (ttm.BatchJob * 1)(job)
    one = L.ttm_batch_workspace_bytes(ctypes.cast(arr, ctypes.c_void_p), 1, 4, ctypes.byref(o), 1)
    assert one > 0
    assert L.ttm_batch_workspace_bytes(ctypes.cast(arr, ctypes.c_void_p), 1, 4, ctypes.byref(o), 3) == 3 * one - 512
    assert L.ttm_batch_workspace_bytes(ctypes.cast(arr, ctypes.c_void_p), 1, 4, ctypes.byref(o), 9) == 0
    bad = ttm.BatchJob.from_buffer_copy(job)
    bad.out_count = None
    arr2 = (ttm.BatchJob * 1)(bad)
    assert L.ttm_batch_match(ctypes.cast(arr2, ctypes.c_void_p), 1, 4, ctypes.byref(o), 1, fake, big, None) == -1
    r2 = _opt(refine=2)
    nt = ttm.BatchJob.from_buffer_copy(job)
    nt.tmpl = None
    arr3 = (ttm.BatchJob * 1)(nt)
    assert L.ttm_batch_match(ctypes.cast(arr3, ctypes.c_void_p), 1, 4, ctypes.byref(r2), 1, fake, big, None) == -1
    wrong = ttm.BatchJob.from_buffer_copy(job)
    wrong.tile = 8
    arr4 = (ttm.BatchJob * 1)(wrong)
    assert L.ttm_batch_match(ctypes.cast(arr4, ctypes.c_void_p), 1, 4, ctypes.byref(o), 1, fake, big, None) == -2
    assert L.ttm_batch_match(ctypes.cast(arr, ctypes.c_void_p), 1, 4, ctypes.byref(o), 1, fake, 64, None) == -3
    # capture needs a created stream and an output handle
    h = ctypes.c_void_p()
    assert L.ttm_batch_graph_create(ctypes.cast(arr, ctypes.c_void_p), 1, 4, ctypes.byref(o), 1, fake, big, None,
                                    ctypes.byref(h)) == -1
    assert L.ttm_batch_graph_create(ctypes.cast(arr, ctypes.c_void_p), 1, 4, ctypes.byref(o), 1, fake, big, fake,
                                    None) == -1
    assert L.ttm_batch_graph_create(ctypes.cast(arr, ctypes.c_void_p), 1, 4, ctypes.byref(o), 0, fake, big, fake,
                                    ctypes.byref(h)) == -1
    assert L.ttm_batch_graph_create(ctypes.cast(arr, ctypes.c_void_p), 1, 4, ctypes.byref(o), 2, fake, one, fake,
                                    ctypes.byref(h)) == -3
    assert L.ttm_graph_launch(None, None) == -1
    L.ttm_graph_destroy(None)
    # the finiteness check waits on the stream: a batch or graph rejects it
    cf = _opt(check_finite=1)
    assert L.ttm_batch_match(ctypes.cast(arr, ctypes.c_void_p), 1, 4, ctypes.byref(cf), 1, fake, big, None) == -1
    assert L.ttm_batch_graph_create(ctypes.cast(arr, ctypes.c_void_p), 1, 4, ctypes.byref(cf), 1, fake, big, fake,
                                    ctypes.byref(h)) == -1
    # ttm_batch_job's layout: natural alignment of its C declaration
    assert ctypes.sizeof(ttm.BatchJob) == 144
    assert (ttm.BatchJob.N.offset, ttm.BatchJob.tile.offset, ttm.BatchJob.L.offset,
            ttm.BatchJob.out_count.offset) == (8, 32, 64, 136)


def test_snorm_validation_without_gpu():
    """ttm_snorm rejects bad arguments before any device work; the workspace
    holds at least the per-window slabs of h~ (one L-box per position plus the
    template) and the rotation table."""
    L = ttm.lib()
    N, T = ttm.Dims(64, 64, 64), ttm.Dims(16, 16, 16)
    fake = ctypes.c_void_p(256)
    big = 1 << 40
    q = np.array([[1.0, 0.0, 0.0, 0.0], [0.0, 1.0, 0.0, 0.0]], dtype=np.float32)
    w = np.array([0.5, 0.5])
    qp, wp = q.ctypes.data, w.ctypes.data

    def call(order=4, n_rot=2, max_pos=8, ws=big, dims=N, box=T, wts=wp, pos=fake, quats=qp):
        return L.ttm_snorm(fake, dims, fake, fake, box, order, quats, wts, n_rot, pos, fake, None, max_pos,
                           fake, fake, fake, fake, ws, None)

    assert call(order=3) == -1
    assert call(order=0) == -1
    assert call(n_rot=0) == -1
    assert call(max_pos=0) == -1
    assert call(max_pos=(1 << 16) + 1) == -1
    assert call(pos=None) == -1
    assert call(quats=None) == -1
    bad_w = np.array([0.5, 0.4])
    assert call(wts=bad_w.ctypes.data) == -1          # weights must sum to 1
    zero_q = np.zeros((2, 4), dtype=np.float32)
    assert call(quats=zero_q.ctypes.data) == -1
    assert call(box=ttm.Dims(1024, 4, 4)) == -2
    assert call(dims=ttm.Dims(9000, 4, 4)) == -2
    assert call(ws=1024) == -3
    assert L.ttm_snorm_workspace_bytes(T, 0, 8) == 0
    assert L.ttm_snorm_workspace_bytes(T, 2, 0) == 0
    need = L.ttm_snorm_workspace_bytes(T, 10000, 64)
    assert need >= 65 * 16 ** 3 * 4 + 10000 * (12 * 4 + 8)


def test_planar_validation_without_gpu():
    """The two-dimensional entry points reject bad arguments before any
    device work; sizes follow the volume path's with a depth-1 box and n + 1
    components."""
    L = ttm.lib()
    fake = ctypes.c_void_p(256)
    big = 1 << 40
    z = np.array([[1.0, 0.0], [0.0, 1.0]], dtype=np.float32)
    w = np.array([0.5, 0.5])

    def build(order=4, L1=16, L2=16, zp=z.ctypes.data, wp=w.ctypes.data, n_rot=2, B=16, n1=64, n2=64, bank=fake,
              ws=big):
        return L.ttm_build_tensor_template_2d(fake, fake, L1, L2, order, zp, wp, n_rot, fake, B, n1, n2, bank,
                                              fake, ws, None)

    assert build(order=3) == -1
    assert build(order=10) == -1
    assert build(n_rot=0) == -1
    assert build(zp=np.zeros((2, 2), dtype=np.float32).ctypes.data) == -1
    assert build(wp=np.array([0.5, 0.6]).ctypes.data) == -1
    assert build(L2=513) == -2
    assert build(n1=96) == -2                     # not a supported length
    assert build(L1=80) == -2                     # larger than the image
    assert build(ws=16) == -3
    assert L.ttm_bank_bytes_2d(16, 64, 64, 16, 16, 4) == L.ttm_bank_bytes(ttm.Dims(16, 64, 64), ttm.Dims(1, 16, 16), 5)
    o = _opt(max_peaks=8, refine=2)

    def match(B=16, n1=64, n2=64, order=4, tmpl=fake, opt=o, ws=big):
        return L.ttm_match_2d(fake, B, n1, n2, fake, fake, tmpl, fake, 16, 16, order, ctypes.byref(opt), fake, None,
                              fake, fake, fake, fake, fake, fake, fake, ws, None)

    assert match(tmpl=None) == -1                 # refine 2 reads the template
    assert match(order=5) == -1
    assert match(opt=_opt(max_peaks=0)) == -1
    assert match(B=12) == -2
    assert match(ws=1024) == -3
    assert L.ttm_match_2d_workspace_bytes(16, 64, 64, 16, 16, 4, ctypes.byref(o)) > 0
