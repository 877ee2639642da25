"""The library's host logic for batches and graphs, on the CPU, under
AddressSanitizer, UndefinedBehaviorSanitizer and LeakSanitizer.

The host source (csrc/ttm_api.hip, which holds no kernels) is compiled with
g++ against a stand-in for the HIP runtime (tests/host_stub): device memory
is a registry of address ranges, every launch checks that its buffers lie in
live ranges with the extents the kernels touch, handles are heap objects
freed on destruction, and stream capture follows the runtime's join and
isolation rules.  tests/host_stub/batch_driver.cpp replays the batching
benchmark's call sequence: 64 tomograms with edges drawn as the batch
workload draws them (96..320), templates of 24, 32 and 48 voxels, refine 3,
tile edges from ttm_choose_tile, eager runs on one and four streams, one
graph of all 192 jobs replayed three times, 64 per-tomogram graphs created,
replayed and destroyed, refused calls, and a negative control (an output
released before a replay) that the stand-in must report.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
STUB = os.path.join(ROOT, "tests", "host_stub")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not found")
    out = tmp_path_factory.mktemp("host_asan")
    exe = str(out / "batch_driver")
    cmd = [gxx, "-std=c++17", "-g", "-O1", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-fno-omit-frame-pointer", f"-I{STUB}", f"-I{os.path.join(ROOT, 'include')}",
           f"-I{os.path.join(ROOT, 'paper_2311_07561_amd', 'csrc')}",
           "-x", "c++", os.path.join(ROOT, "paper_2311_07561_amd", "csrc", "ttm_api.hip"),
           "-x", "none", os.path.join(STUB, "stub_runtime.cpp"), os.path.join(STUB, "batch_driver.cpp"),
           "-o", exe]
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-4000:]
    return exe, out


def _run(exe, jobs_file):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:exitcode=23",
               UBSAN_OPTIONS="print_stacktrace=1")
    return subprocess.run([exe, jobs_file], capture_output=True, text=True, env=env, timeout=300)


def test_batch_host_sequence_is_clean_under_sanitizers(driver):
    exe, out = driver
    # the tomogram edges of the 64-tomogram batch workload (seed 4000: its
    # edges come from the sub-seed 4001, uniform on 96..320)
    edges = np.random.default_rng(4001).integers(96, 321, 64)
    jobs = out / "jobs.txt"
    jobs.write_text("\n".join(str(int(e)) for e in edges))
    res = _run(exe, str(jobs))
    print(res.stdout)
    assert res.returncode == 0, (res.stdout + res.stderr)[-6000:]
    assert "misuse before the control 0, control caught 1, call failures 0" in res.stdout
    assert "ERROR: AddressSanitizer" not in res.stderr and "runtime error" not in res.stderr


def test_batch_host_small_edges(driver):
    exe, out = driver
    # every tile edge and tomograms smaller than a tile, at the extremes
    jobs = out / "jobs_small.txt"
    jobs.write_text("\n".join(str(e) for e in (48, 63, 64, 65, 127, 129, 255, 257, 511)))
    res = _run(exe, str(jobs))
    assert res.returncode == 0, (res.stdout + res.stderr)[-6000:]
    assert "misuse before the control 0, control caught 1, call failures 0" in res.stdout
