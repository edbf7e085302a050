"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

  - The oracle (oracle/ba_oracle.c) built with -fsanitize=address,undefined and driven
    through its whole surface (build for d_p = 9 and 6, S v, preconditioner, back-
    substitution, PCG, MCG with and without eq. (19), the pseudo-inverse, the dense S) in
    a child process that preloads the sanitizer runtimes.
  - The library's host layout planner (plan.cpp, plan_check.cpp) built with the same
    flags into a small driver (tests/sanitize_plan_main.cpp) that plans and validates the
    layouts of several problems, shuffled and ragged ones included, for several chunk
    shapes and partitions.

Any sanitizer report fails the test.
"""
import os
import shutil
import subprocess
import sys

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=undefined", "-g", "-O1"]
ENV = {"ASAN_OPTIONS": "detect_leaks=0:abort_on_error=0:halt_on_error=1",
       "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}


def _runtime(name):
    p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


@pytest.fixture(scope="module")
def tmp(tmp_path_factory):
    if not shutil.which("gcc") or not shutil.which("g++"):
        pytest.skip("gcc/g++ not available")
    return tmp_path_factory.mktemp("san")


ORACLE_DRIVER = r"""
import sys, numpy as np
sys.path.insert(0, {root!r})
import oracle, synth
L = oracle.load({lib!r})
for p in [synth.tiny(n_cams=5, n_lms=40, seed=2, c_hi=5), synth.ring_problem(n_cams=12, n_lms=300, seed=3),
          synth.extrinsics_only(synth.tiny(n_cams=6, n_lms=50, seed=4, c_hi=5)),
          synth.tiny(n_cams=7, n_lms=60, seed=5, c_hi=6, shuffle=True)]:
    o = oracle.System(p, libobj=L)
    v = np.random.default_rng(0).standard_normal(o.n)
    o.matvec(v); o.precond(v); o.back_substitute(v); o.rhs(); o.D_blocks(); o.dense_S()
    o.pcg(eps=1e-10, imax=200)
    for N, tau in [(1, 3.3), (3, 10.0), (p.n_cams, 1e9)]:
        o.mcg(N, tau, eps=1e-10, imax=100, trace=True, history=True)
        o.mcg(N, tau, eps=1e-10, imax=100, q_mode=1)
A = np.random.default_rng(1).standard_normal((6, 6)); A = A @ A.T
A[:, 0] = 0; A[0, :] = 0
oracle.pinv(A)
print("oracle ok")
"""


def test_oracle_under_asan_ubsan(tmp):
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if not asan or not ubsan:
        pytest.skip("sanitizer runtimes not found")
    lib = str(tmp / "liboracle_san.so")
    subprocess.check_call(["gcc", *SAN, "-fopenmp", "-fPIC", "-shared", "-o", lib,
                           os.path.join(ROOT, "oracle", "ba_oracle.c"), "-lm"])
    env = dict(os.environ, LD_PRELOAD=f"{asan}:{ubsan}", OMP_NUM_THREADS="2", **ENV)
    r = subprocess.run([sys.executable, "-c", ORACLE_DRIVER.format(root=ROOT, lib=lib)], env=env,
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0 and "oracle ok" in r.stdout, r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]


def _write(path, p):
    with open(path, "wb") as f:
        np.array([p.n_cams, p.n_lms], np.int32).tofile(f)
        np.array([p.n_obs], np.int64).tofile(f)
        np.ascontiguousarray(p.obs_cam, np.int32).tofile(f)
        np.ascontiguousarray(p.obs_lm, np.int32).tofile(f)


def test_planner_under_asan_ubsan(tmp):
    exe = str(tmp / "plan_san")
    csrc = os.path.join(ROOT, "paper_2110_04015_amd", "csrc")
    subprocess.check_call(["g++", "-std=c++17", *SAN, "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                           f"-I{os.path.join(ROOT, 'include')}", f"-I{csrc}", "-o", exe,
                           os.path.join(ROOT, "tests", "sanitize_plan_main.cpp"), os.path.join(csrc, "plan.cpp"),
                           os.path.join(csrc, "plan_check.cpp")])
    probs = {"tiny": synth.tiny(n_cams=5, n_lms=40, seed=2, c_hi=5, shuffle=True),
             "ring50": synth.config0(seed=1),
             "walk300": synth.walk_problem(n_cams=300, n_lms=30000, seed=2),
             "cap150": synth.cap_problem(n_cams=150, n_lms=8000, seed=3),
             "ragged": synth.ring_problem(n_cams=9, n_lms=77, c_lo=2, c_hi=4, seed=5, shuffle=True)}
    for name, p in probs.items():
        path = str(tmp / f"{name}.bin")
        _write(path, p)
        Ns = [str(N) for N in (1, 2, 4, 16, 64) if N <= p.n_cams]
        for slots, tiles in ((0, 0), (64, 1), (128, 16), (440, 4096)):
            r = subprocess.run([exe, path, str(slots), str(tiles), *Ns], env=dict(os.environ, **ENV),
                               capture_output=True, text=True, timeout=300)
            assert r.returncode == 0, (name, slots, tiles, r.stdout, r.stderr[-4000:])
            assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
