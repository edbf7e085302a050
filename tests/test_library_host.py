"""Host-side checks of libba.so that need no GPU: exported symbols, the HBM layout
plan the kernels index by, the pose partition, and argument errors."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle
import synth
from paper_2110_04015_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    return _lib.load()


def test_exports_every_declared_symbol(L):
    hdr = open(os.path.join(ROOT, "include", "ba.h")).read()
    hdr = re.sub(r"/\*.*?\*/", "", hdr, flags=re.S)
    names = set(re.findall(r"\b(ba_[a-z0-9_]+)\s*\(", hdr))
    assert len(names) >= 20
    for n in sorted(names):
        assert hasattr(L, n), n
    assert {s[0] for s in _lib.SIGNATURES} == names


def _validate(L, p, Ns=(1, 4, 16, 64), max_slots=0, max_tiles=0):
    cam = np.ascontiguousarray(p.obs_cam, np.int32)
    lm = np.ascontiguousarray(p.obs_lm, np.int32)
    Ns = [N for N in Ns if N <= p.n_cams]
    Na = (C.c_int32 * max(len(Ns), 1))(*Ns)
    st = (C.c_int64 * (4 + 3 * len(Ns)))()
    r = L.ba_plan_validate(p.n_cams, p.n_lms, cam.shape[0], cam.ctypes.data_as(C.POINTER(C.c_int32)),
                           lm.ctypes.data_as(C.POINTER(C.c_int32)), max_slots, max_tiles, Na, len(Ns), st)
    return r, L.ba_plan_validate_error().decode(), list(st)


@pytest.mark.parametrize("name,make", [
    ("tiny-shuffled", lambda: synth.tiny(n_cams=5, n_lms=40, seed=2, c_hi=5, shuffle=True)),
    ("ring50", lambda: synth.config0(seed=1)),
    ("ring50-shuffled", lambda: synth.ring_problem(n_cams=50, n_lms=3000, seed=4, shuffle=True)),
    ("walk300", lambda: synth.walk_problem(n_cams=300, n_lms=30000, seed=2)),
    ("cap150", lambda: synth.cap_problem(n_cams=150, n_lms=8000, seed=3)),
    ("ring-batch-member", lambda: synth.ring_problem(n_cams=80, n_lms=16000, c_lo=2, c_hi=20, seed=5)),
])
def test_plan_invariants(L, name, make):
    p = make()
    r, err, st = _validate(L, p)
    assert r == 0, err
    n_tiles, n_chunks, n_part, max_used = st[:4]
    assert n_tiles * 64 >= p.n_obs and n_chunks >= 1 and 1 <= max_used <= 128
    # padding bound: a tile is closed only when the next landmark does not fit
    counts = np.bincount(p.obs_lm, minlength=p.n_lms)
    assert n_tiles <= p.n_obs / (64 - counts.max() + 1) + 1


@pytest.mark.parametrize("max_slots,max_tiles", [(64, 1), (64, 4), (200, 64), (440, 4096)])
def test_plan_invariants_chunk_shapes(L, max_slots, max_tiles):
    p = synth.cap_problem(n_cams=100, n_lms=5000, seed=7)
    r, err, st = _validate(L, p, Ns=(3, 33), max_slots=max_slots, max_tiles=max_tiles)
    assert r == 0, err
    assert st[3] <= max_slots


def test_plan_rejects_bad_observations(L):
    p = synth.tiny(n_cams=4, n_lms=20, seed=0)
    q = synth.tiny(n_cams=4, n_lms=20, seed=0)
    q.obs_cam[1], q.obs_lm[1] = q.obs_cam[0], q.obs_lm[0]
    assert _validate(L, q)[0] == _lib.BA_ERR_INVALID_ARG
    q = synth.tiny(n_cams=4, n_lms=20, seed=0)
    q.obs_lm[3] = 25
    assert _validate(L, q)[0] == _lib.BA_ERR_INVALID_ARG
    q = synth.tiny(n_cams=4, n_lms=20, seed=0)
    q.n_lms = 21                                    # landmark 20 has no observation
    assert _validate(L, q)[0] == _lib.BA_ERR_NOT_SPD
    q = synth.ring_problem(n_cams=70, n_lms=10, c_lo=65, c_hi=65, seed=0)
    assert _validate(L, q)[0] == _lib.BA_ERR_UNSUPPORTED
    assert _validate(L, p)[0] == 0


def test_partition_matches_oracle(L):
    pairs = [(1936, 121), (571, 47), (459, 22), (394, 131), (50, 7), (50, 50), (13, 1)]
    for n, N in pairs:
        g = np.empty(n, dtype=np.int32)
        assert L.ba_partition(n, N, g.ctypes.data_as(C.POINTER(C.c_int32))) == 0
        assert np.array_equal(g, oracle.partition(n, N))
    g = np.empty(5, dtype=np.int32)
    assert L.ba_partition(5, 6, g.ctypes.data_as(C.POINTER(C.c_int32))) == _lib.BA_ERR_INVALID_ARG
    assert L.ba_partition(5, 0, g.ctypes.data_as(C.POINTER(C.c_int32))) == _lib.BA_ERR_INVALID_ARG


def test_host_argument_errors(L):
    out = C.c_void_p()
    assert L.ba_build_system(None, None, None, C.byref(out)) == _lib.BA_ERR_INVALID_ARG
    d = _lib.ProblemDesc()
    d.n_cams, d.n_lms, d.n_obs, d.d_p = 4, 10, 20, 7          # d_p must be 6 or 9
    assert L.ba_build_system(C.byref(d), None, None, C.byref(out)) == _lib.BA_ERR_INVALID_ARG
    assert "d_p" in L.ba_last_error().decode()
    d.d_p = 9
    assert L.ba_build_system(C.byref(d), None, None, C.byref(out)) == _lib.BA_ERR_INVALID_ARG
    assert not out.value
    # chunk shapes are checked before any device memory is touched (the array pointers
    # below are never dereferenced)
    d.obs_cam = d.obs_lm = d.J_p = d.J_l = d.r = 4096
    d.lam = 1e-4
    b = _lib.BuildOpts()
    b.max_tiles_multi = -1
    assert L.ba_build_system(C.byref(d), C.byref(b), None, C.byref(out)) == _lib.BA_ERR_INVALID_ARG
    assert "max_tiles_multi" in L.ba_last_error().decode()
    b.max_tiles_multi, b.max_tiles = 0, 4097
    assert L.ba_build_system(C.byref(d), C.byref(b), None, C.byref(out)) == _lib.BA_ERR_INVALID_ARG
    assert "max_tiles" in L.ba_last_error().decode()
    assert not out.value
    assert L.ba_status_string(_lib.BA_ERR_NOT_SPD).decode().startswith("matrix block")
    o = _lib.SolveOpts()
    L.ba_default_solve_opts(C.byref(o))
    assert o.eps == 1e-6 and o.max_iter == 1000 and o.precision == 0
