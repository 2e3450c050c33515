"""The library's per-pair device math (seg_math.hpp), built for the host, against the oracle.

Checks the GPU path's closed forms (arranged in d = a - x, e = b - x) and its
hand-written adjoint against the oracle's antiderivative forms and dual
numbers, and measures how float32 evaluation of the same forms behaves far
from and near a segment.  Runs without a GPU.
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import oracle as O
import oracle.dual as du

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "hostmath", "segmath_host.hip")
HDR = os.path.join(HERE, "..", "paper_2602_05492_amd", "csrc", "seg_math.hpp")
LIB = os.path.join(HERE, "hostmath", "libsegmath_host.so")


@pytest.fixture(scope="module")
def hm():
    stale = (not os.path.exists(LIB)) or os.path.getmtime(LIB) < max(os.path.getmtime(SRC), os.path.getmtime(HDR))
    if stale:
        cmd = ["/opt/rocm/bin/hipcc", "-O2", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950",
               "-x", "hip", SRC, "-o", LIB]
        subprocess.run(cmd, check=True, capture_output=True)
    L = ctypes.CDLL(LIB)
    for name in ("hm_moments_f64", "hm_moments_f32"):
        getattr(L, name).argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64,
                                     ctypes.c_double, ctypes.c_void_p]
    for name in ("hm_adjoint_f64", "hm_adjoint_f32"):
        getattr(L, name).argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64,
                                     ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    for name in ("hm_adjoint_matrix_f64", "hm_adjoint_matrix_f32"):
        getattr(L, name).argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64,
                                     ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p]
    L.hm_beta_f64.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]
    return L


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _case(seed, n=64, K=40):
    rng = np.random.default_rng(seed)
    a = rng.uniform(0.2, 0.8, (K, 2))
    b = a + rng.normal(scale=0.03, size=(K, 2))
    x = np.concatenate([rng.uniform(0.01, 0.99, (n - 16, 2)),
                        a[:16] + rng.normal(scale=1e-3, size=(16, 2))])
    seg = np.ascontiguousarray(np.concatenate([a, b], 1))
    return np.ascontiguousarray(x), seg, a, b


def _moments(hm, fn, x, seg, eps):
    out = np.zeros((len(x), len(seg), 4))
    getattr(hm, fn)(_p(x), len(x), _p(seg), len(seg), eps, _p(out))
    return out


@pytest.mark.parametrize("eps", [0.0, 1e-4, 1e-2])
def test_device_moments_match_oracle(hm, eps):
    x, seg, a, b = _case(1)
    got = _moments(hm, "hm_moments_f64", x, seg, eps)
    ref = np.stack(O.segment_moments(x, a[:, 0], a[:, 1], b[:, 0], b[:, 1], eps), -1)
    scale = np.abs(ref).max(axis=-1, keepdims=True) + 1e-3 * np.abs(ref).max()
    assert np.abs(got - ref).max() / 1.0 < 1e-11 * np.abs(ref).max() + 0 or (np.abs(got - ref) / scale).max() < 1e-10


@pytest.mark.parametrize("eps", [1e-4, 1e-2])
def test_device_adjoint_matches_oracle_duals(hm, eps):
    x, seg, a, b = _case(2)
    n, K = len(x), len(seg)
    w = np.random.default_rng(3).standard_normal((n, K, 4))
    grad = np.zeros((n, K, 4))
    mom = np.zeros((n, K, 4))
    hm.hm_adjoint_f64(_p(x), n, _p(seg), K, eps, _p(w), _p(grad), _p(mom))
    M = O.segment_moments(x, du.seed(a[:, 0], 4, 0), du.seed(a[:, 1], 4, 1), du.seed(b[:, 0], 4, 2),
                          du.seed(b[:, 1], 4, 3), eps)
    ref = sum(w[:, :, i, None] * M[i].d for i in range(4))
    assert np.allclose(mom, np.stack([m.v for m in M], -1), rtol=1e-9, atol=1e-14)
    scale = np.abs(ref).max()
    assert np.abs(grad - ref).max() < 1e-9 * scale


@pytest.mark.parametrize("eps", [1e-4, 1e-2])
def test_gradient_matrix_form_matches_oracle_duals(hm, eps):
    """The per-pair gradient matrix applied to the cotangents (the J-tile kernel's form, one matrix
    shared by the three colour channels) against the oracle's dual numbers; with nearly equal end
    densities (a smooth colour along the curve) the float32 matrix form stays as accurate as the
    float32 reverse pass."""
    x, seg, a, b = _case(2)
    n, K = len(x), len(seg)
    rng = np.random.default_rng(6)
    w = rng.standard_normal((n, K, 4))
    M = O.segment_moments(x, du.seed(a[:, 0], 4, 0), du.seed(a[:, 1], 4, 1), du.seed(b[:, 0], 4, 2),
                          du.seed(b[:, 1], 4, 3), eps)

    def ref_of(w):
        return sum(w[:, :, i, None] * M[i].d for i in range(4))

    grad = np.zeros((n, K, 4))
    hm.hm_adjoint_matrix_f64(_p(x), n, _p(seg), K, eps, _p(np.ascontiguousarray(w)), _p(grad))
    ref = ref_of(w)
    assert np.abs(grad - ref).max() < 1e-9 * np.abs(ref).max()
    # float32: nearly equal end densities, each pair against its own scale
    base = rng.standard_normal((n, K, 1, 2)) * np.ones((1, 1, 2, 1))
    ws = np.ascontiguousarray((base + 1e-2 * rng.standard_normal((n, K, 2, 2))).reshape(n, K, 4)[:, :, [0, 2, 1, 3]])
    ref = ref_of(ws)
    g32, gm32, mom = np.zeros((n, K, 4)), np.zeros((n, K, 4)), np.zeros((n, K, 4))
    hm.hm_adjoint_f32(_p(x), n, _p(seg), K, eps, _p(ws), _p(g32), _p(mom))
    hm.hm_adjoint_matrix_f32(_p(x), n, _p(seg), K, eps, _p(ws), _p(gm32))
    far = np.hypot(*(x[:, None, :] - 0.5 * (a + b)[None]).transpose(2, 0, 1)) > 0.1
    scale = np.abs(ref).max(-1)[far] + 1e-30
    e_rev = (np.abs(g32 - ref).max(-1)[far] / scale).max()
    e_mat = (np.abs(gm32 - ref).max(-1)[far] / scale).max()
    assert e_mat < max(4 * e_rev, 1e-5), (e_mat, e_rev)


def test_device_beta_matches_oracle(hm):
    bnd = O.boundary(16)
    x = np.ascontiguousarray(np.random.default_rng(4).uniform(0.001, 0.999, (50, 2)))
    el = np.ascontiguousarray(np.concatenate([bnd.ea, bnd.eb], 1))
    out = np.zeros((50, bnd.M))
    hm.hm_beta_f64(_p(x), 50, _p(el), bnd.M, _p(out))
    assert np.allclose(out, O.element_weights(x, bnd), rtol=0, atol=1e-15)


def test_float32_error_far_and_near(hm):
    """Float32 evaluation of the same forms: small far from a segment, large near it (why near pairs use FP64)."""
    x, seg, a, b = _case(5, n=256, K=64)
    eps = 0.0
    ref = _moments(hm, "hm_moments_f64", x, seg, eps)
    f32 = _moments(hm, "hm_moments_f32", x, seg, eps)
    L = np.hypot(*(b - a).T)
    da = np.hypot(*(x[:, None, :] - a[None]).transpose(2, 0, 1))
    db = np.hypot(*(x[:, None, :] - b[None]).transpose(2, 0, 1))
    near = (da < 2 * L[None]) & (db < 2 * L[None])
    err = np.abs(f32 - ref).max(-1)
    assert err[~near].max() < 2e-6
    assert near.any()
