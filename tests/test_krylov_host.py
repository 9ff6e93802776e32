"""The host-side helper of the s-step GMRES basis (Leja-ordered shifts),
compiled on its own with g++ and checked against a closed form and brute
force."""
import ctypes as C
import os
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def kh(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("kh") / "libkh.so")
    subprocess.run(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", os.path.join(HERE, "krylov_host_check.cpp"),
                    "-o", out], check=True)
    lib = C.CDLL(out)
    dp, i = C.POINTER(C.c_double), C.c_int
    lib.kh_leja_order.argtypes = [dp, i, i, dp]
    lib.kh_leja_points.argtypes = [C.c_double, C.c_double, i, dp]
    return lib


def ptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def test_leja_order_brute_force(kh):
    rng = np.random.default_rng(5)
    pts = rng.uniform(-0.3, 1.7, 25)
    out = np.zeros(10)
    assert kh.kh_leja_order(ptr(pts), 25, 10, ptr(out)) == 10
    # first: the largest modulus; then each maximises the product of distances
    assert out[0] == pts[np.argmax(np.abs(pts))]
    for t in range(1, 10):
        rest = [p for p in pts if p not in out[:t]]
        prod = [np.prod(np.abs(p - out[:t])) for p in rest]
        assert out[t] == rest[int(np.argmax(prod))]
    assert len(set(out)) == 10
    # more requested than given: every point once
    out2 = np.zeros(25)
    assert kh.kh_leja_order(ptr(pts[:4].copy()), 4, 25, ptr(out2)) == 4
    assert sorted(out2[:4]) == sorted(pts[:4])


def test_leja_points_of_an_interval(kh):
    out = np.zeros(10)
    kh.kh_leja_points(0.1, 1.2, 10, ptr(out))
    # the end of larger modulus, the other end, then the midpoint (the maximum
    # of (1.2 - x)(x - 0.1)); all within the interval and distinct
    assert out[0] == 1.2 and abs(out[1] - 0.1) < 1e-15 and abs(out[2] - 0.65) < 1e-12
    assert np.all((out >= 0.1 - 1e-15) & (out <= 1.2)) and len(set(out)) == 10
    kh.kh_leja_points(0.65, 0.65, 4, ptr(out))
    assert np.all(out[:4] == 0.65)
