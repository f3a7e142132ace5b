"""Pins for the oracle's matrix entries (oracle/kernels.py).

The Helmholtz kernel is pinned to tabulated Bessel values and zeros
(tests/golden/bessel_values.txt, Abramowitz & Stegun Tables 9.1 and 9.5), to
the small-argument form of H0^(1), to the leading terms of its large-argument
(Hankel) expansion, and to the Wronskian J1 Y0 - J0 Y1 = 2/(pi x).  The
Laplace kernel is pinned to closed-form values of the logarithm.
"""
import math
import os

import numpy as np
import pytest

from conftest import GOLDEN
from oracle import kernels
from paper_2310_15458_amd import workloads as W

EULER_GAMMA = 0.5772156649015329


def _hk(kappa=1.0):
    return W.Kernel("helmholtz", kappa=kappa, weight=1.0, diag=1.0)


def _H0(x):
    """H0^(1)(x) from the oracle's kernel: K = (i/4) H0  =>  H0 = -4i K."""
    K = kernels.kernel_values(_hk(), np.array([[x, 0.0]]), np.zeros((1, 2)))[0, 0]
    return -4j * K


def _golden():
    rows = []
    with open(os.path.join(GOLDEN, "bessel_values.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            kind, x, j0, y0 = line.split()
            rows.append((kind, float(x), float(j0), float(y0)))
    return rows


@pytest.mark.parametrize("row", _golden())
def test_helmholtz_tabulated(row):
    kind, x, j0, y0 = row
    h = _H0(x)
    if not math.isnan(j0):
        assert abs(h.real - j0) <= 2e-15 + 1e-14 * abs(j0)
    if not math.isnan(y0):
        assert abs(h.imag - y0) <= 2e-15 + 1e-14 * abs(y0)


@pytest.mark.parametrize("x", [1e-8, 1e-6, 1e-4])
def test_helmholtz_small_argument(x):
    # H0^(1)(x) = 1 + (2i/pi)(ln(x/2) + gamma) + O(x^2 ln x)
    ref = 1.0 + 2j / math.pi * (math.log(x / 2) + EULER_GAMMA)
    assert abs(_H0(x) - ref) <= 10 * x * x * (1 + abs(math.log(x)))


@pytest.mark.parametrize("x", [200.0, 1000.0, 5000.0])
def test_helmholtz_large_argument(x):
    # H0^(1)(x) ~ sqrt(2/(pi x)) e^{i(x - pi/4)} (1 - i/(8x) - 9/(128 x^2) + 75i/(1024 x^3))
    s = 1 - 1j / (8 * x) - 9 / (128 * x * x) + 75j / (1024 * x ** 3)
    ref = math.sqrt(2 / (math.pi * x)) * np.exp(1j * (x - math.pi / 4)) * s
    # the first omitted term is a_4 / x^4 with a_4 = 1*9*25*49 / (4! 8^4) ~ 0.112
    # (plus the rounding of the phase x - pi/4, about ulp(x))
    assert abs(_H0(x) - ref) <= abs(ref) * (1e-13 + 4e-16 * x + 0.12 / x ** 4)


def test_helmholtz_wronskian():
    import scipy.special
    x = np.linspace(0.3, 60.0, 97)
    h0 = np.array([_H0(t) for t in x])
    h1 = scipy.special.hankel1(1, x)
    w = h1.real * h0.imag - h0.real * h1.imag   # J1 Y0 - J0 Y1
    assert np.max(np.abs(w - 2 / (math.pi * x)) * x) < 1e-13


def test_helmholtz_scaling_by_kappa():
    K = kernels.kernel_values(_hk(25.0), np.array([[0.1, 0.0]]), np.zeros((1, 2)))[0, 0]
    assert abs(-4j * K - _H0(2.5)) < 1e-15


def test_laplace_closed_form():
    k = W.Kernel("laplace", weight=1.0)
    X = np.array([[1.0, 0.0], [math.e, 0.0], [0.0, 0.5], [3.0, 4.0]])
    vals = kernels.kernel_values(k, X, np.zeros((1, 2)))[:, 0]
    ref = np.array([0.0, -1 / (2 * math.pi), math.log(2) / (2 * math.pi), -math.log(5) / (2 * math.pi)])
    assert np.allclose(vals, ref, rtol=0, atol=1e-16)


def test_entries_diag_rule_and_weight():
    n = 4
    P = W.grid_points(n)
    k = W.grid_kernel("laplace", n, diag=0.75)
    A = kernels.dense_matrix(k, P)
    assert np.all(np.diag(A) == 0.75)
    r = math.hypot(*(P[0] - P[5]))
    assert abs(A[0, 5] - (-math.log(r) / (2 * math.pi) / n ** 2)) < 1e-17
    assert np.allclose(A, A.T, rtol=0, atol=0)   # radial kernel: symmetric


@pytest.mark.parametrize("q", [1, 2, 3])
def test_degenerate_rank(q):
    P = np.random.default_rng(7).random((60, 2))
    k = W.Kernel("degenerate", weight=1.0, diag=0.0, q=q)
    K = kernels.kernel_values(k, P, P)
    s = np.linalg.svd(K, compute_uv=False)
    rank = (q + 1) * (q + 2) // 2
    assert s[rank - 1] > 1e-8 * s[0]
    assert s[rank] < 1e-12 * s[0]
