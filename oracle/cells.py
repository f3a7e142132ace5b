"""Self-cell integrals of the paper's discretizations (test infrastructure).

Piecewise-constant collocation on the uniform h x h grid (Sec. 5) puts on the
diagonal the integral of the kernel over the cell around the collocation point
(eqs. e:a1i, e:b2):

    c(h) = integral over [-h/2, h/2]^2 of K(|x|) dx.

The square splits into 8 congruent triangles 0 <= theta <= pi/4,
0 <= r <= a / cos(theta) (a = h/2), so c = 8 int_0^{pi/4} F(a / cos theta) dtheta
with F(rho) = int_0^rho K(r) r dr.

* Laplace, K = -log(r) / (2 pi) (eq. e:kernel_laplace):
  F(rho) = -(rho^2 log(rho) / 2 - rho^2 / 4) / (2 pi), and the theta integral
  in closed form (int sec^2 = 1, int sec^2 log sec = log(2)/2 - 1 + pi/4):
      c_L = -(a^2 / pi) (2 log a + log 2 - 3 + pi / 2).
* Helmholtz, K = (i/4) H0^(1)(kappa r) (eq. e:kernel_helmholtz): from
  d/dz [z H1(z)] = z H0(z) and z H1(z) -> -2i/pi as z -> 0,
      F(rho) = (i/4) [rho H1(kappa rho) / kappa + 2i / (pi kappa^2)],
  and the theta integral by adaptive quadrature (smooth integrand).

A direct two-dimensional quadrature of K over the triangle (cell_integral_2d)
pins both (tests/test_oracle_cells.py).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.integrate
import scipy.special


def laplace_cell(h: float) -> complex:
    a = 0.5 * h
    return complex(-(a * a / math.pi) * (2.0 * math.log(a) + math.log(2.0) - 3.0 + 0.5 * math.pi))


def helmholtz_cell(h: float, kappa: float) -> complex:
    a = 0.5 * h

    def F(theta, part):
        rho = a / math.cos(theta)
        v = 0.25j * (rho * scipy.special.hankel1(1, kappa * rho) / kappa + 2j / (math.pi * kappa * kappa))
        return v.real if part == 0 else v.imag

    opts = dict(epsabs=0.0, epsrel=1e-13, limit=200)
    re = scipy.integrate.quad(F, 0.0, 0.25 * math.pi, args=(0,), **opts)[0]
    im = scipy.integrate.quad(F, 0.0, 0.25 * math.pi, args=(1,), **opts)[0]
    return complex(8.0 * re, 8.0 * im)


def cell_integral(kern) -> complex:
    """c(h) of the kernel description (needs ``h``); 0 for kernels without one."""
    h = float(getattr(kern, "h", 0.0))
    if h <= 0.0:
        return 0j
    if kern.kind == "laplace":
        return laplace_cell(h)
    if kern.kind == "helmholtz":
        return helmholtz_cell(h, float(kern.kappa))
    raise ValueError(f"no cell integral for kernel {kern.kind!r}")


def cell_integral_2d(kern, h: float) -> complex:
    """The same integral by nested adaptive quadrature of K(r) r over the 8
    triangles (no antiderivative): the independent check."""
    a = 0.5 * h

    def K(r):
        if kern.kind == "laplace":
            return complex(-math.log(r) / (2.0 * math.pi))
        return complex(0.25j * scipy.special.hankel1(0, kern.kappa * r))

    out = 0j
    for part in (0, 1):
        def f(r, theta):
            v = K(r) * r if r > 0 else 0j
            return v.real if part == 0 else v.imag
        val = scipy.integrate.dblquad(f, 0.0, 0.25 * math.pi, 0.0, lambda t: a / math.cos(t),
                                      epsabs=0.0, epsrel=1e-12)[0]
        out += val if part == 0 else 1j * val
    return 8.0 * out
