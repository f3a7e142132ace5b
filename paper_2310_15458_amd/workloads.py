"""Seeded synthetic inputs for the RS-S solver: point sets, kernel descriptions,
right-hand sides and the multi-problem / request-stream draws.

This module holds no arithmetic of the method itself (no kernel evaluation, no
factorization).  Both the GPU path and the CPU oracle take what it returns as
plain arrays, so the two sides see bit-identical inputs.

Workload shapes follow the paper's experiments (Sec. 5): a uniform grid of
cell centres on the unit square, h = 1/n, N = n^2 unknowns, random right-hand
sides.  The paper's own matrices integrate the diagonal and scale the
Helmholtz kernel by kappa^2 sqrt(b_i b_j) (eqs. e:a1, e:a1i, e:b1, e:b2); the
workloads here use the simpler diagonal A_ii = 1 with weight w = h^2.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

LAPLACE = "laplace"
HELMHOLTZ = "helmholtz"
DEGENERATE = "degenerate"


@dataclasses.dataclass(frozen=True)
class Kernel:
    """A kernel description: entries are ``weight * K(x_i, x_j)`` off the
    diagonal and ``diag`` on it.  ``kind`` selects K:

    * laplace    : K = -log(r) / (2 pi)                       (eq. e:kernel_laplace)
    * helmholtz  : K = (i/4) H0^(1)(kappa r)                  (eq. e:kernel_helmholtz)
    * degenerate : K = (1 + x.y)^q, an exactly low-rank test kernel
    """
    kind: str
    kappa: float = 0.0
    weight: float = 1.0
    diag: float = 1.0
    q: int = 2
    # the paper's discretizations (Sec. 5): the cell integral of K over an
    # h x h cell on the diagonal, scaled by (weight / h^2) s_i^2, and the
    # scattering potential b(x) = exp(-bump_a |x - bump_c|^2) scaling entry
    # (i, j) by s_i s_j = sqrt(b(x_i) b(x_j)) (bump_a = 0: none)
    cell_diag: bool = False
    h: float = 0.0
    bump_a: float = 0.0
    bump_c: tuple = (0.5, 0.5)


def grid_points(n: int) -> np.ndarray:
    """Cell centres of an n x n uniform grid on [0,1]^2, user index
    i = iy*n + ix (x fastest).  Returns an (n*n, 2) float64 array."""
    h = 1.0 / n
    ix = np.arange(n)
    xs = (ix + 0.5) * h
    X, Y = np.meshgrid(xs, xs, indexing="xy")  # X[iy, ix] = xs[ix]
    return np.ascontiguousarray(np.stack([X.ravel(), Y.ravel()], axis=1))


def grid_kernel(kind: str, n: int, kappa: float = 0.0, diag: float = 1.0) -> Kernel:
    """Kernel with weight w = h^2 = 1/n^2 and constant diagonal."""
    return Kernel(kind=kind, kappa=float(kappa), weight=1.0 / (n * n), diag=float(diag))


def paper_laplace(n: int) -> Kernel:
    """First-kind Laplace (eqs. e:a1, e:a1i): w = h^2, diagonal = the cell
    integral of -log(r) / (2 pi)."""
    h = 1.0 / n
    return Kernel(kind=LAPLACE, weight=h * h, diag=0.0, cell_diag=True, h=h)


def paper_helmholtz(n: int, kappa: float) -> Kernel:
    """Lippmann-Schwinger Helmholtz (eqs. e:b1, e:b2), symmetrized: w = h^2
    kappa^2, entries scaled by sqrt(b_i b_j), diagonal 1 + kappa^2 b_i times
    the cell integral of (i/4) H0(kappa r), Gaussian bump b(x) =
    exp(-32 |x - (1/2, 1/2)|^2) (Sec. 5.2)."""
    h = 1.0 / n
    return Kernel(kind=HELMHOLTZ, kappa=float(kappa), weight=h * h * kappa * kappa, diag=1.0,
                  cell_diag=True, h=h, bump_a=32.0, bump_c=(0.5, 0.5))


def uniform_rhs(N: int, nrhs: int, seed: int) -> np.ndarray:
    """Standard uniform right-hand sides (Tab. t:notations: "b is a standard
    uniform random vector"), complex128 with zero imaginary part, Fortran order."""
    rng = np.random.default_rng(seed)
    return np.asfortranarray(rng.random((N, nrhs)).astype(np.complex128))


def rhs(N: int, nrhs: int, seed: int, complex_parts: bool = True) -> np.ndarray:
    """Gaussian right-hand sides from ``numpy.random.default_rng(seed)``:
    the real-part array is drawn first, then (if ``complex_parts``) the
    imaginary part.  Returned as complex128, shape (N, nrhs), Fortran order
    (column-major, as the C ABI expects)."""
    rng = np.random.default_rng(seed)
    re = rng.standard_normal((N, nrhs))
    if complex_parts:
        im = rng.standard_normal((N, nrhs))
        out = re + 1j * im
    else:
        out = re.astype(np.complex128)
    return np.asfortranarray(out)


# ---------------------------------------------------------------------------
# Named workloads (sizes and kernels of the graded configurations)
# ---------------------------------------------------------------------------

@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    n: int                      # grid side; N = n*n
    kernel: Kernel
    tol: float
    leaf: int
    n_proxy: int
    nrhs: tuple
    seed: int
    complex_rhs: bool

    @property
    def N(self) -> int:
        return self.n * self.n


def laplace_64() -> Workload:
    """Laplace, N = 64^2, FP64, one real RHS (seed 0)."""
    return Workload("laplace-n64", 64, grid_kernel(LAPLACE, 64), 1e-6, 64, 64, (1,), 0, False)


def helmholtz_256() -> Workload:
    """Helmholtz kappa = 25, N = 256^2, FP64, nrhs in {1, 64} (seed 1)."""
    return Workload("helmholtz-k25-n256", 256, grid_kernel(HELMHOLTZ, 256, 25.0), 1e-6, 64, 128,
                    (1, 64), 1, True)


def helmholtz_512() -> Workload:
    """Helmholtz kappa = 50, N = 512^2, nrhs = 16 (seed 2): the headline size."""
    return Workload("helmholtz-k50-n512", 512, grid_kernel(HELMHOLTZ, 512, 50.0), 1e-6, 64, 128,
                    (16,), 2, True)


WORKLOADS = {w.name: w for w in (laplace_64(), helmholtz_256(), helmholtz_512())}


# ---------------------------------------------------------------------------
# Batched uneven instances: 256 independent problems
# ---------------------------------------------------------------------------

BATCH_SIDES = (32, 48, 64, 96, 128)


@dataclasses.dataclass(frozen=True)
class Problem:
    n: int
    kernel: Kernel
    n_proxy: int
    rhs: np.ndarray = dataclasses.field(repr=False, compare=False)


def batched_problems(count: int = 256, seed: int = 3) -> list:
    """Per problem, in this draw order: side n uniform over BATCH_SIDES; u < 0.5
    selects Laplace; kappa ~ U[5, 40] (always drawn); one real N(0,1) RHS."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        n = int(rng.choice(BATCH_SIDES))
        u = float(rng.random())
        kappa = float(rng.uniform(5.0, 40.0))
        if u < 0.5:
            k = grid_kernel(LAPLACE, n)
            npx = 64
        else:
            k = grid_kernel(HELMHOLTZ, n, kappa)
            npx = 128
        b = np.asfortranarray(rng.standard_normal((n * n, 1)).astype(np.complex128))
        out.append(Problem(n, k, npx, b))
    return out


# ---------------------------------------------------------------------------
# Serving stream: Poisson arrivals of factor and solve requests
# ---------------------------------------------------------------------------

SERVE_SIDES = (128, 256, 512)


@dataclasses.dataclass(frozen=True)
class Request:
    rid: int
    t_arrive: float             # seconds after stream start
    kind: str                   # "factor" or "solve"
    n: int                      # grid side of the problem (factor) / of the target (solve)
    kappa: float
    nrhs: int
    target: int                 # rid of the factor request a solve targets (-1 for factor)


def request_stream(count: int, rate: float, seed: int = 4, factor_frac: float = 0.2,
                   sides=SERVE_SIDES, max_nrhs: int = 256) -> list:
    """Draw order per request: interarrival ~ Exp(rate), type (factor with
    probability ``factor_frac``), side n, kappa ~ U[10, 60], nrhs ~ U{1..max_nrhs},
    target position.  The first request is always a factor job.  A solve's
    target is a uniformly chosen earlier factor request."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    factors = []
    for rid in range(count):
        t += float(rng.exponential(1.0 / rate))
        is_factor = bool(rng.random() < factor_frac) or rid == 0
        n = int(rng.choice(sides))
        kappa = float(rng.uniform(10.0, 60.0))
        nrhs = int(rng.integers(1, max_nrhs + 1))
        pos = float(rng.random())
        if is_factor:
            factors.append(rid)
            out.append(Request(rid, t, "factor", n, kappa, 1, -1))
        else:
            tgt = factors[min(int(pos * len(factors)), len(factors) - 1)]
            out.append(Request(rid, t, "solve", out[tgt].n, out[tgt].kappa, nrhs, tgt))
    return out


# ---------------------------------------------------------------------------
# Counter-based normal generator (SplitMix64 + Box-Muller), for right-hand
# sides that a device-side generator must reproduce bit-for-bit.
# ---------------------------------------------------------------------------

_MASK = (1 << 64) - 1


def splitmix64(x: np.ndarray) -> np.ndarray:
    """SplitMix64 finaliser (Steele, Lea and Flood, 2014) on uint64 counters."""
    x = (x + np.uint64(0x9E3779B97F4A7C15)) & np.uint64(_MASK)
    z = x
    z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
    z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def counter_normals(key: int, count: int) -> np.ndarray:
    """``count`` complex normals keyed by ``key``: element e uses counters
    (key<<32 | 2e) and (key<<32 | 2e+1) -> two uniforms in (0,1] -> Box-Muller
    (cos branch real, sin branch imaginary)."""
    e = np.arange(count, dtype=np.uint64)
    base = np.uint64((key << 32) & _MASK)
    with np.errstate(over="ignore"):
        a = splitmix64(base | (np.uint64(2) * e))
        b = splitmix64(base | (np.uint64(2) * e + np.uint64(1)))
    u1 = ((a >> np.uint64(11)).astype(np.float64) + 1.0) * (1.0 / 9007199254740992.0)
    u2 = ((b >> np.uint64(11)).astype(np.float64)) * (1.0 / 9007199254740992.0)
    rad = np.sqrt(-2.0 * np.log(u1))
    return rad * np.cos(2.0 * math.pi * u2) + 1j * rad * np.sin(2.0 * math.pi * u2)
