"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module produces *data* only: random numbers, knot vectors, control nets
and coefficient fields.  It holds none of the assembly arithmetic (no basis
evaluation at quadrature points, no integrands, no element loops), so both the
FP64 CPU oracle and the HIP library can consume its output without sharing
code with each other.

Random numbers come from a counter-based SplitMix64 generator (Steele, Lea and
Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014):
value(seed, stream, i) = mix64(key(seed, stream) + (i + 1) * GOLDEN), with
uniforms (x >> 11) * 2**-53 and normals by the Box-Muller transform.  No numpy
or torch generator is used, so every draw is reproducible from its definition.
"""
from __future__ import annotations

import functools
import math
from dataclasses import dataclass, field

import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_STREAM_MUL = np.uint64(0xD1B54A32D192ED03)


def _mix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 finaliser (wrapping uint64 arithmetic)."""
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def _key(seed: int, stream: int) -> np.uint64:
    with np.errstate(over="ignore"):
        k = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) * GOLDEN
        k = k ^ (np.uint64(stream & 0xFFFFFFFFFFFFFFFF) * _STREAM_MUL)
    return _mix64(np.array([k], dtype=np.uint64))[0]


def rand_u64(seed: int, stream: int, n: int, offset: int = 0) -> np.ndarray:
    """n raw 64-bit outputs of the counter generator, counters offset..offset+n-1."""
    idx = np.arange(offset + 1, offset + n + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = _key(seed, stream) + idx * GOLDEN
    return _mix64(z)


def uniform(seed: int, stream: int, n: int, lo: float = 0.0, hi: float = 1.0, offset: int = 0) -> np.ndarray:
    """Uniform doubles in [lo, hi) with 53 random bits each."""
    x = rand_u64(seed, stream, n, offset)
    u = (x >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
    return lo + (hi - lo) * u


def normal(seed: int, stream: int, n: int, offset: int = 0) -> np.ndarray:
    """Standard normals by Box-Muller from pairs of uniforms (2 counters per pair)."""
    m = (n + 1) // 2
    u = uniform(seed, stream, 2 * m, offset=2 * offset)
    u1 = 1.0 - u[0::2]          # (0, 1]: log is finite
    u2 = u[1::2]
    r = np.sqrt(-2.0 * np.log(u1))
    z = np.empty(2 * m)
    z[0::2] = r * np.cos(2.0 * np.pi * u2)
    z[1::2] = r * np.sin(2.0 * np.pi * u2)
    return z[:n]


def randint(seed: int, stream: int, n: int, lo: int, hi: int, offset: int = 0) -> np.ndarray:
    """Integers uniform in the inclusive range [lo, hi] (floor of a uniform)."""
    u = uniform(seed, stream, n, offset=offset)
    return lo + np.minimum(np.floor(u * (hi - lo + 1)).astype(np.int64), hi - lo)


# --------------------------------------------------------------------------------------------
# Knot vectors
# --------------------------------------------------------------------------------------------

def open_uniform_knots(nel: int, p: int, cont: int | None = None, a: float = 0.0, b: float = 1.0) -> np.ndarray:
    """Open knot vector on [a,b] with nel equal spans, end multiplicity p+1 and
    interior multiplicity p-cont (continuity C^cont, default C^(p-1))."""
    if cont is None:
        cont = p - 1
    mult = p - cont
    if not (1 <= mult <= p):
        raise ValueError("continuity must be in [0, p-1]")
    inner = [a + (b - a) * i / nel for i in range(1, nel)]
    kv = [a] * (p + 1)
    for x in inner:
        kv += [x] * mult
    kv += [b] * (p + 1)
    return np.array(kv, dtype=np.float64)


def ndofs_1d(knots: np.ndarray, p: int) -> int:
    return len(knots) - p - 1


# --------------------------------------------------------------------------------------------
# Exact NURBS quarter annulus / thick quarter cylinder (homogeneous-coordinate refinement)
# --------------------------------------------------------------------------------------------

def _elevate_bezier(Pw: np.ndarray, axis: int) -> np.ndarray:
    """Raise a single-span Bezier control net by one degree along `axis`
    (homogeneous coordinates): Q_i = (i/(p+1)) P_{i-1} + (1 - i/(p+1)) P_i."""
    Pw = np.moveaxis(Pw, axis, 0)
    p = Pw.shape[0] - 1
    Q = np.zeros((p + 2,) + Pw.shape[1:])
    for i in range(p + 2):
        a = i / (p + 1)
        if i >= 1:
            Q[i] += a * Pw[i - 1]
        if i <= p:
            Q[i] += (1.0 - a) * Pw[i]
    return np.moveaxis(Q, 0, axis)


def _insert_knot(U: np.ndarray, p: int, Pw: np.ndarray, x: float, axis: int):
    """Insert knot x once (Boehm) along `axis` of a homogeneous control net."""
    Pw = np.moveaxis(Pw, axis, 0)
    n = Pw.shape[0]
    k = int(np.searchsorted(U, x, side="right")) - 1      # U[k] <= x < U[k+1]
    Q = np.zeros((n + 1,) + Pw.shape[1:])
    for i in range(n + 1):
        if i <= k - p:
            Q[i] = Pw[i]
        elif i >= k + 1:
            Q[i] = Pw[i - 1]
        else:
            al = (x - U[i]) / (U[i + p] - U[i])
            Q[i] = al * Pw[i] + (1.0 - al) * Pw[i - 1]
    U2 = np.insert(U, k + 1, x)
    return U2, np.moveaxis(Q, 0, axis)


@dataclass
class Patch:
    """A tensor-product NURBS patch: knots per axis, degrees, control points (N x dim, natural
    order with axis 0 fastest) and weights (N)."""
    knots: list
    degree: list
    ctrl: np.ndarray | None = None
    weights: np.ndarray | None = None

    @property
    def dim(self):
        return len(self.knots)

    @property
    def shape(self):
        return [len(U) - p - 1 for U, p in zip(self.knots, self.degree)]

    @property
    def ndof(self):
        return int(np.prod(self.shape))


def unit_box(dim: int, nel: int | list, p: int | list, cont=None) -> Patch:
    nel = [nel] * dim if np.isscalar(nel) else list(nel)
    p = [p] * dim if np.isscalar(p) else list(p)
    return Patch([open_uniform_knots(n, q, cont) for n, q in zip(nel, p)], p, None, None)


def quarter_cylinder(nel: int | list, p: int, dim: int = 3, r0: float = 1.0, r1: float = 2.0,
                     height: float = 1.0) -> Patch:
    """Thick quarter cylinder (dim=3) or quarter annulus (dim=2).

    Axis 0 is radial (r0 -> r1, linear), axis 1 the angle 0 -> pi/2 (exact rational quadratic,
    weights 1, sqrt(2)/2, 1), axis 2 the height (linear).  This ordering keeps det J > 0.
    Each axis is degree-elevated to p on its single Bezier span, then nel-1 uniform
    parametric knots are inserted once each, giving C^(p-1) continuity.
    """
    nel = [nel] * dim if np.isscalar(nel) else list(nel)
    s = math.sqrt(0.5)
    deg = [1, 2, 1][:dim]
    shape = [2, 3, 2][:dim]
    Pw = np.zeros(tuple(shape) + (dim + 1,))
    for idx in np.ndindex(*shape):
        r = r0 + (r1 - r0) * idx[0]
        ang = [(r, 0.0, 1.0), (r, r, s), (0.0, r, 1.0)][idx[1]]
        w = ang[2]
        x = np.array([ang[0], ang[1]] + ([height * idx[2]] if dim == 3 else []))
        Pw[idx][:dim] = w * x
        Pw[idx][dim] = w
    knots = []
    for ax in range(dim):
        q = deg[ax]
        while q < p:
            Pw = _elevate_bezier(Pw, ax)
            q += 1
        U = np.array([0.0] * (p + 1) + [1.0] * (p + 1))
        for i in range(1, nel[ax]):
            U, Pw = _insert_knot(U, p, Pw, i / nel[ax], ax)
        knots.append(U)
    # natural order: axis 0 fastest  -> transpose index order (i0,i1,i2) to (i2,i1,i0) flattening
    N = int(np.prod(Pw.shape[:dim]))
    Pw_nat = np.transpose(Pw, tuple(range(dim - 1, -1, -1)) + (dim,)).reshape(N, dim + 1)
    w = Pw_nat[:, dim].copy()
    ctrl = Pw_nat[:, :dim] / w[:, None]
    return Patch(knots, [p] * dim, np.ascontiguousarray(ctrl), np.ascontiguousarray(w))


def greville(U: np.ndarray, p: int) -> np.ndarray:
    n = len(U) - p - 1
    return np.array([U[i + 1:i + p + 1].mean() for i in range(n)])


# --------------------------------------------------------------------------------------------
# Gaussian random fields (squared-exponential covariance) by random Fourier features
# --------------------------------------------------------------------------------------------

def grf_rff(points: np.ndarray, seed: int, stream: int, var: float = 0.5, corr: float = 0.2,
            nfeat: int = 4096) -> np.ndarray:
    """Zero-mean field with covariance var*exp(-|x-y|^2/(2 corr^2)) approximated by nfeat random
    Fourier features: g(x) = sqrt(2 var / M) sum_m cos(w_m . x + b_m), w ~ N(0, corr^-2 I),
    b ~ U[0, 2 pi)."""
    pts = np.atleast_2d(points)
    d = pts.shape[1]
    w = normal(seed, stream, nfeat * d).reshape(nfeat, d) / corr
    b = uniform(seed, stream + 1_000_003, nfeat, 0.0, 2.0 * np.pi)
    out = np.empty(pts.shape[0])
    step = 8192
    for i in range(0, pts.shape[0], step):
        ph = pts[i:i + step] @ w.T + b
        out[i:i + step] = np.cos(ph).sum(axis=1)
    return math.sqrt(2.0 * var / nfeat) * out


def grf_grid(n: int, seed: int, stream: int, var: float = 0.5, corr: float = 0.2, h: float | None = None) -> np.ndarray:
    """Zero-mean field with covariance var*exp(-|x-y|^2/(2 corr^2)) at the centres of an n x n
    grid of spacing h (default 1/n), by circulant embedding: the grid is embedded in a 2n x 2n
    periodic grid (period 2 n h, so wrap-around correlation is exp(-(n h)^2/(2 corr^2)), below
    1e-5 for n h = 1, corr = 0.2), the covariance's eigenvalues are its FFT, and the field is
    the inverse FFT of sqrt(eigenvalues) times the FFT of white noise.  Returns [n, n] with axis 1
    varying along x."""
    h = 1.0 / n if h is None else h
    m = 2 * n
    xi = normal(seed, stream, m * m).reshape(m, m)
    g = np.fft.ifft2(_grf_sqrt_eigs(n, h, var, corr) * np.fft.fft2(xi)).real
    return g[:n, :n]


@functools.lru_cache(maxsize=16)
def _grf_sqrt_eigs(n: int, h: float, var: float, corr: float) -> np.ndarray:
    m = 2 * n
    d = np.minimum(np.arange(m), m - np.arange(m)) * h
    r2 = d[:, None] ** 2 + d[None, :] ** 2
    lam = np.fft.fft2(var * np.exp(-r2 / (2.0 * corr * corr))).real
    return np.sqrt(np.maximum(lam, 0.0))


# --------------------------------------------------------------------------------------------
# Workload recipes (the configurations the tests and the benchmark use)
# --------------------------------------------------------------------------------------------

def boundary_mask(shape: list) -> np.ndarray:
    """Boolean mask (natural order) of coefficients on any face of the patch."""
    dim = len(shape)
    grids = np.meshgrid(*[np.arange(n) for n in shape[::-1]], indexing="ij")
    m = np.zeros(grids[0].shape, dtype=bool)
    for ax in range(dim):
        g = grids[dim - 1 - ax]
        m |= (g == 0) | (g == shape[ax] - 1)
    return m.reshape(-1)


def initial_guess(shape: list, seed: int, stream: int = 0, lo: float = 0.0, hi: float = 0.1,
                  dirichlet: bool = True) -> np.ndarray:
    """U0 ~ U[lo,hi) drawn over all N coefficients in natural order, then the Dirichlet
    coefficients overwritten with 0."""
    N = int(np.prod(shape))
    U = uniform(seed, stream, N, lo, hi)
    if dirichlet:
        U[boundary_mask(shape)] = 0.0
    return U


@dataclass
class Workload:
    name: str
    patch: Patch
    lam: float
    kappa_mode: int = 0          # 0 one, 1 nodal, 2 element
    kappa: np.ndarray | None = None
    U0: np.ndarray | None = None
    tol: float = 1e-10
    tol_relative: bool = False
    extra: dict = field(default_factory=dict)


def bratu_box(dim: int, nel: int, p: int, lam: float, seed: int, stream: int = 0) -> Workload:
    patch = unit_box(dim, nel, p)
    U0 = initial_guess(patch.shape, seed, stream)
    return Workload(f"bratu{dim}d-{nel}^{dim}-p{p}", patch, lam, 0, None, U0)


def config_2d_small() -> Workload:
    """2D Bratu, unit square, 16x16 elements, p=2 C^1, 3x3 Gauss points, lambda=6, seed 1."""
    w = bratu_box(2, 16, 2, 6.0, seed=1)
    w.tol, w.tol_relative = 1e-10, False
    return w


def config_3d_bratu(nel: int = 64, p: int = 3) -> Workload:
    """3D Bratu, unit cube, 64^3 elements, p=3 C^2, 4^3 Gauss points, lambda=5, seed 2."""
    w = bratu_box(3, nel, p, 5.0, seed=2)
    w.tol, w.tol_relative = 1e-10, True
    return w


def config_cylinder(nel: int = 48, p: int = 2, lam: float = 1.0, dim: int = 3) -> Workload:
    """Nonlinear diffusion on the thick quarter cylinder; kappa = exp(GRF(0.5, 0.2)) at the
    control points; lambda=1 (reading); seed 3."""
    patch = quarter_cylinder(nel, p, dim=dim)
    g = grf_rff(patch.ctrl, seed=3, stream=1)
    kappa = np.exp(g)
    U0 = initial_guess(patch.shape, seed=3, stream=0)
    return Workload(f"cylinder{dim}d-{nel}^{dim}-p{p}", patch, lam, 1, kappa, U0, 1e-10, True)


def batched_instances(n: int = 512, seed: int = 4):
    """Uneven 2D Bratu instances: n_el ~ U{8..128}, p ~ U{2,3,4}, lambda ~ U[1,6.5)."""
    nel = randint(seed, 1_000_001, n, 8, 128)
    deg = randint(seed, 1_000_002, n, 2, 4)
    lam = uniform(seed, 1_000_003, n, 1.0, 6.5)
    out = []
    for i in range(n):
        w = bratu_box(2, int(nel[i]), int(deg[i]), float(lam[i]), seed=seed, stream=i)
        out.append(w)
    return out


def learned_instance(index: int, seed: int = 5, nel: int = 64, p: int = 3, ncell: int = 32):
    """Instance for the learned-guess workload: log kappa = GRF(0.5, 0.2) at the ncell^2 cell
    centres (kappa constant per cell = (nel/ncell)^2 elements), lambda ~ U[1,6]."""
    logk = grf_grid(ncell, seed=seed, stream=2 * index + 10)        # [y][x]
    lam = float(uniform(seed, 7, 1, 1.0, 6.0, offset=index)[0])
    r = nel // ncell
    kel = np.exp(np.repeat(np.repeat(logk, r, axis=0), r, axis=1)).reshape(-1)   # element natural order
    patch = unit_box(2, nel, p)
    return logk, lam, Workload(f"learned-{index}", patch, lam, 2, kel, np.zeros(patch.ndof), 1e-10, False)
