"""Seeded synthetic inputs shared by the CPU oracle and the HIP path.

This module only builds problem data (sparse A, dense B and C, shift sets
chosen from closed-form spectral bounds).  A shift set is an input of the
method (the paper's heuristic is implemented on both sides separately); the
real sets here only need the spectral interval.  It holds none of the method's
arithmetic: no Riccati/Lyapunov algebra, no ADI, no factor decompositions.

Problem families (the paper's workloads and the synthetic stand-ins for the
SuiteSparse matrices that are not available here):

* ``fdm2d``  - 2D convection-diffusion, 5-point central differences.
* ``fdm3d``  - 3D convection-diffusion, 7-point central differences, with a
  constant or a rotating convection field.
* ``ex1``    - the deterministic dense problem of Example 1 (Sec. 5.1).
* ``dense_instance`` - dense A = -Q diag(logspace(0, q, n)) Q^T with Haar Q
  (a batch of these sweeps the Lyapunov-operator condition number).
* ``toeplitz`` - the 5-diagonal Toeplitz matrix of the Toeplitz example
  (Sec. 5.2).

Random data come from ``numpy.random.default_rng(seed)`` (PCG64).  The paper
fixes its MATLAB stream with seed 1220 (Sec. 5); the same integer is the
default seed here, MATLAB's stream itself cannot be reproduced.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

DEFAULT_SEED = 1220


# ----------------------------------------------------------------------------
# sparse generators
# ----------------------------------------------------------------------------
def _tridiag(N: int, lo: float, d: float, up: float) -> sp.csr_matrix:
    """N x N tridiagonal Toeplitz matrix (sub-diagonal lo, diagonal d, super up)."""
    return sp.diags([np.full(N - 1, lo), np.full(N, d), np.full(N - 1, up)],
                    [-1, 0, 1], shape=(N, N), format="csr")


def fdm1d_coeffs(N: int, nu: float):
    """Central-difference coefficients of u'' - nu u' on N interior points of
    (0, 1) with h = 1/(N+1): (sub, diag, super)."""
    h = 1.0 / (N + 1)
    return 1.0 / h ** 2 + nu / (2 * h), -2.0 / h ** 2, 1.0 / h ** 2 - nu / (2 * h)


def fdm2d(N: int, nu: float = 10.0) -> sp.csr_matrix:
    """2D convection-diffusion  Lap(u) - nu (u_x + u_y)  on the unit square,
    homogeneous Dirichlet boundary, N x N interior grid, lexicographic order
    with x fastest.  A = I (x) T + T (x) I (Kronecker sum), n = N^2 rows,
    5N^2 - 4N nonzeros.  Stable and nonsymmetric for nu > 0 with cell Peclet
    number nu h / 2 < 1 (real spectrum)."""
    T = _tridiag(N, *fdm1d_coeffs(N, nu))
    I = sp.identity(N, format="csr")
    A = (sp.kron(I, T) + sp.kron(T, I)).tocsr()
    A.sort_indices()
    A.eliminate_zeros()
    return A


def fdm2d_eigenvalues(N: int, nu: float = 10.0) -> np.ndarray:
    """Closed-form spectrum of ``fdm2d``: sums of the tridiagonal Toeplitz
    eigenvalues  d + 2 sqrt(lo*up) cos(k pi/(N+1)), k = 1..N."""
    lo, d, up = fdm1d_coeffs(N, nu)
    k = np.arange(1, N + 1)
    t = d + 2.0 * math.sqrt(lo * up) * np.cos(k * math.pi / (N + 1))
    return (t[:, None] + t[None, :]).ravel()


def fdm2d_spectral_bounds(N: int, nu: float = 10.0):
    """(lambda_min, lambda_max) magnitudes of the real negative spectrum of
    ``fdm2d`` from the closed form: |lambda| in [lo, hi]."""
    lo, d, up = fdm1d_coeffs(N, nu)
    c = 2.0 * math.sqrt(lo * up)
    t_max = d + c * math.cos(math.pi / (N + 1))       # closest to zero
    t_min = d + c * math.cos(N * math.pi / (N + 1))   # most negative
    return -2.0 * t_max, -2.0 * t_min


def fdm3d(N: int, nu: float = 100.0, field_kind: str = "rotating") -> sp.csr_matrix:
    """3D convection-diffusion  Lap(u) - v . grad(u)  on the unit cube with
    homogeneous Dirichlet boundary, N^3 interior points, 7-point central
    differences, lexicographic order with x fastest.

    field_kind = "rotating": v = nu * (-(y - 1/2), x - 1/2, 0)  (complex
    spectrum for large enough nu); "constant": v = (nu, nu, nu) (real
    spectrum)."""
    h = 1.0 / (N + 1)
    n = N ** 3
    idx = np.arange(n)
    i = idx % N
    j = (idx // N) % N
    k = idx // (N * N)
    x = (i + 1) * h
    y = (j + 1) * h
    if field_kind == "rotating":
        vx = -nu * (y - 0.5)
        vy = nu * (x - 0.5)
        vz = np.zeros(n)
    elif field_kind == "constant":
        vx = np.full(n, nu)
        vy = np.full(n, nu)
        vz = np.full(n, nu)
    else:
        raise ValueError(field_kind)
    inv_h2 = 1.0 / h ** 2
    rows, cols, vals = [idx], [idx], [np.full(n, -6.0 * inv_h2)]
    for coord, stride, v in ((i, 1, vx), (j, N, vy), (k, N * N, vz)):
        m = coord > 0                       # neighbour at -h
        rows.append(idx[m]); cols.append(idx[m] - stride)
        vals.append(inv_h2 + v[m] / (2 * h))
        m = coord < N - 1                   # neighbour at +h
        rows.append(idx[m]); cols.append(idx[m] + stride)
        vals.append(inv_h2 - v[m] / (2 * h))
    A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n))
    A.sort_indices()
    A.eliminate_zeros()
    return A


def toeplitz5(n: int) -> sp.csr_matrix:
    """5-diagonal Toeplitz matrix of the Toeplitz example (Sec. 5.2):
    sub-diagonal 1, diagonal -2.8, first three super-diagonals -1."""
    A = sp.diags([np.ones(n - 1), np.full(n, -2.8), -np.ones(n - 1), -np.ones(n - 2),
                  -np.ones(n - 3)], [-1, 0, 1, 2, 3], shape=(n, n), format="csr")
    A.sort_indices()
    return A


# ----------------------------------------------------------------------------
# dense generators
# ----------------------------------------------------------------------------
def gallery_orthog(n: int) -> np.ndarray:
    """Symmetric orthogonal matrix V_ij = sqrt(2/(n+1)) sin(i j pi/(n+1))
    (MATLAB gallery('orthog', n) with its default kind 1)."""
    i = np.arange(1, n + 1)
    return math.sqrt(2.0 / (n + 1)) * np.sin(np.outer(i, i) * math.pi / (n + 1))


def ex1(n: int = 1000, m: int = 10, p: int = 5, q: float = 1.0):
    """Example 1 (Sec. 5.1): A = -V diag(logspace(0, q, n)) V^T,
    B = 0.2 ones(n, m), C = 0.1 ones(p, n).  kappa_2(A) = 10^q."""
    V = gallery_orthog(n)
    A = -(V * np.logspace(0.0, q, n)) @ V.T
    return A, np.full((n, m), 0.2), np.full((p, n), 0.1)


def haar_orthogonal(n: int, rng: np.random.Generator) -> np.ndarray:
    """Haar-distributed orthogonal matrix: QR of a Gaussian matrix with the
    signs of diag(R) made positive."""
    G = rng.standard_normal((n, n))
    Q, R = np.linalg.qr(G)
    return Q * np.sign(np.diag(R))


DENSE_SIZES = (256, 384, 512, 768, 1024, 1536, 2048)


def dense_instance(i: int, count: int = 64, m: int = 4, p: int = 4, seed: int = DEFAULT_SEED,
                   sizes=DENSE_SIZES):
    """Instance i of the dense batch: n = sizes[i mod len(sizes)],
    q = 2 + 10 i/(count-1), A = -Q diag(logspace(0, q, n)) Q^T (kappa_2 = 10^q),
    Gaussian B (n x m) and C (p x n).  Draw order: Q, B, C."""
    n = sizes[i % len(sizes)]
    q = 2.0 + 10.0 * i / max(count - 1, 1)
    rng = np.random.default_rng(seed + i)
    Q = haar_orthogonal(n, rng)
    A = -(Q * np.logspace(0.0, q, n)) @ Q.T
    B = rng.standard_normal((m, n)).T.copy()
    C = rng.standard_normal((p, n))
    return A, B, C, q


# ----------------------------------------------------------------------------
# low-rank factors and shifts
# ----------------------------------------------------------------------------
def gaussian_factors(n: int, m: int, p: int, seed: int = DEFAULT_SEED):
    """Gaussian B (n x m, filled column by column) then C (p x n), N(0, 1)."""
    rng = np.random.default_rng(seed)
    B = rng.standard_normal((m, n)).T.copy()
    C = rng.standard_normal((p, n))
    return B, C


def logspaced_real_shifts(lo: float, hi: float, count: int, descending: bool = True) -> np.ndarray:
    """`count` negative real shifts, geometrically spaced over the spectral
    magnitude interval [lo, hi]; returned as complex128 (imaginary part 0).

    The default order starts at the largest magnitude.  The shift set, not its
    order, fixes the iterate after a full cycle (the ADI factors commute), but
    a stopping test met mid-cycle sees the order: a random right-hand side
    carries most of its energy in the many large-magnitude modes of a
    diffusion operator, so the large shifts first reach a loose tolerance in
    fewer steps."""
    s = np.geomspace(lo, hi, count)
    if descending:
        s = s[::-1]
    return -s.astype(np.complex128)


def wachspress_real_shifts(lo: float, hi: float, count: int) -> np.ndarray:
    """`count` negative real ADI shifts for a real spectrum with magnitudes in
    [lo, hi]: the parameters that minimise max over lambda in [lo, hi] of
    prod_j |lambda - p_j| / |lambda + p_j| (Zolotarev's third problem, solved
    by Wachspress with Jacobi elliptic functions):
    p_j = hi dn((2j - 1) K / (2 count), k), j = 1..count, with modulus
    k = sqrt(1 - (lo/hi)^2) and K = K(k) the complete elliptic integral of
    the first kind.  dn falls from 1 at u = 0 to lo/hi at u = K, so the set
    starts at the largest magnitude (the order used for the log-spaced sets).
    Returned as complex128 (imaginary part 0)."""
    from scipy.special import ellipj, ellipk   # parameter m = k^2
    if not (0 < lo <= hi) or count < 1:
        raise ValueError("need 0 < lo <= hi and count >= 1")
    m = 1.0 - (lo / hi) ** 2
    u = (2.0 * np.arange(1, count + 1) - 1.0) * ellipk(m) / (2.0 * count)
    dn = ellipj(u, m)[2]
    return -(hi * dn).astype(np.complex128)


# ----------------------------------------------------------------------------
# named configurations
# ----------------------------------------------------------------------------
@dataclass
class Problem:
    name: str
    A: object                 # scipy.sparse.csr_matrix or dense ndarray
    B: np.ndarray
    C: np.ndarray
    shifts: np.ndarray = field(default=None)
    meta: dict = field(default_factory=dict)

    @property
    def n(self):
        return self.A.shape[0]


def fdm2d_problem(N: int, m: int, p: int, nu: float = 10.0, seed: int = DEFAULT_SEED,
                  nshifts: int = 12, name: str = None, shift_set: str = "wachspress") -> Problem:
    """2D FDM CARE with Gaussian B, C and real shifts for the closed-form
    spectral interval: ``nshifts`` Wachspress (minimax) shifts by default,
    or log-spaced ones (``shift_set="logspaced"``)."""
    A = fdm2d(N, nu)
    B, C = gaussian_factors(N * N, m, p, seed)
    lo, hi = fdm2d_spectral_bounds(N, nu)
    if shift_set == "wachspress":
        shifts = wachspress_real_shifts(lo, hi, nshifts)
    elif shift_set == "logspaced":
        shifts = logspaced_real_shifts(lo, hi, nshifts)
    else:
        raise ValueError(f"unknown shift set {shift_set!r}")
    return Problem(name or f"fdm2d_N{N}_m{m}_p{p}", A, B, C, shifts,
                   dict(N=N, nu=nu, seed=seed, lam_lo=lo, lam_hi=hi, shift_set=shift_set))


def fdm3d_problem(N: int, m: int, p: int, nu: float = 100.0, field_kind: str = "rotating",
                  seed: int = DEFAULT_SEED, name: str = None) -> Problem:
    """3D FDM CARE with Gaussian B, C; no shift set (the complex spectrum of
    the rotating field has no closed form: the shifts come from the
    heuristic)."""
    A = fdm3d(N, nu, field_kind)
    B, C = gaussian_factors(N ** 3, m, p, seed)
    return Problem(name or f"fdm3d_N{N}_m{m}_p{p}_{field_kind}", A, B, C, None,
                   dict(N=N, nu=nu, field=field_kind, seed=seed))


def toeplitz_problem(n: int, m: int = 10, p: int = 5, seed: int = DEFAULT_SEED, name: str = None) -> Problem:
    """The Toeplitz example of Sec. 5.2: the 5-diagonal Toeplitz A, Gaussian
    B scaled to ||B||_F = 1, Gaussian C; no shift set (the paper generates
    its shifts from Krylov subspaces: the heuristic here)."""
    A = toeplitz5(n)
    B, C = gaussian_factors(n, m, p, seed)
    B /= np.linalg.norm(B)
    return Problem(name or f"toeplitz_n{n}_m{m}_p{p}", A, B, C, None, dict(seed=seed))


def config3() -> Problem:
    """64^3 grid (n = 262,144, nnz = 1,810,432), rotating field, m = 1, p = 10."""
    return fdm3d_problem(64, 1, 10, name="cfg3_fdm3d_64")


def config1() -> Problem:
    """20 x 20 grid (n = 400, nnz = 1920), nu = 10, m = p = 1."""
    return fdm2d_problem(20, 1, 1, name="cfg1_fdm2d_20x20")


def config2() -> Problem:
    """500 x 500 grid (n = 250000, nnz = 1,248,000), nu = 10, m = p = 5."""
    return fdm2d_problem(500, 5, 5, name="cfg2_fdm2d_500x500")


def fdm_batch_sizes(count: int = 32, seed: int = DEFAULT_SEED):
    """Grid sizes and (m, p) of the uneven FDM batch:
    N_i = round(100 * 6.32^(i/(count-1))), m_i, p_i uniform in {1..8}."""
    rng = np.random.default_rng(seed)
    Ns = [int(round(100 * 6.32 ** (i / (count - 1)))) for i in range(count)]
    ms = rng.integers(1, 9, size=count)
    ps = rng.integers(1, 9, size=count)
    return Ns, [int(v) for v in ms], [int(v) for v in ps]


def fdm_batch_problem(i: int, count: int = 32, seed: int = DEFAULT_SEED) -> Problem:
    """Instance i of the uneven FDM batch: grid N_i, (m_i, p_i) from
    ``fdm_batch_sizes``, Gaussian factors from seed + i, 12 Wachspress shifts."""
    Ns, ms, ps = fdm_batch_sizes(count, seed)
    return fdm2d_problem(Ns[i], ms[i], ps[i], seed=seed + i, name=f"batch{i}_fdm2d_{Ns[i]}")
