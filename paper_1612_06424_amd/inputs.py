"""Seeded synthetic inputs for the Wilson-Dirac hot path.

This module only draws random numbers and shapes them into gauge links,
sources and pseudofermion fields; it holds none of the operator's arithmetic
and imports nothing else from this package, so both the HIP path and the
CPU oracle can take their inputs from it.

The paper's quenched beta = 6.0 ensembles (Sec. 5) are not available; random
SU(3) links U = exp(i eps H) stand in for them (H traceless Hermitian with
Gaussian entries).  Bandwidth does not depend on the values; iteration counts
do.

Natural layouts returned here (site s = ((t*L + z)*L + y)*L + x):
  links   complex128 (V, 4, 3, 3)   U[s, mu, row, col], mu = 0 time, 1..3 = x, y, z
  fields  complex128 (ncol, V, 12)  component c = 3*spin + colour
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "random_links", "point_sources", "gaussian_field", "site_index",
    "WORKLOADS", "batched_domains",
]


def site_index(T: int, L: int, t: int, x: int, y: int, z: int) -> int:
    """Linear site index with time slowest and x fastest."""
    return ((t * L + z) * L + y) * L + x


def _expi_traceless_hermitian(q):
    """exp(i Q) for traceless Hermitian 3x3 matrices Q given entry-wise:
    q[i][j] are equally shaped complex arrays.  Returns the entries likewise.

    Cayley-Hamilton form exp(iQ) = f0 + f1 Q + f2 Q^2 with the coefficients of
    Morningstar and Peardon, Phys. Rev. D 69 (2004) 054501, Eqs. (23)-(34):
    c0 = det Q, c1 = tr Q^2 / 2, theta = arccos(|c0| / c0_max),
    u = sqrt(c1/3) cos(theta/3), w = sqrt(c1) sin(theta/3); negative c0 uses
    f_j(-c0) = (-1)^j conj(f_j(c0)).  Exact up to rounding, fully vectorised.
    """
    q2 = [[q[i][0] * q[0][j] + q[i][1] * q[1][j] + q[i][2] * q[2][j] for j in range(3)] for i in range(3)]
    c1 = 0.5 * (q2[0][0] + q2[1][1] + q2[2][2]).real
    c0 = (q[0][0] * (q[1][1] * q[2][2] - q[1][2] * q[2][1])
          - q[0][1] * (q[1][0] * q[2][2] - q[1][2] * q[2][0])
          + q[0][2] * (q[1][0] * q[2][1] - q[1][1] * q[2][0])).real
    neg = c0 < 0
    c0max = 2.0 * (c1 / 3.0) ** 1.5
    ratio = np.where(c0max > 0, np.abs(c0) / np.where(c0max > 0, c0max, 1.0), 0.0)
    theta = np.arccos(np.clip(ratio, -1.0, 1.0))
    u = np.sqrt(c1 / 3.0) * np.cos(theta / 3.0)
    w = np.sqrt(c1) * np.sin(theta / 3.0)
    small = np.abs(w) < 0.05
    w2 = w * w
    xi0 = np.where(small, 1 - w2 / 6 * (1 - w2 / 20 * (1 - w2 / 42)), np.sin(w) / np.where(small, 1.0, w))
    e2iu = np.exp(2j * u)
    emiu = np.exp(-1j * u)
    cw = np.cos(w)
    h0 = (u * u - w2) * e2iu + emiu * (8 * u * u * cw + 2j * u * (3 * u * u + w2) * xi0)
    h1 = 2 * u * e2iu - emiu * (2 * u * cw - 1j * (3 * u * u - w2) * xi0)
    h2 = e2iu - emiu * (cw + 3j * u * xi0)
    den = 9 * u * u - w2
    f0, f1, f2 = h0 / den, h1 / den, h2 / den
    f0 = np.where(neg, np.conj(f0), f0)
    f1 = np.where(neg, -np.conj(f1), f1)
    f2 = np.where(neg, np.conj(f2), f2)
    return [[f1 * q[i][j] + f2 * q2[i][j] + (f0 if i == j else 0.0) for j in range(3)] for i in range(3)]


def expi_matrices(Q: np.ndarray) -> np.ndarray:
    """exp(i Q) for an array (..., 3, 3) of traceless Hermitian matrices."""
    e = _expi_traceless_hermitian([[np.ascontiguousarray(Q[..., i, j]) for j in range(3)] for i in range(3)])
    out = np.empty(Q.shape, dtype=np.complex128)
    for i in range(3):
        for j in range(3):
            out[..., i, j] = e[i][j]
    return out


def random_links(T: int, L: int, eps: float, seed: int) -> np.ndarray:
    """U = exp(i eps H) per link, H traceless Hermitian with Gaussian entries.

    Normalisation: H_ii ~ N(0,1); for i < j, H_ij = a + i b with a, b ~ N(0,1)
    and H_ji = conj(H_ij); then H <- H - tr(H)/3, so E tr H^2 = 14.  The nine
    reals per link come from numpy PCG64 ``standard_normal((T,L,L,L,4,9))`` in
    the order (H00, H11, H22, Re H01, Im H01, Re H02, Im H02, Re H12, Im H12).
    The exponential is exact up to rounding (closed Cayley-Hamilton form);
    tr H = 0 gives det U = 1.
    """
    rng = np.random.default_rng(seed)
    n = T * L * L * L * 4
    g = np.ascontiguousarray(rng.standard_normal((T, L, L, L, 4, 9)).reshape(n, 9).T)
    out = np.empty((n, 3, 3), dtype=np.complex128)
    chunk = 1 << 18  # bounds host memory on large lattices
    for lo in range(0, n, chunk):
        sl = slice(lo, min(n, lo + chunk))
        tr = (g[0, sl] + g[1, sl] + g[2, sl]) / 3.0
        d = [eps * (g[k, sl] - tr) + 0j for k in range(3)]
        h01 = eps * (g[3, sl] + 1j * g[4, sl])
        h02 = eps * (g[5, sl] + 1j * g[6, sl])
        h12 = eps * (g[7, sl] + 1j * g[8, sl])
        q = [[d[0], h01, h02], [np.conj(h01), d[1], h12], [np.conj(h02), np.conj(h12), d[2]]]
        e = _expi_traceless_hermitian(q)
        for i in range(3):
            for j in range(3):
                out[sl, i, j] = e[i][j]
    return out.reshape(T * L * L * L, 4, 3, 3)


def point_sources(T: int, L: int, t: int, x: int, y: int, z: int) -> np.ndarray:
    """The 12 spin-colour point sources eta^(j)(y) = delta_{y,x_s} e_j, shape (12, V, 12)."""
    V = T * L * L * L
    s = site_index(T, L, t, x, y, z)
    eta = np.zeros((12, V, 12), dtype=np.complex128)
    for j in range(12):
        eta[j, s, j] = 1.0
    return eta


def gaussian_field(nsite: int, ncol: int, seed: int) -> np.ndarray:
    """Complex Gaussian field with Re, Im ~ N(0, 1/2), shape (ncol, nsite, 12)."""
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((ncol, nsite, 12, 2)) * np.sqrt(0.5)
    return (g[..., 0] + 1j * g[..., 1]).astype(np.complex128)


# Workloads of the hot path, named by what they are.  Seeds follow the recipe
# stated in the design notes; domains are time slabs [t0, t0+nt).
WORKLOADS = {
    "16x4^3": dict(T=16, L=4, eps=0.3, kappa=0.125, bc=-1, link_seed=101,
                   sources=[(0, 0, 0, 0)], domains=[(0, 8), (8, 8)], tol=1e-12),
    "32x16^3": dict(T=32, L=16, eps=0.2, kappa=0.13, bc=-1, link_seed=201,
                    sources=[(8 * k, 4 * k, 4 * k, 4 * k) for k in range(4)],
                    domains=[(0, 16), (16, 16)], tol=1e-10),
    "64x32^3": dict(T=64, L=32, eps=0.15, kappa=0.135, bc=-1, link_seed=301,
                    sources=[(0, 0, 0, 0)],
                    domains=[(0, 16), (16, 16), (32, 16), (48, 16)], tol=1e-10,
                    stencil_seed=302),
    "force-32x16^3": dict(T=32, L=16, eps=0.2, kappa=0.13, bc=0, link_seed=501,
                          phi_seed=502, fd_seed=503, tol=1e-10),
}

BATCH_SHAPES = [(8, 8), (8, 12), (16, 8), (16, 16)]  # (T_i, L_i)


def batched_domains(n: int = 96):
    """The uneven batch of independent Dirichlet domains.

    Shape i is drawn uniformly from BATCH_SHAPES with ``rng(401).integers``,
    kappa_i uniformly from [0.125, 0.135] with ``rng(402)``; each domain has
    its own links (eps = 0.2, seed 41000 + i), time Dirichlet walls, periodic
    space, and a point source at (T_i/2, 0, 0, 0).
    """
    shapes = np.random.default_rng(401).integers(0, 4, n)
    kappas = np.random.default_rng(402).uniform(0.125, 0.135, n)
    out = []
    for i in range(n):
        T, L = BATCH_SHAPES[int(shapes[i])]
        out.append(dict(T=T, L=L, eps=0.2, kappa=float(kappas[i]), bc=0,
                        link_seed=41000 + i, source=(T // 2, 0, 0, 0)))
    return out
