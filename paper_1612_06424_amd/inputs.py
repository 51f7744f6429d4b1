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


def random_links(T: int, L: int, eps: float, seed: int) -> np.ndarray:
    """U = exp(i eps H) per link, H traceless Hermitian with Gaussian entries.

    Normalisation: H_ii ~ N(0,1); for i < j, H_ij = a + i b with a, b ~ N(0,1)
    and H_ji = conj(H_ij); then H <- H - tr(H)/3, so E tr H^2 = 14.  The nine
    reals per link come from numpy PCG64 ``standard_normal((T,L,L,L,4,9))`` in
    the order (H00, H11, H22, Re H01, Im H01, Re H02, Im H02, Re H12, Im H12).
    The exponential is exact through the eigen-decomposition of H (no
    re-unitarisation is needed: tr H = 0 gives det U = 1).
    """
    rng = np.random.default_rng(seed)
    V = T * L * L * L
    out = np.empty((V, 4, 3, 3), dtype=np.complex128)
    # chunked to bound host memory on large lattices
    chunk = 1 << 18
    g_all = rng.standard_normal((T, L, L, L, 4, 9)).reshape(V, 4, 9)
    for lo in range(0, V, chunk):
        g = g_all[lo:lo + chunk]
        n = g.shape[0]
        H = np.zeros((n, 4, 3, 3), dtype=np.complex128)
        H[..., 0, 0] = g[..., 0]
        H[..., 1, 1] = g[..., 1]
        H[..., 2, 2] = g[..., 2]
        H[..., 0, 1] = g[..., 3] + 1j * g[..., 4]
        H[..., 0, 2] = g[..., 5] + 1j * g[..., 6]
        H[..., 1, 2] = g[..., 7] + 1j * g[..., 8]
        H[..., 1, 0] = np.conj(H[..., 0, 1])
        H[..., 2, 0] = np.conj(H[..., 0, 2])
        H[..., 2, 1] = np.conj(H[..., 1, 2])
        tr = (g[..., 0] + g[..., 1] + g[..., 2]) / 3.0
        for a in range(3):
            H[..., a, a] -= tr
        w, vec = np.linalg.eigh(H)
        ph = np.exp(1j * eps * w)
        out[lo:lo + n] = np.einsum("...ak,...k,...bk->...ab", vec, ph, np.conj(vec))
    return out


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
