"""Pins of the oracle's solves, block inverses, factorised propagator and correlator.

- BiCGStab and CGNR against LU (scipy) of the dense matrix of D, D_Lambda;
- the free-field point-to-all propagator against its momentum-space closed form
  S(x,0) = (1/V) sum_p e^{ipx} (M(p) - i gamma.sin p) / (M(p)^2 + sum_mu sin^2 p_mu);
- the exact block inverse through Schur complements (Sec. 3, Eqs. 10-11), the Woodbury
  form of the first case (Eq. 13) and the exact first equality of the second case (Eq. 14);
- the factorised chain against dense block products, and the identity that feeding the
  exact propagator into the frontier hop reproduces the exact propagator;
- overlap regions (Delta > 0): the chain against dense block products, the form of the
  correction (Eq. 15) and its fall-off with Delta;
- the pion correlator (Eq. 4): free-field closed form, time-reflection symmetry,
  positivity and invariance under a random gauge transformation.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import oracle as O
from paper_1612_06424_amd.inputs import random_links, point_sources, gaussian_field


def dense_block(U, kappa, T, L, bc, dst, src):
    """Matrix of P_dst D P_src, built column by column from unit vectors."""
    ns = (T if src is None else src[1]) * L ** 3 * 12
    E = np.eye(ns, dtype=complex).reshape(ns, ns // 12, 12)
    cols = O.block_apply(U, kappa, T, L, bc, dst, src, E)
    return cols.reshape(ns, -1).T


@pytest.mark.parametrize("bc,dom", [(-1, None), (-1, (2, 3)), (0, None), (1, (6, 4))])
@pytest.mark.parametrize("method", [0, 1])
def test_solver_vs_lu(bc, dom, method):
    T, L, kappa = 8, 2, 0.15
    U = random_links(T, L, 0.6, 41)
    A = dense_block(U, kappa, T, L, bc, dom, dom)
    n = A.shape[0]
    b = gaussian_field(n // 12, 3, 42)
    x, it, rr, st = O.solve(U, kappa, T, L, bc, b, dom=dom, tol=1e-13, method=method, maxit=3000)
    assert st == 0 and max(rr) <= 1e-13
    ref = sla.lu_solve(sla.lu_factor(A), b.reshape(3, n).T).T.reshape(b.shape)
    assert np.linalg.norm(x - ref) <= 1e-11 * np.linalg.norm(ref)


def free_propagator(T, L, kappa, bc):
    """Closed-form free point-to-all propagator from the origin, shape (12, V, 12)."""
    g = [-np.kron(np.array([[0, 1], [1, 0]]), np.eye(2))]
    S2 = np.array([[0, -1j], [1j, 0]])
    for s in (np.array([[0, 1], [1, 0]]), S2, np.array([[1, 0], [0, -1]])):
        g.append(np.kron(S2, s))
    p0 = (2 * np.arange(T) + (1 if bc == -1 else 0)) * np.pi / T
    pk = 2 * np.pi * np.arange(L) / L
    P = np.meshgrid(p0, pk, pk, pk, indexing="ij")  # order (t, z, y, x) below
    pt, pz, py, px = P[0], P[1], P[2], P[3]
    mom = [pt, px, py, pz]
    M = 1 / (2 * kappa) - sum(np.cos(q) for q in mom)
    den = M ** 2 + sum(np.sin(q) ** 2 for q in mom)
    Sp = M[..., None, None] * np.eye(4) - 1j * sum(np.sin(mom[m])[..., None, None] * g[m] for m in range(4))
    Sp = Sp / den[..., None, None]
    # x-space: (1/V) sum_p e^{ipx} S(p); time momenta shifted by pi/T for antiperiodic bc
    t = np.arange(T)
    shift = np.exp(1j * np.pi * t / T) if bc == -1 else np.ones(T)
    # numpy ifft computes (1/N) sum_k e^{+2 pi i k n / N} a_k on the unshifted grid
    Sx = np.fft.ifftn(Sp, axes=(0, 1, 2, 3)) * shift[:, None, None, None, None, None]
    Sx = Sx.reshape(T * L ** 3, 4, 4)  # (site, sink spin, source spin)
    out = np.zeros((12, T * L ** 3, 12), dtype=complex)
    for a in range(4):
        for b in range(4):
            for col in range(3):
                out[3 * b + col, :, 3 * a + col] = Sx[:, a, b]
    return out


@pytest.mark.parametrize("bc", [-1, 1])
def test_free_propagator_closed_form(bc):
    T, L, kappa = 16, 4, 0.125
    V = T * L ** 3
    U = np.broadcast_to(np.eye(3, dtype=complex), (V, 4, 3, 3)).copy()
    if bc == 1:
        kappa = 0.12  # keeps the periodic zero-momentum mode away from zero
    S, info = O.exact_propagator(U, kappa, T, L, bc, (0, 0, 0, 0), tol=1e-13)
    ref = free_propagator(T, L, kappa, bc)
    assert np.linalg.norm(S - ref) <= 1e-11 * np.linalg.norm(ref)
    C = O.pion_correlator(T, L, S, 0)
    Cref = np.array([np.sum(np.abs(ref.reshape(12, T, -1, 12)[:, t]) ** 2) for t in range(T)])
    assert np.allclose(C, Cref, rtol=1e-10, atol=0)
    # time reflection t -> T - t maps the free correlator onto itself
    assert np.allclose(C[1:], C[1:][::-1], rtol=1e-10)
    assert np.all(C > 0)


def test_block_inverse_schur_and_factorisation_identities():
    T, L, kappa, bc = 8, 2, 0.14, -1
    U = random_links(T, L, 0.5, 51)
    G, Gs = (0, 5), (5, 3)  # Gamma = [0,5), Gamma* = [5,8)
    DG = dense_block(U, kappa, T, L, bc, G, G)
    DGs = dense_block(U, kappa, T, L, bc, Gs, Gs)
    DdG = dense_block(U, kappa, T, L, bc, G, Gs)    # D_{dGamma}: Gamma* -> Gamma
    DdGs = dense_block(U, kappa, T, L, bc, Gs, G)   # D_{dGamma*}: Gamma -> Gamma*
    D = dense_block(U, kappa, T, L, bc, None, None)
    n0 = DG.shape[0]
    assert np.allclose(D[:n0, :n0], DG) and np.allclose(D[n0:, n0:], DGs)
    assert np.allclose(D[:n0, n0:], DdG) and np.allclose(D[n0:, :n0], DdGs)
    Dinv = np.linalg.inv(D)
    inv = np.linalg.inv
    SG = DG - DdG @ inv(DGs) @ DdGs            # Schur complements, Eq. 11
    SGs = DGs - DdGs @ inv(DG) @ DdG
    tol = 1e-11 * np.abs(Dinv).max()
    assert np.abs(Dinv[:n0, :n0] - inv(SG)).max() < tol        # Eq. 10
    assert np.abs(Dinv[n0:, n0:] - inv(SGs)).max() < tol
    assert np.abs(Dinv[:n0, n0:] + inv(DG) @ DdG @ inv(SGs)).max() < tol
    assert np.abs(Dinv[n0:, :n0] + inv(DGs) @ DdGs @ inv(SG)).max() < tol
    # first case (Eq. 13): Woodbury form
    wood = inv(DG) + inv(DG) @ DdG @ inv(SGs) @ DdGs @ inv(DG)
    assert np.abs(Dinv[:n0, :n0] - wood).max() < tol
    # second case (Eq. 14), exact first equality
    assert np.abs(Dinv[n0:, :n0] + inv(DGs) @ DdGs @ inv(SG)).max() < tol


@pytest.mark.parametrize("domains", [[(0, 4), (4, 4)], [(0, 2), (2, 2), (4, 2), (6, 2)],
                                     [(6, 3), (1, 3), (4, 2)]])
@pytest.mark.parametrize("bc", [-1, 0])
def test_factorised_chain_vs_dense(domains, bc):
    """The factorised chain over several slabs (Eqs. 13-14 chained outward by block
    distance) against dense block products, including a ring of four slabs."""
    T, L, kappa = 8, 2, 0.14
    if bc == 0 and domains[0][0] != 0:
        pytest.skip("open time edge: slabs must start at 0 for a chain")
    U = random_links(T, L, 0.5, 61)
    t0 = domains[0][0]
    src = (t0, 1, 0, 1)
    S, info = O.factorized_propagator(U, kappa, T, L, bc, src, domains, tol=1e-13)
    dist = O.domain_distances(T, bc, domains)
    eta = point_sources(T, L, *src)
    blk = {(a, b): dense_block(U, kappa, T, L, bc, domains[a], domains[b])
           for a in range(len(domains)) for b in range(len(domains))}
    psi = {}
    for k in sorted(range(len(domains)), key=lambda k: dist[k]):
        if dist[k] == 0:
            rhs = O.slab_extract(T, L, eta, domains[k]).reshape(12, -1).T
        else:
            rhs = -sum(blk[(k, j)] @ psi[j] for j in range(len(domains)) if dist[j] == dist[k] - 1)
        psi[k] = np.linalg.solve(blk[(k, k)], rhs)
    for k, dk in enumerate(domains):
        got = O.slab_extract(T, L, S, dk).reshape(12, -1).T
        assert np.linalg.norm(got - psi[k]) <= 1e-11 * np.linalg.norm(psi[k])


@pytest.mark.parametrize("domains,overlap", [([(0, 6), (6, 6)], 1), ([(0, 6), (6, 6)], 2),
                                             ([(0, 3), (3, 3), (6, 3), (9, 3)], 2),
                                             ([(10, 4), (2, 5), (7, 3)], 1)])
@pytest.mark.parametrize("bc", [-1, 0])
def test_factorised_overlap_vs_dense(domains, overlap, bc):
    """The chain with overlap regions against dense block products: every domain
    that feeds a frontier hop is solved on its extension (Delta slices on both
    time sides, P D P of the grown slab) and only the part on the domain crosses
    the frontier; S_fact on each domain stays the unextended solve."""
    T, L, kappa = 12, 2, 0.14
    if bc == 0 and domains[0][0] != 0:
        pytest.skip("open time edge: slabs must start at 0 for a chain")
    U = random_links(T, L, 0.5, 62)
    src = (domains[0][0] + 1, 1, 0, 1)
    S, info = O.factorized_propagator(U, kappa, T, L, bc, src, domains, tol=1e-13, overlap=overlap)
    dist = O.domain_distances(T, bc, domains)
    eta = point_sources(T, L, *src)
    n = len(domains)
    blk = {(a, b): dense_block(U, kappa, T, L, bc, domains[a], domains[b]) for a in range(n) for b in range(n)}
    psi, hop = {}, {}
    for k in sorted(range(n), key=lambda k: dist[k]):
        if dist[k] == 0:
            rhs = O.slab_extract(T, L, eta, domains[k]).reshape(12, -1).T
        else:
            rhs = -sum(blk[(k, j)] @ hop[j] for j in range(n) if dist[j] == dist[k] - 1)
        psi[k] = np.linalg.solve(blk[(k, k)], rhs)
        hop[k] = psi[k]
        if any(dist[j] == dist[k] + 1 for j in range(n)):
            ext = ((domains[k][0] - overlap) % T, domains[k][1] + 2 * overlap)
            a, b = overlap * L ** 3 * 12, (overlap + domains[k][1]) * L ** 3 * 12
            rext = np.zeros((ext[1] * L ** 3 * 12, 12), complex)
            rext[a:b] = rhs
            hop[k] = np.linalg.solve(dense_block(U, kappa, T, L, bc, ext, ext), rext)[a:b]
            assert "extended" in info[k]
    for k, dk in enumerate(domains):
        got = O.slab_extract(T, L, S, dk).reshape(12, -1).T
        assert np.linalg.norm(got - psi[k]) <= 1e-11 * np.linalg.norm(psi[k])


def test_overlap_correction_form():
    """Two regions, Delta = 2 (Eqs. 14 and 15, with the indices of Eq. 15 read as
    for x in Gamma, y in Gamma*): on Gamma*, S_exact - S_fact =
    D_Gamma*^-1 D_{Gamma*,Gamma} ([D_Gamma-bar^-1]_{Gamma Gamma} - S_Gamma^-1) eta,
    with S_Gamma^-1 = [D^-1]_{Gamma Gamma} (Eq. 10)."""
    T, L, kappa, bc, dlt = 12, 2, 0.14, -1, 2
    U = random_links(T, L, 0.5, 63)
    G, Gs = (0, 6), (6, 6)
    src = (2, 0, 1, 1)
    Sf, _ = O.factorized_propagator(U, kappa, T, L, bc, src, [G, Gs], tol=1e-13, overlap=dlt)
    Se, _ = O.exact_propagator(U, kappa, T, L, bc, src, tol=1e-13)
    D = dense_block(U, kappa, T, L, bc, None, None)
    n0 = G[1] * L ** 3 * 12
    SG = np.linalg.inv(D)[:n0, :n0]
    Gb = O.extended_domain(T, G, dlt)
    a = dlt * L ** 3 * 12
    DGb = np.linalg.inv(dense_block(U, kappa, T, L, bc, Gb, Gb))[a:a + n0, a:a + n0]
    eta = O.slab_extract(T, L, point_sources(T, L, *src), G).reshape(12, -1).T
    corr = np.linalg.solve(dense_block(U, kappa, T, L, bc, Gs, Gs),
                           dense_block(U, kappa, T, L, bc, Gs, G) @ ((DGb - SG) @ eta))
    got = (O.slab_extract(T, L, Se, Gs) - O.slab_extract(T, L, Sf, Gs)).reshape(12, -1).T
    ref = np.linalg.norm(O.slab_extract(T, L, Se, Gs))
    # both sides carry the solves' rounding, ~1e-13 of the propagator; the correction is ~1e-5 of it
    assert np.linalg.norm(got - corr) <= 1e-11 * ref
    assert np.linalg.norm(corr) > 1e-6 * ref


def test_overlap_correction_shrinks():
    """The correction on Gamma* falls quickly as the overlap grows (Sec. 3.2:
    suppressed like exp(-M_pi Delta / 2)): a heavy quark on 16x4^3, two slabs."""
    T, L, bc, kappa = 16, 4, -1, 0.11
    U = random_links(T, L, 0.3, 91)
    src = (3, 1, 2, 0)
    doms = [(0, 8), (8, 8)]
    Se, _ = O.exact_propagator(U, kappa, T, L, bc, src, tol=1e-13)
    ref = np.linalg.norm(O.slab_extract(T, L, Se, doms[1]))
    err = []
    for dlt in range(3):
        Sf, _ = O.factorized_propagator(U, kappa, T, L, bc, src, doms, tol=1e-13, overlap=dlt)
        err.append(np.linalg.norm(O.slab_extract(T, L, Se - Sf, doms[1])) / ref)
    assert err[0] > 3 * err[1] > 9 * err[2] > 0


def test_exact_propagator_through_frontier_hop():
    """D S_exact = eta restricted to a slab k off the source: S_k = -D_k^-1 sum_j D_kj S_j."""
    T, L, kappa, bc = 16, 2, 0.13, -1
    U = random_links(T, L, 0.4, 71)
    doms = [(0, 6), (6, 5), (11, 5)]
    S, _ = O.exact_propagator(U, kappa, T, L, bc, (1, 0, 1, 0), tol=1e-13)
    for k in (1, 2):
        rhs = np.zeros((12, doms[k][1] * L ** 3, 12), complex)
        for j in range(3):
            if j != k:
                rhs -= O.block_apply(U, kappa, T, L, bc, doms[k], doms[j], O.slab_extract(T, L, S, doms[j]))
        xk, *_ = O.solve(U, kappa, T, L, bc, rhs, dom=doms[k], tol=1e-13)
        ref = O.slab_extract(T, L, S, doms[k])
        assert np.linalg.norm(xk - ref) <= 1e-10 * np.linalg.norm(ref)


def test_correlator_gauge_invariance():
    T, L, kappa, bc = 8, 3, 0.13, -1
    V = T * L ** 3
    U = random_links(T, L, 0.4, 81)
    Om = random_links(T, L, 2.0, 82)[:, 0]
    t, z, y, x = [a.reshape(-1) for a in np.meshgrid(*(np.arange(n) for n in (T, L, L, L)), indexing="ij")]
    ext = [T, L, L, L]
    Ug = np.empty_like(U)
    for mu in range(4):
        cn = [t.copy(), x.copy(), y.copy(), z.copy()]
        cn[mu] = (cn[mu] + 1) % ext[mu]
        sn = ((cn[0] * L + cn[3]) * L + cn[2]) * L + cn[1]
        Ug[:, mu] = Om @ U[:, mu] @ np.conj(np.swapaxes(Om[sn], -1, -2))
    src = (2, 1, 2, 0)
    doms = [(0, 4), (4, 4)]
    S0, _ = O.exact_propagator(U, kappa, T, L, bc, src, tol=1e-13)
    S1, _ = O.exact_propagator(Ug, kappa, T, L, bc, src, tol=1e-13)
    C0 = O.pion_correlator(T, L, S0, src[0])
    C1 = O.pion_correlator(T, L, S1, src[0])
    assert np.allclose(C0, C1, rtol=1e-10)
    F0, _ = O.factorized_propagator(U, kappa, T, L, bc, src, doms, tol=1e-13)
    F1, _ = O.factorized_propagator(Ug, kappa, T, L, bc, src, doms, tol=1e-13)
    Cf0 = O.pion_correlator(T, L, F0, src[0])
    Cf1 = O.pion_correlator(T, L, F1, src[0])
    assert np.allclose(Cf0, Cf1, rtol=1e-10)
    assert np.all(C0 > 0) and np.all(Cf0 >= 0)
    # on the source slab the factorised term is the Dirichlet propagator, elsewhere the hop
    # chain; both differ from the exact propagator but not wildly for this mass
    assert np.allclose(Cf0[:2], C0[:2], rtol=0.5)


def test_correlator_decays_away_from_source():
    """Locality (Eq. 12): with the time edge closed (bc = 0) the correlator falls
    monotonically with the sink distance t = y0 - x0 >= 0 from a source at x0 = 2."""
    T, L, kappa, bc = 12, 2, 0.12, 0
    U = random_links(T, L, 0.3, 99)
    ts = 2
    S, _ = O.exact_propagator(U, kappa, T, L, bc, (ts, 0, 0, 0), tol=1e-13)
    C = O.pion_correlator(T, L, S, ts)
    fwd = C[: T - ts]
    assert np.all(np.diff(fwd) < 0)
    # beyond the closed edge the sink comes back towards the source
    assert C[T - 1] > C[T - ts]
