"""Pins of the oracle's factorised nucleon contraction (Sec. 4.2, Eqs. 22-26).

- C = gamma_0 gamma_2 is a charge conjugation (C gamma_mu C^-1 = -gamma_mu^T), C gamma5 is
  antisymmetric, the spin matrix between the blocks, P_+ = (1 + gamma_0)/2, is a projector.
- The spin matrix is the one of a nucleon propagating forward in time: in the free field at
  small kappa the factorised correlator with P_+ is non-zero and falls by about (2 kappa)^3
  per time slice (three quark lines, each (2 kappa) per hop), while with P_- it is zero to
  rounding, and so is the text's gamma5 P_- (and gamma5 P_+) in this basis.
- The blocks of Eq. 25 are symmetric in their first two quark fields (from the antisymmetry of
  C gamma5 and of eps), colour singlets (unchanged by an SU(3) rotation at every site) and
  transform as spinors under a Euclidean spin rotation S = exp(theta gamma_mu gamma_nu / 2).
- Substituting the projected factorised propagator S_f(y, x) = -sum_i eta_i(y) xi_i^T(x)
  (Eqs. 17, 26) into Eqs. 23-24 turns the block contraction into three-propagator
  contractions at each site pair:
    W1 = eps^{abc} eps^{a'b'c'} (C g5)_{gd} (C g5)_{g'd'} M_{lm} S^{a'b}_{g'd} S^{b'a}_{d'g} S^{c'c}_{ml}
    W2 = eps^{abc} eps^{a'b'c'} (C g5)_{gd} (C g5)_{g'd'} M_{lm} S^{a'b}_{g'd} S^{b'c}_{d'l} S^{c'a}_{mg}
  (M = P_+).  Evaluated with S_f from the oracle's projected factorised propagator (its
  own pins tie it to dense block products) from point sources at every site of the source
  slice, they must equal the O(N_m^3) block path built from xi and eta.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import oracle as O
from paper_1612_06424_amd.inputs import gaussian_field, random_links

EPS = np.zeros((3, 3, 3))
for _a, _b, _c in ((0, 1, 2), (1, 2, 0), (2, 0, 1)):
    EPS[_a, _b, _c], EPS[_b, _a, _c] = 1.0, -1.0


def test_charge_conjugation_and_projector():
    g = O.gamma_matrices()
    C = O.charge_conjugation()
    for mu in range(4):
        assert np.abs(C @ g[mu] @ np.linalg.inv(C) + g[mu].T).max() < 1e-14
    cg5 = C @ g[4]
    assert np.abs(cg5.T + cg5).max() < 1e-14
    P = O.nucleon_parity_projector()
    assert np.abs(P @ P - P).max() < 1e-14 and abs(np.trace(P) - 2) < 1e-14
    assert np.abs(g[0] @ P - P).max() < 1e-14  # the range of (1 + gamma_0)/2


def test_block_symmetry_colour_singlet_spin_covariance():
    L, n, nt = 2, 4, 3
    s = gaussian_field(nt * L ** 3, n, 61)
    B = O.baryon_blocks(L, s)
    assert B.shape == (nt, n, n, n, 4)
    assert np.abs(B).max() > 1e-3
    assert np.abs(B - B.transpose(0, 2, 1, 3, 4)).max() < 1e-13
    # not symmetric in the last two
    assert np.abs(B - B.transpose(0, 1, 3, 2, 4)).max() > 1e-3
    # an SU(3) rotation at every site leaves the colour singlet unchanged
    g = random_links(nt, L, 1.0, 62)[:, 0]                      # (sites, 3, 3) SU(3)
    q = s.reshape(n, nt * L ** 3, 4, 3)
    s_rot = np.einsum("xab,ixsb->ixsa", g, q).reshape(s.shape)
    assert np.abs(O.baryon_blocks(L, s_rot) - B).max() < 1e-12 * np.abs(B).max()
    # a Euclidean spin rotation acts on the free spinor index
    gm = O.gamma_matrices()
    for mu, nu, th in ((0, 1, 0.7), (2, 3, -1.1), (1, 3, 0.4)):
        S = sla.expm(0.5 * th * gm[mu] @ gm[nu])
        s_sp = np.einsum("rs,ixsa->ixra", S, q).reshape(s.shape)
        B_sp = O.baryon_blocks(L, s_sp)
        assert np.abs(B_sp - np.einsum("pq,tijkq->tijkp", S, B)).max() < 1e-12 * np.abs(B).max()


@pytest.mark.parametrize("nvec", [5, 12])
def test_blocks_equal_the_three_propagator_contraction(nvec):
    T, L, bc, kappa = 8, 2, 0, 0.13
    L3 = L ** 3
    U = random_links(T, L, 0.5, 63)
    doms, dlt = [(0, 4), (4, 4)], 1
    gbar, gstar, t_phi, x0 = (0, 5), (4, 4), 3, 1
    v0 = gaussian_field(4 * L3, nvec, 64)
    phi, _ = O.projection_basis(U, kappa, T, L, bc, (2, 4), t_phi, +1, v0, 3, tol=1e-13)
    xi, eta = O.nucleon_lines(U, kappa, T, L, bc, gbar, gstar, t_phi, phi, x0, tol=1e-13)
    Bx = O.baryon_blocks(L, xi)
    By = O.baryon_blocks(L, eta)
    W1, W2, Cf = O.nucleon_factorized(L, Bx, By)
    assert W1.shape == (4, 1)
    # the same from the projected factorised propagator, sources at every site of slice x0
    cg5 = O.charge_conjugation() @ O.gamma_matrices()[4]
    M = O.nucleon_parity_projector()
    P1 = np.zeros(4, dtype=complex)
    P2 = np.zeros(4, dtype=complex)
    for sp in range(L3):
        x, y, z = sp % L, (sp // L) % L, sp // (L * L)
        S, _ = O.factorized_propagator(U, kappa, T, L, bc, (x0, x, y, z), doms, tol=1e-13, overlap=dlt,
                                       projections={t_phi: phi})
        # P[site, row spin, row colour, col spin, col colour] on Gstar
        P = O.slab_extract(T, L, S, gstar).reshape(4, 3, 4 * L3, 4, 3).transpose(2, 3, 4, 0, 1)
        w1 = np.einsum("abc,ABC,gd,GD,lm,yGAdb,yDBga,ymClc->y", EPS, EPS, cg5, cg5, M, P, P, P, optimize=True)
        w2 = np.einsum("abc,ABC,gd,GD,lm,yGAdb,yDBlc,ymCga->y", EPS, EPS, cg5, cg5, M, P, P, P, optimize=True)
        P1 += w1.reshape(4, L3).sum(axis=1)
        P2 += w2.reshape(4, L3).sum(axis=1)
    scale = np.abs(P1).max()
    assert scale > 1e-12
    assert np.abs(W1[:, 0] - P1).max() < 1e-9 * scale
    assert np.abs(W2[:, 0] - P2).max() < 1e-9 * np.abs(P2).max()
    assert np.abs(Cf[:, 0] - (P1 - P2) / L3).max() < 1e-9 * scale / L3


def _free_chain_blocks(kappa):
    """Blocks of the xi and eta lines in the free field (U = 1) on a 16 x 2^3 lattice with
    Dirichlet time walls: Gbar = [0, 8), Gstar = [7, 16), lines cut on t_phi = 6, source
    slice x0 = 2, 12 vectors from 2 inverse iterations on [4, 8)."""
    T, L, bc = 16, 2, 0
    U = np.zeros((T * L ** 3, 4, 3, 3), dtype=complex)
    U[:] = np.eye(3)
    v0 = gaussian_field(4 * L ** 3, 12, 64)
    phi, _ = O.projection_basis(U, kappa, T, L, bc, (4, 4), 6, +1, v0, 2, tol=1e-14)
    xi, eta = O.nucleon_lines(U, kappa, T, L, bc, (0, 8), (7, 9), 6, phi, 2, tol=1e-14)
    return L, O.baryon_blocks(L, xi), O.baryon_blocks(L, eta)


def _contract(L, Bx, By, M):
    W1 = -np.einsum("xjika,ab,yijkb->yx", Bx, M, By, optimize=True)
    W2 = -np.einsum("xkija,ab,yijkb->yx", Bx, M, By, optimize=True)
    return ((W1 - W2) / L ** 3)[:, 0]


@pytest.mark.parametrize("kappa", [0.02, 0.05])
def test_free_field_nucleon_propagates_forward_with_the_chosen_projector(kappa):
    L, Bx, By = _free_chain_blocks(kappa)
    _, _, Cf = O.nucleon_factorized(L, Bx, By)
    g = O.gamma_matrices()
    scale = np.abs(Cf).max()
    assert scale > 0 and np.all(np.abs(Cf) > 0)
    # three quark lines, one power of 2 kappa per hop each: (2 kappa)^3 per slice at small kappa
    ratio = np.abs(Cf[1:] / Cf[:-1])
    assert np.all(ratio > 0.5 * (2 * kappa) ** 3) and np.all(ratio < 4 * (2 * kappa) ** 3), ratio
    # the other parity projector, and the text's gamma5 P_-+, vanish at leading order
    for M in (0.5 * (np.eye(4) - g[0]), g[4] @ (0.5 * (np.eye(4) - g[0])), g[4] @ (0.5 * (np.eye(4) + g[0]))):
        assert np.abs(_contract(L, Bx, By, M)).max() < 1e-12 * scale
