"""Pin of the oracle's link force against central finite differences.

S(U) = phi^dagger (D_L^dagger D_L)^-1 phi with U_mu(x) -> exp(i w T^a) U_mu(x) (T^a = lambda^a/2).
S(+d) - S(-d) is evaluated through the cancellation-free identity
    S+ - S- = (D- X+)^dagger (dD X-) + (dD X+)^dagger (D+ X-),  dD = D- - D+,
(X = (D^dagger D)^-1 phi at the two link values), which only involves the two sites
the perturbed link touches, so neither the size of S nor solver error is amplified.
Links outside the slab or crossing its Dirichlet walls must have exactly zero force.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import oracle as O
from paper_1612_06424_amd.inputs import random_links, gaussian_field


def fd_force(U, kappa, T, L, bc, dom, phi, site, mu, a, delta=1e-5):
    Tg = O.su3_generators()
    Up, Um = U.copy(), U.copy()
    Up[site, mu] = sla.expm(1j * delta * Tg[a]) @ U[site, mu]
    Um[site, mu] = sla.expm(-1j * delta * Tg[a]) @ U[site, mu]
    _, Xp, _ = O.domain_action(Up, kappa, T, L, bc, dom, phi)
    _, Xm, _ = O.domain_action(Um, kappa, T, L, bc, dom, phi)
    DmXp = O.apply_dirac(Um, kappa, T, L, bc, Xp, dom)
    DpXm = O.apply_dirac(Up, kappa, T, L, bc, Xm, dom)
    dDXm = O.apply_dirac(Um, kappa, T, L, bc, Xm, dom) - DpXm
    dDXp = O.apply_dirac(Um, kappa, T, L, bc, Xp, dom) - O.apply_dirac(Up, kappa, T, L, bc, Xp, dom)
    diff = np.vdot(DmXp, dDXm) + np.vdot(dDXp, DpXm)
    return diff.real / (2 * delta)


@pytest.mark.parametrize("bc,dom", [(0, None), (-1, (5, 5))])
def test_force_vs_finite_differences(bc, dom):
    T, L, kappa = 8, 2, 0.13
    U = random_links(T, L, 0.5, 91)
    t0, nt = (0, T) if dom is None else dom
    phi = gaussian_field(nt * L ** 3, 1, 92)[0]
    S, X, Y = O.domain_action(U, kappa, T, L, bc, dom, phi)
    g = O.link_grad(T, L, bc, dom, X, Y, coeff=1.0)
    F = O.su3_force(U, g)
    rng = np.random.default_rng(93)
    L3 = L ** 3
    checked_nonzero = 0
    # random links plus the time link across the time edge (t = T-1 -> 0)
    picks = [(int(rng.integers(0, T * L3)), int(rng.integers(0, 4))) for _ in range(5)]
    picks.append(((T - 1) * L3 + 3, 0))
    for site, mu in picks:
        t = site // L3
        inside = (t - t0) % T < nt
        fwd_inside = ((t + (1 if mu == 0 else 0)) - t0) % T < nt
        edge_dropped = mu == 0 and t == T - 1 and bc == 0
        for a in range(8):
            fd = fd_force(U, kappa, T, L, bc, dom, phi, site, mu, a)
            if not (inside and fwd_inside) or edge_dropped:
                assert F[site, mu, a] == 0.0
                assert abs(fd) < 1e-12
            else:
                assert abs(F[site, mu, a] - fd) <= 1e-7 * max(1.0, abs(fd)), (site, mu, a)
                checked_nonzero += abs(fd) > 1e-6
    assert checked_nonzero > 0


def test_force_zero_across_walls_and_outside():
    T, L, kappa, bc = 8, 2, 0.13, -1
    U = random_links(T, L, 0.5, 94)
    dom = (2, 4)  # slab [2, 6)
    phi = gaussian_field(4 * L ** 3, 1, 95)[0]
    _, X, Y = O.domain_action(U, kappa, T, L, bc, dom, phi)
    g = O.link_grad(T, L, bc, dom, X, Y).reshape(T, L ** 3, 4, 3, 3)
    for t in range(T):
        for mu in range(4):
            inside = 2 <= t < 6 and (mu > 0 or t + 1 < 6)
            nz = np.abs(g[t, :, mu]).max()
            assert (nz > 0) == inside, (t, mu)


def test_phi_gradient_is_2X():
    """d S / d conj(phi) convention: dS = 2 Re <X, d phi> for S = phi^dagger (D^dagger D)^-1 phi."""
    T, L, kappa, bc = 4, 2, 0.13, 0
    U = random_links(T, L, 0.5, 96)
    phi = gaussian_field(T * L ** 3, 1, 97)[0]
    S0, X, _ = O.domain_action(U, kappa, T, L, bc, None, phi)
    rng = np.random.default_rng(98)
    dphi = (rng.standard_normal(phi.shape) + 1j * rng.standard_normal(phi.shape)) * 1e-6
    Sp, *_ = O.domain_action(U, kappa, T, L, bc, None, phi + dphi)
    Sm, *_ = O.domain_action(U, kappa, T, L, bc, None, phi - dphi)
    assert abs((Sp - Sm) / 2 - np.vdot(2 * X, dphi).real) <= 1e-6 * abs(np.vdot(2 * X, dphi).real)
