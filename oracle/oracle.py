"""Python face of the FP64 CPU oracle (test infrastructure only).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark
import this module.  It loads ``liboracle.so`` built from ``dd_oracle.c`` in
this directory and never touches the HIP library.

Every array here uses the natural layout:
  links  complex128 (V, 4, 3, 3)
  fields complex128 (ncol, nsite, 12), nsite = nt * L^3 on a slab [t0, t0+nt)
         (local site index ((t - t0) mod T) * L^3 + spatial index)
  propagators: 12 columns, S[j, s, c] = D^-1(s, x_src)_{c j}
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from collections import deque

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SRC_PATH = os.path.join(HERE, "dd_oracle.c")

_c = ctypes
_dp = _c.POINTER(_c.c_double)
_ip = _c.POINTER(_c.c_int)


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (C11, OpenMP, no fast-math)."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, SRC_PATH, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def _configure(L):
    L.ora_threads.argtypes = []
    L.ora_threads.restype = _c.c_int
    L.ora_gamma.argtypes = [_c.c_void_p]
    L.ora_block_apply.argtypes = [_c.c_int, _c.c_int, _c.c_int, _c.c_void_p, _c.c_double,
                                  _c.c_int, _c.c_int, _c.c_int, _c.c_int,
                                  _c.c_void_p, _c.c_void_p]
    L.ora_gamma5.argtypes = [_c.c_long, _c.c_void_p, _c.c_void_p]
    L.ora_solve.argtypes = [_c.c_int, _c.c_int, _c.c_int, _c.c_void_p, _c.c_double,
                            _c.c_int, _c.c_int, _c.c_int, _c.c_void_p, _c.c_void_p,
                            _c.c_double, _c.c_int, _c.c_int, _ip, _dp]
    L.ora_solve.restype = _c.c_int
    L.ora_pion.argtypes = [_c.c_int, _c.c_int, _c.c_int, _c.c_void_p, _c.c_int, _dp]
    L.ora_link_grad.argtypes = [_c.c_int, _c.c_int, _c.c_int, _c.c_int, _c.c_int, _c.c_int,
                                _c.c_void_p, _c.c_void_p, _c.c_double, _c.c_void_p]
    return L


def lib():
    global _lib
    if _lib is None:
        build()
        _lib = _configure(_c.CDLL(LIB_PATH))
    return _lib


def use_library(path):
    """Point this module at another build of the oracle (the mutation tests use
    this to check that planted mistakes are caught).  Returns the previous one."""
    global _lib
    prev = lib()
    _lib = _configure(_c.CDLL(path))
    return prev


def restore_library(prev):
    global _lib
    _lib = prev


def _ptr(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"] and a.dtype == np.complex128, (a.dtype, a.flags)
    return a.ctypes.data_as(_c.c_void_p)


def _links(U: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(U, dtype=np.complex128)


def gamma_matrices() -> np.ndarray:
    """(5, 4, 4): gamma_0..gamma_3 and gamma_5 of the oracle's chiral basis."""
    g = np.zeros((5, 4, 4), dtype=np.complex128)
    lib().ora_gamma(_ptr(g))
    return g


def _norm_dom(T: int, dom):
    return (0, T) if dom is None else (int(dom[0]) % T, int(dom[1]))


def block_apply(U, kappa, T, L, bc, dst, src, psi):
    """P_dst D P_src psi for slabs dst, src ((t0, nt) or None = whole lattice).

    psi: (ncol, nsrc, 12) or (nsrc, 12).  Returns the same rank on dst.
    """
    U = _links(U)
    dt0, dnt = _norm_dom(T, dst)
    st0, snt = _norm_dom(T, src)
    L3 = L ** 3
    one = psi.ndim == 2
    p = np.ascontiguousarray(psi.reshape(-1, snt * L3, 12), dtype=np.complex128)
    out = np.empty((p.shape[0], dnt * L3, 12), dtype=np.complex128)
    for j in range(p.shape[0]):
        lib().ora_block_apply(T, L, bc, _ptr(U), float(kappa), dt0, dnt, st0, snt,
                              _ptr(p[j]), _ptr(out[j]))
    return out[0] if one else out


def threads() -> int:
    """Host threads the oracle's parallel loops use."""
    return int(lib().ora_threads())


def apply_dirac(U, kappa, T, L, bc, psi, dom=None):
    """D psi on the whole lattice (dom None) or D_Lambda psi on the slab dom."""
    return block_apply(U, kappa, T, L, bc, dom, dom, psi)


def gamma5(psi: np.ndarray) -> np.ndarray:
    p = np.ascontiguousarray(psi, dtype=np.complex128)
    out = np.empty_like(p)
    lib().ora_gamma5(p.size // 12, _ptr(p), _ptr(out))
    return out


def solve(U, kappa, T, L, bc, b, dom=None, tol=1e-12, maxit=100000, method=0):
    """x = D_Lambda^-1 b column by column.  Returns (x, iters, relres, status).

    method 0 = BiCGStab, 1 = CGNR.
    """
    U = _links(U)
    t0, nt = _norm_dom(T, dom)
    L3 = L ** 3
    one = b.ndim == 2
    bb = np.ascontiguousarray(b.reshape(-1, nt * L3, 12), dtype=np.complex128)
    x = np.zeros_like(bb)
    ncol = bb.shape[0]
    it = (_c.c_int * ncol)()
    rr = (_c.c_double * ncol)()
    st = lib().ora_solve(T, L, bc, _ptr(U), float(kappa), t0, nt, ncol, _ptr(bb), _ptr(x),
                         float(tol), int(maxit), int(method), it, rr)
    return (x[0] if one else x), list(it), list(rr), st


def slab_extract(T, L, field, dom):
    """Restrict whole-lattice field(s) (..., V, 12) to the slab dom (compact)."""
    t0, nt = _norm_dom(T, dom)
    L3 = L ** 3
    f = field.reshape(field.shape[:-2] + (T, L3, 12))
    ts = [(t0 + k) % T for k in range(nt)]
    return f[..., ts, :, :].reshape(field.shape[:-2] + (nt * L3, 12))


def slab_insert(T, L, field, dom, part):
    """Write the compact slab field part into the whole-lattice field (in place)."""
    t0, nt = _norm_dom(T, dom)
    L3 = L ** 3
    f = field.reshape(field.shape[:-2] + (T, L3, 12))
    p = part.reshape(part.shape[:-2] + (nt, L3, 12))
    for k in range(nt):
        f[..., (t0 + k) % T, :, :] = p[..., k, :, :]


def domain_distances(T, bc, domains):
    """Block distances of the slabs from slab 0 on the graph of non-zero D blocks.

    Two slabs are adjacent when a time hop of D joins them: consecutive slabs,
    and the last and first one across the time edge unless bc == 0.
    """
    n = len(domains)
    adj = [set() for _ in range(n)]
    for a in range(n):
        ta0, tan = domains[a]
        end = (ta0 + tan) % T  # first slice after slab a
        for b in range(n):
            if b != a and domains[b][0] % T == end:
                if bc == 0 and ta0 + tan >= T:
                    continue  # the hop across the time edge is absent
                adj[a].add(b)
                adj[b].add(a)
    d = [None] * n
    d[0] = 0
    q = deque([0])
    while q:
        a = q.popleft()
        for b in adj[a]:
            if d[b] is None:
                d[b] = d[a] + 1
                q.append(b)
    return d


def orthonormalize(V):
    """An orthonormal basis of the span of the fields V (n, ...): the Q factor of the
    QR factorisation (numpy) of V flattened to n columns, reshaped like V."""
    n = V.shape[0]
    Q, _ = np.linalg.qr(np.asarray(V, dtype=np.complex128).reshape(n, -1).T)
    return np.ascontiguousarray(Q.T).reshape(V.shape)


def hop_spin_projector(sign):
    """(1 + sign gamma_0) / 2 on the 12 (spin, colour) components, c = 3 spin + colour:
    the spin projection that the time hop leaving a slice forward (sign = +1, towards
    t + 1) or backward (sign = -1) applies to the field on that slice (Sec. 5, D_w)."""
    g0 = gamma_matrices()[0]
    return np.kron((np.eye(4) + sign * g0) / 2, np.eye(3))


def projection_basis(U, kappa, T, L, bc, pi_dom, t_slice, sign, v0, n_iter, tol=1e-12, method=0):
    """Quark-line projection vectors (Sec. 3.3) for the frontier hop that leaves time
    slice t_slice forward (sign = +1) or backward (-1), N_m = len(v0):
      inverse iteration of the Wilson-Dirac operator of the slab pi_dom around the
      frontier, V <- orthonormalize(D_Pi^-1 V), n_iter times from orthonormalize(v0)
      (v0: N_m fields on pi_dom), then
      phi = orthonormalize((1 + sign gamma_0)/2 V restricted to t_slice),
    N_m orthonormal vectors on the slice in the range of the hop's spin projector (the
    6 L^3 entries per column that cross the frontier).  Returns (phi (N_m, L^3, 12), V)."""
    U = _links(U)
    L3 = L ** 3
    t0, nt = _norm_dom(T, pi_dom)
    k = (t_slice - t0) % T
    if k >= nt:
        raise ValueError("t_slice outside pi_dom")
    if len(v0) > 6 * L3:
        raise ValueError("more vectors than the 6 L^3 entries of a frontier slice")
    V = orthonormalize(np.asarray(v0, dtype=np.complex128))
    for _ in range(n_iter):
        V, _, _, st = solve(U, kappa, T, L, bc, V, dom=pi_dom, tol=tol, method=method)
        if st != 0:
            raise RuntimeError("inverse iteration solve did not converge")
        V = orthonormalize(V)
    W = V.reshape(len(V), nt, L3, 12)[:, k] @ hop_spin_projector(sign).T
    return orthonormalize(W), V


def _project_slices(T, L, dom, field, projections):
    """field (ncol, |dom|, 12) with every time slice t of dom that is a key of projections
    replaced by P_L field = sum_i phi_i (phi_i^+ field) on that slice (Eq. 16)."""
    if not projections:
        return field
    t0, nt = _norm_dom(T, dom)
    L3 = L ** 3
    out = field.reshape(field.shape[0], nt, L3, 12).copy()
    for t, phi in projections.items():
        k = (t - t0) % T
        if k < nt:
            P = phi.reshape(len(phi), -1)
            x = out[:, k].reshape(field.shape[0], -1)
            out[:, k] = ((x @ P.conj().T) @ P).reshape(field.shape[0], L3, 12)
    return out.reshape(field.shape)


def extended_domain(T, dom, overlap):
    """The slab dom = (t0, nt) grown by `overlap` time slices on both sides (mod T):
    Gamma-bar = Gamma plus the boundary layer of thickness Delta of Sec. 3.2."""
    t0, nt = dom
    return ((t0 - overlap) % T, nt + 2 * overlap)


def factorized_propagator(U, kappa, T, L, bc, src, domains, tol=1e-12, maxit=100000,
                          method=0, eta=None, overlap=0, projections=None):
    """Factorised point-to-all propagator across time-slab domains.

    domains: list of (t0, nt) partitioning [0, T); the source must lie in
    domains[0].  With psi_0 = D_L0^-1 eta (first case, Eq. 13, factorised
    term) and, outward by block distance d,
        psi_k = - D_Lk^-1 sum_{j : d(j) = d(k) - 1} D_{Lk,Lj} h_j
    (second case, Eq. 14, iterated over the chain of regions), the result is
    S_fact = sum_k psi_k.  The field h_j that crosses the frontier is the
    solution of domain j's equation (same source) on its extension Lj-bar =
    Lj grown by `overlap` slices on both time sides, restricted to Lj: for two
    domains h_0 = [D_Gamma-bar^-1 eta] on Gamma, i.e. Eq. 14 with an overlap
    region of thickness Delta = overlap (h_j = psi_j for Delta = 0).  With
    projections = {t: phi} (projection_basis), the quark line is cut at every
    frontier slice t: h_j on slice t is replaced by P_L h_j, P_L = sum_i phi_i
    phi_i^+ (Eqs. 16-17).  Returns (S_fact (12, V, 12), per-domain solve info).
    """
    U = _links(U)
    L3 = L ** 3
    V = T * L3
    if eta is None:
        t, x, y, z = src
        eta = np.zeros((12, V, 12), dtype=np.complex128)
        s = ((t * L + z) * L + y) * L + x
        for j in range(12):
            eta[j, s, j] = 1.0
    dist = domain_distances(T, bc, domains)
    if any(dd is None for dd in dist):
        raise ValueError("domains are not connected")
    order = sorted(range(len(domains)), key=lambda k: dist[k])
    hop = {}
    info = {}
    S = np.zeros((eta.shape[0], V, 12), dtype=np.complex128)
    for k in order:
        dk = domains[k]
        if dist[k] == 0:
            rhs = slab_extract(T, L, eta, dk)
        else:
            rhs = np.zeros((eta.shape[0], dk[1] * L3, 12), dtype=np.complex128)
            for j in range(len(domains)):
                if dist[j] == dist[k] - 1:
                    hj = _project_slices(T, L, domains[j], hop[j], projections)
                    rhs -= block_apply(U, kappa, T, L, bc, dk, domains[j], hj)
        x, it, rr, st = solve(U, kappa, T, L, bc, rhs, dom=dk, tol=tol, maxit=maxit, method=method)
        info[k] = dict(iters=it, relres=rr, status=st)
        slab_insert(T, L, S, dk, x)
        hop[k] = x
        if overlap > 0 and any(dist[j] == dist[k] + 1 for j in range(len(domains))):
            ext = extended_domain(T, dk, overlap)
            if ext[1] >= T:
                raise ValueError("overlap too thick for slab %d" % k)
            a, b = overlap * L3, (overlap + dk[1]) * L3
            rhs_ext = np.zeros((eta.shape[0], ext[1] * L3, 12), dtype=np.complex128)
            rhs_ext[:, a:b] = rhs
            xe, it, rr, st = solve(U, kappa, T, L, bc, rhs_ext, dom=ext, tol=tol, maxit=maxit, method=method)
            info[k]["extended"] = dict(iters=it, relres=rr, status=st)
            hop[k] = xe[:, a:b]
    return S, info


def exact_propagator(U, kappa, T, L, bc, src, tol=1e-12, maxit=100000, method=0):
    """S_exact = D^-1 eta for the 12 point sources at src (whole lattice)."""
    V = T * L ** 3
    t, x, y, z = src
    eta = np.zeros((12, V, 12), dtype=np.complex128)
    s = ((t * L + z) * L + y) * L + x
    for j in range(12):
        eta[j, s, j] = 1.0
    S, it, rr, st = solve(U, kappa, T, L, bc, eta, dom=None, tol=tol, maxit=maxit, method=method)
    return S, dict(iters=it, relres=rr, status=st)


def pion_correlator(T, L, S, t_src):
    """C(t) = sum_xvec tr[S S^dagger] at sink time (t_src + t) mod T (Eq. 4, W_Pc)."""
    S = np.ascontiguousarray(S, dtype=np.complex128)
    C = (_c.c_double * T)()
    lib().ora_pion(T, L, S.shape[0], _ptr(S), int(t_src), C)
    return np.array(list(C))


def hop_power(U, kappa, T, L, bc, psi, n, dom=None):
    """(kappa D_hop)^n psi on the whole lattice or the slab dom, with kappa D_hop = 1 - 2 kappa D
    (the definition 2 kappa D = 1 - kappa D_hop of Sec. 5; on a slab D is the Dirichlet block)."""
    out = np.array(psi, dtype=np.complex128, copy=True)
    for _ in range(n):
        out = out - 2.0 * kappa * apply_dirac(U, kappa, T, L, bc, out, dom)
    return out


def disconnected_traces(U, kappa, T, L, bc, eta, domains=None, n_hop=8, tol=1e-12, maxit=100000, method=0):
    """Per-source, per-time-slice stochastic estimates of sum_xvec tr{gamma5 D_Lambda^-1(x, x)}
    (Eq. 27 of Sec. 5, with the Dirichlet block D_Lambda of each domain of
    Sec. 4.1 in place of D):
      tau[i, t] = sum_xvec eta_i^+(x) [(kappa D_hop)^n_hop D_Lambda^-1 gamma5 eta_i](x),  x_0 = t,
    eta: (nsrc, V, 12) whole-lattice sources; each domain (t0, nt) of `domains` (None = the
    whole lattice) solves with the restriction of eta to it and fills the slices it covers.
    Returns tau (nsrc, T) complex (zero on slices no domain covers)."""
    L3 = L ** 3
    eta = np.asarray(eta, dtype=np.complex128)
    nsrc = eta.shape[0]
    tau = np.zeros((nsrc, T), dtype=np.complex128)
    for dom in (domains if domains is not None else [None]):
        t0, nt = _norm_dom(T, dom)
        e = slab_extract(T, L, eta, dom) if dom is not None else eta
        x, _, _, st = solve(U, kappa, T, L, bc, gamma5(e), dom=dom, tol=tol, maxit=maxit, method=method)
        if st != 0:
            raise RuntimeError("disconnected-trace solve did not converge")
        y = hop_power(U, kappa, T, L, bc, x, n_hop, dom)
        prod = (e.conj() * y).reshape(nsrc, nt, L3 * 12).sum(axis=2)
        for k in range(nt):
            tau[:, (t0 + k) % T] = prod[:, k]
    return tau


def disconnected_correlator(L, tau):
    """Two-trace product of the disconnected contraction, summed over xvec and yvec (W_Pd of
    Eq. 4; its factorised term W_Pd^(f) of Eq. 19 when tau holds the traces of the domains that
    contain x_0 and y_0):
      C[y0, x0] = 1/L^3 * 1/(n (n - 1)) sum_{i != j} tau_i(x0) tau_j(y0)
    over distinct sources, so that the estimate of the product is unbiased.  tau: (n, T).
    Returns C (T, T) complex."""
    tau = np.asarray(tau, dtype=np.complex128)
    n = tau.shape[0]
    C = np.zeros((tau.shape[1], tau.shape[1]), dtype=np.complex128)
    for i in range(n):
        for j in range(n):
            if i != j:
                C += np.outer(tau[j], tau[i])
    return C / (n * (n - 1) * L ** 3)


def charge_conjugation():
    """C = gamma_0 gamma_2: C gamma_mu C^-1 = -gamma_mu^T in the oracle's basis (the nucleon
    interpolator's charge conjugation, which the text leaves to its conventions)."""
    g = gamma_matrices()
    return g[0] @ g[2]


def nucleon_parity_projector():
    """P_+ = (1 + gamma_0)/2, the spin matrix between the source and sink blocks of the
    factorised nucleon contractions (Eqs. 23-24, read for this basis and operator).

    The text writes gamma5 P_- there, in conventions it leaves to another paper.  With
    this oracle's operator ((1 - gamma_mu) on the forward hop) and lines (xi_i^T =
    phi_i^+ D^-1, Eq. 26, no gamma5), a quark propagating forward in time carries
    (1 + gamma_0)/2 on both sides, so both blocks lie in the range of P_+ and
    B_x^T gamma5 P_(+-) B_y vanishes identically at leading order in the hopping
    expansion; B_x^T P_+ B_y is the positive-parity nucleon two-point function
    tr[P_+ <N(y) Nbar(x)>] of a forward-propagating nucleon (pinned in the free field)."""
    return 0.5 * (np.eye(4) + gamma_matrices()[0])


def baryon_blocks(L, s):
    """Colourless spinors of Eq. 25, summed over each time slice of the field:
      B[t, i, j, k, alpha] = sum_xvec eps^{abc} (s_i^{aT}(x) C gamma5 s_j^b(x)) s_k^c_alpha(x)
    for s (n, nt L^3, 12) (component = spin * 3 + colour).  Returns (nt, n, n, n, 4)."""
    s = np.asarray(s, dtype=np.complex128)
    n = s.shape[0]
    nt = s.shape[1] // L ** 3
    q = s.reshape(n, nt, L ** 3, 4, 3)
    eps = np.zeros((3, 3, 3))
    for a, b, c in ((0, 1, 2), (1, 2, 0), (2, 0, 1)):
        eps[a, b, c] = 1.0
        eps[b, a, c] = -1.0
    cg5 = charge_conjugation() @ gamma_matrices()[4]
    return np.einsum("abc,itxra,rs,jtxsb,ktxpc->tijkp", eps, q, cg5, q, q, optimize=True)


def nucleon_lines(U, kappa, T, L, bc, gbar, gstar, t_phi, phi, x0, tol=1e-12, maxit=100000, method=0):
    """The two factors of each projected quark line (Eq. 26):
      xi_i^T(x) = [phi_i^+ D_Gbar^-1](x) on the time slice x0 of Gbar, and
      eta_i(y) = [D_Gstar^-1 D_{Gstar, dGstar} phi_i](y) on Gstar,
    phi (n, L^3, 12) living on the slice t_phi of Gbar just outside Gstar (D_{Gstar,dGstar}
    is the frontier block of D from that slice into Gstar).  xi_i(x) = conj([D_Gbar^-1+ phi_i](x)),
    and D^-1+ = gamma5 D^-1 gamma5 (gamma5-hermiticity).  Returns (xi (n, L^3, 12),
    eta (n, |Gstar|, 12))."""
    L3 = L ** 3
    phi = np.asarray(phi, dtype=np.complex128)
    n = phi.shape[0]
    gb0, gbn = _norm_dom(T, gbar)
    kp = (t_phi - gb0) % T
    kx = (x0 - gb0) % T
    if kp >= gbn or kx >= gbn:
        raise ValueError("t_phi and x0 must lie in Gbar")
    src = np.zeros((n, gbn * L3, 12), dtype=np.complex128)
    src[:, kp * L3:(kp + 1) * L3] = phi
    z, _, _, st = solve(U, kappa, T, L, bc, gamma5(src), dom=gbar, tol=tol, maxit=maxit, method=method)
    if st != 0:
        raise RuntimeError("nucleon line solve on Gbar did not converge")
    xi = np.conj(gamma5(z))[:, kx * L3:(kx + 1) * L3]
    b = block_apply(U, kappa, T, L, bc, gstar, (t_phi, 1), phi)
    eta, _, _, st = solve(U, kappa, T, L, bc, b, dom=gstar, tol=tol, maxit=maxit, method=method)
    if st != 0:
        raise RuntimeError("nucleon line solve on Gstar did not converge")
    return xi, eta


def nucleon_factorized(L, Bx, By):
    """Factorised nucleon Wick contractions summed over xvec and yvec (Eqs. 22-24):
      W1[y0, x0] = - sum_{ijk} Bx[x0, j, i, k]^T P_+ By[y0, i, j, k]
      W2[y0, x0] = - sum_{ijk} Bx[x0, k, i, j]^T P_+ By[y0, i, j, k]
    with Bx the blocks of the xi lines and By those of the eta lines (baryon_blocks) and
    P_+ the spin matrix of nucleon_parity_projector (the text's gamma5 P_- read for this
    basis).  Returns (W1, W2, C_f = (W1 - W2) / L^3), each (nty, ntx)."""
    M = nucleon_parity_projector()
    W1 = -np.einsum("xjika,ab,yijkb->yx", Bx, M, By, optimize=True)
    W2 = -np.einsum("xkija,ab,yijkb->yx", Bx, M, By, optimize=True)
    return W1, W2, (W1 - W2) / L ** 3


def link_grad(T, L, bc, dom, X, Y, coeff=1.0, grad=None):
    """grad += coeff * d/dU [-2 Re <Y, D_Lambda X>] at fixed X, Y, shape (V, 4, 3, 3)."""
    t0, nt = _norm_dom(T, dom)
    V = T * L ** 3
    if grad is None:
        grad = np.zeros((V, 4, 3, 3), dtype=np.complex128)
    Xc = np.ascontiguousarray(X.reshape(-1, nt * L ** 3, 12), dtype=np.complex128)
    Yc = np.ascontiguousarray(Y.reshape(-1, nt * L ** 3, 12), dtype=np.complex128)
    lib().ora_link_grad(T, L, bc, t0, nt, Xc.shape[0], _ptr(Xc), _ptr(Yc), float(coeff), _ptr(grad))
    return grad


def domain_action(U, kappa, T, L, bc, dom, phi, tol=1e-13, method=0):
    """S = phi^dagger (D_L^dagger D_L)^-1 phi = |Y|^2 with D_L^dagger Y = phi, X = D_L^-1 Y.

    D_L^dagger = gamma_5 D_L gamma_5, so Y = gamma_5 D_L^-1 gamma_5 phi.
    Returns (S, X, Y).
    """
    y5, *_ = solve(U, kappa, T, L, bc, gamma5(phi), dom=dom, tol=tol, method=method)
    Y = gamma5(y5)
    X, *_ = solve(U, kappa, T, L, bc, Y, dom=dom, tol=tol, method=method)
    return float(np.vdot(Y, Y).real), X, Y


def su3_generators() -> np.ndarray:
    """T^a = lambda^a / 2 (Gell-Mann), shape (8, 3, 3)."""
    lam = np.zeros((8, 3, 3), dtype=np.complex128)
    lam[0][0, 1] = lam[0][1, 0] = 1
    lam[1][0, 1] = -1j
    lam[1][1, 0] = 1j
    lam[2][0, 0] = 1
    lam[2][1, 1] = -1
    lam[3][0, 2] = lam[3][2, 0] = 1
    lam[4][0, 2] = -1j
    lam[4][2, 0] = 1j
    lam[5][1, 2] = lam[5][2, 1] = 1
    lam[6][1, 2] = -1j
    lam[6][2, 1] = 1j
    lam[7][0, 0] = lam[7][1, 1] = 1 / np.sqrt(3)
    lam[7][2, 2] = -2 / np.sqrt(3)
    return lam / 2


def su3_force(U, grad):
    """F^a_mu(x) = dS/d omega^a for U -> exp(i omega^a T^a) U, from the gradient
    g = dS/dRe U + i dS/dIm U:  F^a = Re tr[g^dagger i T^a U].  Shape (V, 4, 8)."""
    Tg = su3_generators()
    TU = np.einsum("aij,...jk->...aik", 1j * Tg, U)
    return np.einsum("...ji,...aji->...a", np.conj(grad), TU).real
