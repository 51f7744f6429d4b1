"""Thin Python binding of libdd.so (C ABI in include/dd.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of libdd.so.  Fields are torch tensors on the GPU in the library's
layouts (see include/dd.h):
  links   complex128 / complex64  (4, 9, V)            [mu][3*row+col][site]
  fields  complex128 / complex64  (ncol, 12, nsite)    [col][3*spin+colour][site]
``pack_links`` / ``pack_field`` / ``unpack_field`` convert from the natural
site-major arrays (V, 4, 3, 3) and (ncol, nsite, 12).

Importing this module loads libdd.so and raises ImportError when it has not
been built (``python -m paper_1612_06424_amd.build``); there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdd.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built: run `python -m paper_1612_06424_amd.build`")

_lib = C.CDLL(LIB_PATH)

DD_OK, DD_ERR_ARG, DD_ERR_HIP, DD_ERR_NOMEM, DD_ERR_NOCONV, DD_ERR_BREAKDOWN, DD_ERR_UNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
DD_FP64, DD_FP32, DD_MIXED = 0, 1, 2
DD_BICGSTAB, DD_CGNR = 0, 1
DD_PRECOND_EO, DD_PRECOND_NONE = 0, 1
DD_MAX_RHS = 12

EXPORTS = [
    "dd_create", "dd_destroy", "dd_last_error", "dd_apply_dirac", "dd_frontier_hop", "dd_block_solve",
    "dd_factorized_propagator", "dd_pion_correlator", "dd_block_solve_backward", "dd_domain_action",
    "dd_link_force", "dd_block_solve_batched", "dd_set_kernel_timing", "dd_kernel_timing_count",
    "dd_kernel_timing", "dd_projection_basis", "dd_factorized_propagator_projected",
    "dd_disconnected_traces", "dd_disconnected_correlator", "dd_nucleon_lines", "dd_baryon_blocks",
    "dd_nucleon_contract", "dd_domain_action_backward", "dd_pion_correlator_noalloc",
]


class dd_lattice(C.Structure):
    _fields_ = [("T", C.c_int), ("L", C.c_int), ("time_bc", C.c_int)]


class dd_domain(C.Structure):
    _fields_ = [("t0", C.c_int), ("nt", C.c_int)]


class dd_solver_params(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int), ("prec", C.c_int), ("solver", C.c_int),
                ("delta", C.c_double), ("check_every", C.c_int), ("precond", C.c_int), ("x0", C.c_int)]


class dd_solve_stats(C.Structure):
    _fields_ = [("nrhs", C.c_int), ("iters", C.c_int), ("updates", C.c_int), ("restarts", C.c_int),
                ("true_rel_resid", C.c_double * DD_MAX_RHS), ("ms", C.c_double)]

    def as_dict(self):
        return dict(nrhs=self.nrhs, iters=self.iters, updates=self.updates, restarts=self.restarts,
                    true_rel_resid=list(self.true_rel_resid)[: self.nrhs], ms=self.ms)


class dd_batch_item(C.Structure):
    _fields_ = [("lat", dd_lattice), ("U", C.c_void_p), ("kappa", C.c_double), ("nrhs", C.c_int),
                ("b", C.c_void_p), ("x", C.c_void_p)]


_vp, _d, _i = C.c_void_p, C.c_double, C.c_int
_sig = {
    "dd_create": ([C.POINTER(dd_lattice), _vp, C.POINTER(_vp)], _i),
    "dd_destroy": ([_vp], None),
    "dd_last_error": ([_vp], C.c_char_p),
    "dd_apply_dirac": ([_vp, _vp, _d, C.POINTER(dd_domain), _i, _vp, _vp, _i], _i),
    "dd_frontier_hop": ([_vp, _vp, C.POINTER(dd_domain), C.POINTER(dd_domain), _i, _vp, _vp, _d], _i),
    "dd_block_solve": ([_vp, _vp, _d, C.POINTER(dd_domain), _i, _vp, _vp, C.POINTER(dd_solver_params),
                        C.POINTER(dd_solve_stats)], _i),
    "dd_factorized_propagator": ([_vp, _vp, _d, C.POINTER(C.c_int), C.POINTER(dd_domain), _i, _i,
                                  C.POINTER(dd_solver_params), _vp, _vp, C.POINTER(dd_solve_stats)], _i),
    "dd_factorized_propagator_projected": ([_vp, _vp, _d, C.POINTER(C.c_int), C.POINTER(dd_domain), _i, _i, _i,
                                            C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(_vp),
                                            C.POINTER(dd_solver_params), _vp, _vp, C.POINTER(dd_solve_stats)], _i),
    "dd_projection_basis": ([_vp, _vp, _d, C.POINTER(dd_domain), _i, _i, _i, _i, _vp, _vp,
                             C.POINTER(dd_solver_params), C.POINTER(dd_solve_stats)], _i),
    "dd_pion_correlator": ([_vp, _vp, _i, _i, C.POINTER(C.c_double)], _i),
    "dd_pion_correlator_noalloc": ([_vp, _vp, _i, _i, C.POINTER(C.c_double)], _i),
    "dd_disconnected_traces": ([_vp, _vp, _d, C.POINTER(dd_domain), _i, _i, _vp, _i, C.POINTER(dd_solver_params),
                                _vp, C.POINTER(dd_solve_stats)], _i),
    "dd_disconnected_correlator": ([_vp, _i, _vp, C.POINTER(C.c_double)], _i),
    "dd_nucleon_lines": ([_vp, _vp, _d, C.POINTER(dd_domain), C.POINTER(dd_domain), _i, _i, _vp, _i, _vp, _vp,
                          C.POINTER(dd_solver_params), C.POINTER(dd_solve_stats)], _i),
    "dd_baryon_blocks": ([_vp, _i, _i, _vp, _vp], _i),
    "dd_nucleon_contract": ([_vp, _i, _i, _vp, _i, _vp, C.POINTER(C.c_double)], _i),
    "dd_block_solve_backward": ([_vp, _vp, _d, C.POINTER(dd_domain), _i, _vp, _vp, _vp, _vp,
                                 C.POINTER(dd_solver_params), C.POINTER(dd_solve_stats)], _i),
    "dd_domain_action": ([_vp, _vp, _d, C.POINTER(dd_domain), _i, _vp, _vp, _vp, C.POINTER(C.c_double),
                          C.POINTER(dd_solver_params), C.POINTER(dd_solve_stats)], _i),
    "dd_link_force": ([_vp, C.POINTER(dd_domain), _i, _vp, _vp, _d, _vp], _i),
    "dd_domain_action_backward": ([_vp, C.POINTER(dd_domain), _i, _vp, _vp, _d, _vp, _vp], _i),
    "dd_block_solve_batched": ([_vp, _i, C.POINTER(dd_batch_item), C.POINTER(dd_solver_params),
                                C.POINTER(dd_solve_stats)], _i),
    "dd_set_kernel_timing": ([_vp, _i], _i),
    "dd_kernel_timing_count": ([_vp, C.POINTER(C.c_int)], _i),
    "dd_kernel_timing": ([_vp, _i, C.c_char_p, _i, C.POINTER(C.c_double), C.POINTER(C.c_longlong),
                          C.POINTER(C.c_double)], _i),
}
for _name, (_args, _res) in _sig.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = _res


class DDError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"libdd status {status}: {msg}")
        self.status = status


def solver_params(tol=1e-10, max_iter=20000, prec=DD_FP64, solver=DD_CGNR, delta=0.0, check_every=0,
                  precond=None):
    """Solver parameters; delta = 0 takes the library's reliable-update threshold; precond
    defaults to even-odd (used where the lattice allows it); solves start from zero (x0 = 0,
    see block_solve for an initial guess)."""
    return dd_solver_params(float(tol), int(max_iter), int(prec), int(solver), float(delta), int(check_every),
                            DD_PRECOND_EO if precond is None else int(precond), 0)


def _dom(dom):
    if dom is None:
        return None
    return C.byref(dd_domain(int(dom[0]), int(dom[1])))


def _ptr(t, dtype, name):
    if not isinstance(t, torch.Tensor) or t.dtype != dtype or not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{name}: need a contiguous {dtype} CUDA tensor")
    return C.c_void_p(t.data_ptr())


class Context:
    """A libdd context for a T x L^3 lattice on the current HIP stream."""

    def __init__(self, T, L, time_bc=-1, stream=None):
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        self.T, self.L, self.time_bc = int(T), int(L), int(time_bc)
        self.V = self.T * self.L ** 3
        h = C.c_void_p()
        st = _lib.dd_create(C.byref(dd_lattice(self.T, self.L, self.time_bc)), C.c_void_p(stream.cuda_stream),
                            C.byref(h))
        if st != DD_OK:
            raise DDError(st, "dd_create failed")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            _lib.dd_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st, allow=()):
        if st != DD_OK and st not in allow:
            raise DDError(st, _lib.dd_last_error(self._h).decode())
        return st

    def nsite(self, dom):
        return self.V if dom is None else int(dom[1]) * self.L ** 3


def apply_dirac(ctx, U, kappa, psi, dom=None, out=None):
    """out = D psi (dom None) or D_Lambda psi; FP64 for complex128, FP32 for complex64."""
    prec = DD_FP64 if psi.dtype == torch.complex128 else DD_FP32
    if out is None:
        out = torch.empty_like(psi)
    ncol = psi.shape[0]
    ctx._check(_lib.dd_apply_dirac(ctx._h, _ptr(U, psi.dtype, "U"), float(kappa), _dom(dom), ncol,
                                   _ptr(psi, psi.dtype, "psi"), _ptr(out, psi.dtype, "out"), prec))
    return out


def frontier_hop(ctx, U, dst, src, psi, out, alpha=1.0):
    """out += alpha P_dst D P_src psi (FP64)."""
    ctx._check(_lib.dd_frontier_hop(ctx._h, _ptr(U, torch.complex128, "U"), _dom(dst), _dom(src), psi.shape[0],
                                    _ptr(psi, torch.complex128, "psi"), _ptr(out, torch.complex128, "out"),
                                    float(alpha)))
    return out


def block_solve(ctx, U, kappa, b, dom=None, params=None, x=None, allow_noconv=False, guess=False):
    """x = D_Lambda^-1 b for the columns of b (complex128, (ncol, 12, nsite)).  With guess=True
    the given x is the initial guess (overwritten by the solution); otherwise the solve starts
    from zero.  Returns (x, stats)."""
    params = params or solver_params()
    if guess and x is None:
        raise ValueError("guess=True needs x")
    if x is None:
        x = torch.empty_like(b)
    p = dd_solver_params(params.tol, params.max_iter, params.prec, params.solver, params.delta,
                         params.check_every, params.precond, 1 if guess else 0)
    stats = dd_solve_stats()
    ctx._check(_lib.dd_block_solve(ctx._h, _ptr(U, torch.complex128, "U"), float(kappa), _dom(dom), b.shape[0],
                                   _ptr(b, torch.complex128, "b"), _ptr(x, torch.complex128, "x"),
                                   C.byref(p), C.byref(stats)),
               allow=(DD_ERR_NOCONV,) if allow_noconv else ())
    return x, stats.as_dict()


def factorized_propagator(ctx, U, kappa, src, doms, params=None, exact=False, S_fact=None, S_exact=None, overlap=0,
                          projections=None):
    """S_fact (and S_exact) as complex128 (12, 12, V), with overlap regions of `overlap` time
    slices and the quark line cut on the slices t of projections = {t: phi} (phi complex128
    (nvec, 12, L^3)).  Returns (S_fact, S_exact or None, stats)."""
    params = params or solver_params()
    V = ctx.V
    if S_fact is None:
        S_fact = torch.empty((12, 12, V), dtype=torch.complex128, device=U.device)
    if exact and S_exact is None:
        S_exact = torch.empty((12, 12, V), dtype=torch.complex128, device=U.device)
    srcarr = (C.c_int * 4)(*[int(v) for v in src])
    darr = (dd_domain * len(doms))(*[dd_domain(int(a), int(b)) for a, b in doms])
    stats = (dd_solve_stats * (len(doms) + 1))()
    if projections:
        ts = sorted(projections)
        n = len(ts)
        ctx._check(_lib.dd_factorized_propagator_projected(
            ctx._h, _ptr(U, torch.complex128, "U"), float(kappa), srcarr, darr, len(doms), int(overlap), n,
            (C.c_int * n)(*[int(t) for t in ts]), (C.c_int * n)(*[int(projections[t].shape[0]) for t in ts]),
            (_vp * n)(*[_ptr(projections[t], torch.complex128, "phi") for t in ts]), C.byref(params),
            _ptr(S_fact, torch.complex128, "S_fact"),
            _ptr(S_exact, torch.complex128, "S_exact") if exact else None, stats))
    else:
        ctx._check(_lib.dd_factorized_propagator(
            ctx._h, _ptr(U, torch.complex128, "U"), float(kappa), srcarr, darr, len(doms), int(overlap),
            C.byref(params), _ptr(S_fact, torch.complex128, "S_fact"),
            _ptr(S_exact, torch.complex128, "S_exact") if exact else None, stats))
    return S_fact, (S_exact if exact else None), [s.as_dict() for s in stats]


def projection_basis(ctx, U, kappa, pi, t_slice, sign, v0, n_iter, params=None, phi=None, allow_noconv=False):
    """Quark-line projection vectors phi (complex128 (nvec, 12, L^3)) of the hop leaving slice
    t_slice of the slab pi = (t0, nt) forward (sign +1) or backward (-1), by n_iter inverse
    iterations from v0 (complex128 (nvec, 12, nt L^3)).  Returns (phi, stats)."""
    params = params or solver_params()
    nvec = v0.shape[0]
    if phi is None:
        phi = torch.empty((nvec, 12, ctx.L ** 3), dtype=torch.complex128, device=v0.device)
    stats = dd_solve_stats()
    ctx._check(_lib.dd_projection_basis(
        ctx._h, _ptr(U, torch.complex128, "U"), float(kappa), _dom(pi), int(t_slice), int(sign), nvec,
        int(n_iter), _ptr(v0, torch.complex128, "v0"), _ptr(phi, torch.complex128, "phi"), C.byref(params),
        C.byref(stats)), allow=(DD_ERR_NOCONV,) if allow_noconv else ())
    return phi, stats.as_dict()


def pion_correlator(ctx, S, t_src):
    """C(t), t = 0..T-1, as a numpy float64 array."""
    out = (C.c_double * ctx.T)()
    ctx._check(_lib.dd_pion_correlator(ctx._h, _ptr(S, torch.complex128, "S"), S.shape[0], int(t_src), out))
    return np.array(list(out))


def pion_correlator_noalloc(ctx, S, t_src):
    """pion_correlator through the allocation-free entry point (static device scratch)."""
    out = (C.c_double * ctx.T)()
    ctx._check(_lib.dd_pion_correlator_noalloc(ctx._h, _ptr(S, torch.complex128, "S"), S.shape[0], int(t_src), out))
    return np.array(list(out))


def disconnected_traces(ctx, U, kappa, eta, doms=None, n_hop=8, params=None, tau=None, allow_noconv=False):
    """Per-source, per-slice stochastic traces tau (complex128 (nsrc, T)) of gamma5 D_Lambda^-1
    with n_hop powers of kappa D_hop, from whole-lattice sources eta (complex128 (nsrc, 12, V)),
    over the slabs doms (None: the whole lattice).  Returns (tau, per-domain stats)."""
    params = params or solver_params()
    nsrc = eta.shape[0]
    if tau is None:
        tau = torch.empty((nsrc, ctx.T), dtype=torch.complex128, device=eta.device)
    nd = len(doms) if doms else 0
    darr = (dd_domain * nd)(*[dd_domain(int(a), int(b)) for a, b in doms]) if nd else None
    stats = (dd_solve_stats * max(nd, 1))()
    ctx._check(_lib.dd_disconnected_traces(
        ctx._h, _ptr(U, torch.complex128, "U"), float(kappa), darr, nd, nsrc, _ptr(eta, torch.complex128, "eta"),
        int(n_hop), C.byref(params), _ptr(tau, torch.complex128, "tau"), stats),
        allow=(DD_ERR_NOCONV,) if allow_noconv else ())
    return tau, [s.as_dict() for s in stats]


def disconnected_correlator(ctx, tau):
    """C[y0, x0] = 1/(n (n-1) L^3) sum_{i != j} tau_i(x0) tau_j(y0) as numpy complex128 (T, T)."""
    out = (C.c_double * (2 * ctx.T * ctx.T))()
    ctx._check(_lib.dd_disconnected_correlator(ctx._h, tau.shape[0], _ptr(tau, torch.complex128, "tau"), out))
    a = np.array(list(out)).reshape(ctx.T, ctx.T, 2)
    return a[..., 0] + 1j * a[..., 1]


def nucleon_lines(ctx, U, kappa, gbar, gstar, t_phi, phi, x0, params=None, allow_noconv=False):
    """xi (complex128 (nvec, 12, L^3), slice x0) and eta (complex128 (nvec, 12, |gstar|)) of the
    quark lines cut by phi (complex128 (nvec, 12, L^3)) on slice t_phi.  Returns (xi, eta, stats)."""
    params = params or solver_params()
    nvec = phi.shape[0]
    L3 = ctx.L ** 3
    xi = torch.empty((nvec, 12, L3), dtype=torch.complex128, device=phi.device)
    eta = torch.empty((nvec, 12, int(gstar[1]) * L3), dtype=torch.complex128, device=phi.device)
    stats = (dd_solve_stats * 2)()
    ctx._check(_lib.dd_nucleon_lines(
        ctx._h, _ptr(U, torch.complex128, "U"), float(kappa), _dom(gbar), _dom(gstar), int(t_phi), nvec,
        _ptr(phi, torch.complex128, "phi"), int(x0), _ptr(xi, torch.complex128, "xi"),
        _ptr(eta, torch.complex128, "eta"), C.byref(params), stats), allow=(DD_ERR_NOCONV,) if allow_noconv else ())
    return xi, eta, [s.as_dict() for s in stats]


def baryon_blocks(ctx, s, B=None):
    """Blocks of Eq. 25 per time slice of s (complex128 (n, 12, nt L^3)) as complex128
    (nt, n, 4, n, n), index [t][k][alpha][i][j]."""
    n = s.shape[0]
    nt = s.shape[2] // ctx.L ** 3
    if B is None:
        B = torch.empty((nt, n, 4, n, n), dtype=torch.complex128, device=s.device)
    ctx._check(_lib.dd_baryon_blocks(ctx._h, n, nt, _ptr(s, torch.complex128, "s"), _ptr(B, torch.complex128, "B")))
    return B


def nucleon_contract(ctx, Bx, By):
    """(W1, W2) as numpy complex128 (nty, ntx) from blocks of baryon_blocks."""
    n = Bx.shape[1]
    ntx, nty = Bx.shape[0], By.shape[0]
    out = (C.c_double * (4 * nty * ntx))()
    ctx._check(_lib.dd_nucleon_contract(ctx._h, n, ntx, _ptr(Bx, torch.complex128, "Bx"), nty,
                                        _ptr(By, torch.complex128, "By"), out))
    a = np.array(list(out)).reshape(2, nty, ntx, 2)
    W = a[..., 0] + 1j * a[..., 1]
    return W[0], W[1]


def block_solve_backward(ctx, U, kappa, x, grad_x, dom=None, params=None, grad_U=None):
    """Returns (grad_b, grad_U, stats); grad_U accumulates into the given tensor."""
    params = params or solver_params()
    grad_b = torch.empty_like(grad_x)
    if grad_U is None:
        grad_U = torch.zeros_like(U)
    stats = dd_solve_stats()
    ctx._check(_lib.dd_block_solve_backward(
        ctx._h, _ptr(U, torch.complex128, "U"), float(kappa), _dom(dom), x.shape[0], _ptr(x, torch.complex128, "x"),
        _ptr(grad_x, torch.complex128, "grad_x"), _ptr(grad_b, torch.complex128, "grad_b"),
        _ptr(grad_U, torch.complex128, "grad_U"), C.byref(params), C.byref(stats)))
    return grad_b, grad_U, stats.as_dict()


def domain_action(ctx, U, kappa, phi, dom=None, params=None):
    """(S, X, Y, stats) with Y = D^-+ phi, X = D^-1 Y, S = |Y|^2."""
    params = params or solver_params()
    X = torch.empty_like(phi)
    Y = torch.empty_like(phi)
    S = C.c_double()
    stats = dd_solve_stats()
    ctx._check(_lib.dd_domain_action(ctx._h, _ptr(U, torch.complex128, "U"), float(kappa), _dom(dom), phi.shape[0],
                                     _ptr(phi, torch.complex128, "phi"), _ptr(X, torch.complex128, "X"),
                                     _ptr(Y, torch.complex128, "Y"), C.byref(S), C.byref(params), C.byref(stats)))
    return S.value, X, Y, stats.as_dict()


def domain_action_backward(ctx, X, Y, g_S, grad_U, dom=None, grad_phi=None):
    """grad_U += g_S * force(X, Y) and grad_phi = 2 g_S X, both in libdd.  Returns grad_phi."""
    if grad_phi is None:
        grad_phi = torch.empty_like(X)
    ctx._check(_lib.dd_domain_action_backward(ctx._h, _dom(dom), X.shape[0], _ptr(X, torch.complex128, "X"),
                                              _ptr(Y, torch.complex128, "Y"), float(g_S),
                                              _ptr(grad_U, torch.complex128, "grad_U"),
                                              _ptr(grad_phi, torch.complex128, "grad_phi")))
    return grad_phi


def link_force(ctx, X, Y, coeff, grad_U, dom=None):
    """grad_U += coeff * d/dU [-2 Re <Y, D X>]."""
    ctx._check(_lib.dd_link_force(ctx._h, _dom(dom), X.shape[0], _ptr(X, torch.complex128, "X"),
                                  _ptr(Y, torch.complex128, "Y"), float(coeff),
                                  _ptr(grad_U, torch.complex128, "grad_U")))
    return grad_U


def block_solve_batched(ctx, items, params=None):
    """items: list of dicts(T, L, time_bc, U, kappa, b, x).  Returns per-item stats."""
    params = params or solver_params()
    arr = (dd_batch_item * len(items))()
    for k, it in enumerate(items):
        arr[k] = dd_batch_item(dd_lattice(int(it["T"]), int(it["L"]), int(it.get("time_bc", 0))),
                               _ptr(it["U"], torch.complex128, "U"), float(it["kappa"]), int(it["b"].shape[0]),
                               _ptr(it["b"], torch.complex128, "b"), _ptr(it["x"], torch.complex128, "x"))
    stats = (dd_solve_stats * len(items))()
    ctx._check(_lib.dd_block_solve_batched(ctx._h, len(items), arr, C.byref(params), stats))
    return [s.as_dict() for s in stats]


def set_kernel_timing(ctx, enable):
    ctx._check(_lib.dd_set_kernel_timing(ctx._h, int(bool(enable))))


def kernel_timing(ctx):
    """{kernel instance name: (ms, launches, algorithmic bytes)} of the stencil launches
    timed with HIP events since timing was last switched."""
    cnt = C.c_int()
    ctx._check(_lib.dd_kernel_timing_count(ctx._h, C.byref(cnt)))
    out = {}
    for i in range(cnt.value):
        name = C.create_string_buffer(128)
        ms, n, b = C.c_double(), C.c_longlong(), C.c_double()
        ctx._check(_lib.dd_kernel_timing(ctx._h, i, name, 128, C.byref(ms), C.byref(n), C.byref(b)))
        out[name.value.decode()] = (ms.value, n.value, b.value)
    return out


# ------------------------------------------------------------------ layout marshalling

def pack_links(U_nat, dtype=torch.complex128, device="cuda"):
    """(V, 4, 3, 3) natural links -> (4, 9, V) device tensor."""
    t = torch.as_tensor(np.asarray(U_nat)).reshape(-1, 4, 9).permute(1, 2, 0).contiguous()
    return t.to(device=device, dtype=dtype)


def pack_field(f_nat, dtype=torch.complex128, device="cuda"):
    """(ncol, nsite, 12) natural field -> (ncol, 12, nsite) device tensor."""
    t = torch.as_tensor(np.asarray(f_nat))
    if t.dim() == 2:
        t = t[None]
    return t.permute(0, 2, 1).contiguous().to(device=device, dtype=dtype)


def unpack_field(f):
    """(ncol, 12, nsite) device tensor -> (ncol, nsite, 12) numpy complex128."""
    return f.detach().to("cpu", torch.complex128).permute(0, 2, 1).contiguous().numpy()


def unpack_links(Ut):
    """(4, 9, V) device tensor -> (V, 4, 3, 3) numpy complex128."""
    return Ut.detach().to("cpu", torch.complex128).permute(2, 0, 1).contiguous().numpy().reshape(-1, 4, 3, 3)


# ------------------------------------------------------------------ autograd

class BlockSolveFn(torch.autograd.Function):
    """x = D_Lambda(U)^-1 b, differentiable in U and b through the hand-written
    adjoint solve (dd_block_solve_backward)."""

    @staticmethod
    def forward(fctx, U, b, ctx, kappa, dom, params):
        x, _ = block_solve(ctx, U, kappa, b.contiguous(), dom, params)
        fctx.save_for_backward(U, x)
        fctx.dd = (ctx, kappa, dom, params)
        return x

    @staticmethod
    def backward(fctx, grad_x):
        U, x = fctx.saved_tensors
        ctx, kappa, dom, params = fctx.dd
        grad_b, grad_U, _ = block_solve_backward(ctx, U, kappa, x, grad_x.contiguous(), dom, params)
        return grad_U, grad_b, None, None, None, None


class DomainActionFn(torch.autograd.Function):
    """S = phi^+ (D_Lambda^+ D_Lambda)^-1 phi with its link force from one extra
    (adjoint) solve: forward solves D^+ Y = phi and D X = Y; backward needs no
    further solve (grad_U = force(X, Y), grad_phi = 2 X)."""

    @staticmethod
    def forward(fctx, U, phi, ctx, kappa, dom, params):
        S, X, Y, _ = domain_action(ctx, U, kappa, phi.contiguous(), dom, params)
        fctx.save_for_backward(X, Y, U)
        fctx.dd = (ctx, dom)
        return torch.tensor(S, dtype=torch.float64, device=phi.device)

    @staticmethod
    def backward(fctx, gS):
        X, Y, U = fctx.saved_tensors
        ctx, dom = fctx.dd
        grad_U = torch.zeros_like(U)
        grad_phi = domain_action_backward(ctx, X, Y, float(gS.item()), grad_U, dom)
        return grad_U, grad_phi, None, None, None, None
