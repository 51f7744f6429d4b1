"""GPU parity of the solves, the factorised propagator, the pion correlator and the
adjoint (link force) against the oracle, plus the error paths of the C ABI.

Bars: FP64 results within 1e-10 of the oracle (relative field norm), mixed precision
within 1e-6; the correlator gated on max_t |dC(t)| / max_t C(t).
"""
import numpy as np
import pytest
import torch

import oracle as O
from helpers import gaussian_field, lib, random_links, relerr, step
from paper_1612_06424_amd.inputs import WORKLOADS, point_sources

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("solver", [0, 1])
@pytest.mark.parametrize("T,L,bc,dom,kappa,eps", [
    (16, 4, -1, None, 0.125, 0.3),
    (16, 4, -1, (0, 8), 0.125, 0.3),
    (12, 6, -1, (9, 5), 0.13, 0.3),
    (8, 5, 0, None, 0.135, 0.2),
])
def test_block_solve_vs_oracle(prec, solver, T, L, bc, dom, kappa, eps):
    dd = lib()
    step(f"solve {prec} solver={solver} T={T} L={L} bc={bc} dom={dom}")
    U = random_links(T, L, eps, 2000 + T)
    nsite = (T if dom is None else dom[1]) * L ** 3
    b = gaussian_field(nsite, 3, 2001)
    ref, it, rr, st = O.solve(U, kappa, T, L, bc, b, dom=dom, tol=1e-13, method=solver)
    assert st == 0
    ctx = dd.Context(T, L, bc)
    p = dd.solver_params(tol=1e-12 if prec == "fp64" else 1e-10, max_iter=20000,
                         prec=dd.DD_FP64 if prec == "fp64" else dd.DD_MIXED, solver=solver)
    x, stats = dd.block_solve(ctx, dd.pack_links(U), kappa, dd.pack_field(b), dom, p)
    got = dd.unpack_field(x)
    assert max(stats["true_rel_resid"]) <= p.tol
    assert relerr(got, ref) < (1e-10 if prec == "fp64" else 1e-6)
    # the residual also holds when measured by the oracle's own operator
    Dx = O.apply_dirac(U, kappa, T, L, bc, got, dom)
    assert relerr(Dx, b) <= 2 * p.tol


def test_adjoint_solve_through_backward():
    """grad_b of x = D^-1 b is D^-+ grad_x: check D^+ grad_b = grad_x with the oracle."""
    dd = lib()
    step("adjoint solve")
    T, L, bc, kappa, dom = 12, 4, -1, 0.13, (2, 6)
    U = random_links(T, L, 0.3, 2100)
    nsite = dom[1] * L ** 3
    b = gaussian_field(nsite, 2, 2101)
    g = gaussian_field(nsite, 2, 2102)
    ctx = dd.Context(T, L, bc)
    Ud = dd.pack_links(U)
    p = dd.solver_params(tol=1e-12)
    x, _ = dd.block_solve(ctx, Ud, kappa, dd.pack_field(b), dom, p)
    gb, gU, _ = dd.block_solve_backward(ctx, Ud, kappa, x, dd.pack_field(g), dom, p)
    lam = dd.unpack_field(gb)
    # D^+ = gamma5 D gamma5
    Ddag_lam = O.gamma5(O.apply_dirac(U, kappa, T, L, bc, O.gamma5(lam), dom))
    assert relerr(Ddag_lam, g) < 1e-11
    # link gradient of the loss: grad_U = 1/2 * grad of -2 Re<lambda, D x>
    ref = O.link_grad(T, L, bc, dom, dd.unpack_field(x), lam, coeff=0.5)
    assert relerr(dd.unpack_links(gU), ref) < 1e-12


def _workload_16x4():
    w = WORKLOADS["16x4^3"]
    return w, random_links(w["T"], w["L"], w["eps"], w["link_seed"])


def test_factorised_propagator_and_correlator_16x4():
    """The 16x4^3 workload: two slabs [0,8), [8,16), point source at the origin."""
    dd = lib()
    step("factorised propagator 16x4^3")
    w, U = _workload_16x4()
    T, L, bc, kappa = w["T"], w["L"], w["bc"], w["kappa"]
    src = w["sources"][0]
    Sf_ref, _ = O.factorized_propagator(U, kappa, T, L, bc, src, w["domains"], tol=1e-13)
    Se_ref, _ = O.exact_propagator(U, kappa, T, L, bc, src, tol=1e-13)
    ctx = dd.Context(T, L, bc)
    p = dd.solver_params(tol=1e-13)
    Sf, Se, stats = dd.factorized_propagator(ctx, dd.pack_links(U), kappa, src, w["domains"], p, exact=True)
    assert relerr(dd.unpack_field(Sf), Sf_ref) < 1e-10
    assert relerr(dd.unpack_field(Se), Se_ref) < 1e-10
    Cf = dd.pion_correlator(ctx, Sf, src[0])
    Ce = dd.pion_correlator(ctx, Se, src[0])
    Cf_ref = O.pion_correlator(T, L, Sf_ref, src[0])
    Ce_ref = O.pion_correlator(T, L, Se_ref, src[0])
    assert np.abs(Cf - Cf_ref).max() / Cf_ref.max() < 1e-10
    assert np.abs(Ce - Ce_ref).max() / Ce_ref.max() < 1e-10
    # the contraction itself on identical input: exact to summation order
    Cg = O.pion_correlator(T, L, dd.unpack_field(Se), src[0])
    assert np.abs(Ce - Cg).max() / Cg.max() < 1e-14


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_factorised_four_slabs_with_wrap(prec):
    """Four slabs on a ring (the middle slab reached from both sides), source off the origin."""
    dd = lib()
    step(f"factorised 4 slabs {prec}")
    T, L, bc, kappa = 16, 4, -1, 0.13
    U = random_links(T, L, 0.3, 2200)
    doms = [(14, 4), (2, 4), (6, 4), (10, 4)]
    src = (15, 1, 2, 3)
    Sf_ref, _ = O.factorized_propagator(U, kappa, T, L, bc, src, doms, tol=1e-13)
    ctx = dd.Context(T, L, bc)
    p = dd.solver_params(tol=1e-13 if prec == "fp64" else 1e-10,
                         prec=dd.DD_FP64 if prec == "fp64" else dd.DD_MIXED)
    Sf, _, _ = dd.factorized_propagator(ctx, dd.pack_links(U), kappa, src, doms, p)
    assert relerr(dd.unpack_field(Sf), Sf_ref) < (1e-10 if prec == "fp64" else 1e-6)
    C = dd.pion_correlator(ctx, Sf, src[0])
    Cr = O.pion_correlator(T, L, Sf_ref, src[0])
    assert np.abs(C - Cr).max() / Cr.max() < (1e-10 if prec == "fp64" else 1e-6)


@pytest.mark.parametrize("case", ["two-slabs-1", "two-slabs-3", "ring-2", "dirichlet-2"])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_factorised_overlap_vs_oracle(case, prec):
    """Overlap regions (Sec. 3.2, Delta > 0): the slabs that feed a frontier are also
    solved on their extension; S_fact and its correlator against the oracle."""
    dd = lib()
    step(f"factorised overlap {case} {prec}")
    T, L, kappa = 16, 4, 0.13
    geo = {"two-slabs-1": (-1, [(0, 8), (8, 8)], (3, 1, 2, 0), 1),
           "two-slabs-3": (-1, [(0, 8), (8, 8)], (3, 1, 2, 0), 3),
           "ring-2": (-1, [(14, 4), (2, 4), (6, 4), (10, 4)], (15, 1, 2, 3), 2),
           "dirichlet-2": (0, [(0, 6), (6, 5), (11, 5)], (2, 0, 1, 3), 2)}
    bc, doms, src, dlt = geo[case]
    U = random_links(T, L, 0.3, 2400)
    Sf_ref, _ = O.factorized_propagator(U, kappa, T, L, bc, src, doms, tol=1e-13, overlap=dlt)
    ctx = dd.Context(T, L, bc)
    p = dd.solver_params(tol=1e-13 if prec == "fp64" else 1e-10,
                         prec=dd.DD_FP64 if prec == "fp64" else dd.DD_MIXED)
    Sf, _, stats = dd.factorized_propagator(ctx, dd.pack_links(U), kappa, src, doms, p, overlap=dlt)
    bar = 1e-10 if prec == "fp64" else 1e-6
    assert relerr(dd.unpack_field(Sf), Sf_ref) < bar
    C = dd.pion_correlator(ctx, Sf, src[0])
    Cr = O.pion_correlator(T, L, Sf_ref, src[0])
    assert np.abs(C - Cr).max() / Cr.max() < bar
    assert all(max(st["true_rel_resid"]) <= p.tol for st in stats[:len(doms)])


@pytest.mark.parametrize("dlt", [4, 6])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_factorised_thick_overlap_vs_oracle(dlt, prec):
    """Thick overlap regions (Delta = 4 and 6 on a ring of four 8-slice slabs of a 32 x 4^3
    lattice: the extended slabs span 16 and 20 slices) against the oracle; the correction to
    the exact correlator just past the first frontier then shrinks with Delta (Sec. 3.2 Eq. 15;
    kappa below the free critical value so that the fall-off shows on a lattice this small)."""
    dd = lib()
    step(f"factorised thick overlap {dlt} {prec}")
    T, L, kappa, bc = 32, 4, 0.115, -1
    doms, src = [(0, 8), (8, 8), (16, 8), (24, 8)], (3, 1, 2, 0)
    U = random_links(T, L, 0.3, 2450)
    Sf_ref, _ = O.factorized_propagator(U, kappa, T, L, bc, src, doms, tol=1e-13, overlap=dlt)
    ctx = dd.Context(T, L, bc)
    p = dd.solver_params(tol=1e-13 if prec == "fp64" else 1e-10,
                         prec=dd.DD_FP64 if prec == "fp64" else dd.DD_MIXED)
    Ud = dd.pack_links(U)
    Sf, Se, stats = dd.factorized_propagator(ctx, Ud, kappa, src, doms, p, overlap=dlt, exact=True)
    bar = 1e-10 if prec == "fp64" else 1e-6
    assert relerr(dd.unpack_field(Sf), Sf_ref) < bar
    C = dd.pion_correlator(ctx, Sf, src[0])
    Cr = O.pion_correlator(T, L, Sf_ref, src[0])
    assert np.abs(C - Cr).max() / Cr.max() < bar
    if prec == "fp64":
        # the correction on the first slice across the frontier falls with Delta (the oracle
        # gives 1e-5, 1e-7, 2e-9 relative for Delta = 2, 4, 6; slices further on carry the
        # truncation of the chain over four slabs as well, which Delta does not change)
        S0, _, _ = dd.factorized_propagator(ctx, Ud, kappa, src, doms, p, overlap=dlt - 2)
        Ce = dd.pion_correlator(ctx, Se, src[0])
        C0 = dd.pion_correlator(ctx, S0, src[0])
        t = 8 - src[0]  # slice 8
        assert abs(Ce[t] - C[t]) < 0.1 * abs(Ce[t] - C0[t]), (Ce[t], C[t], C0[t])


def test_factorised_overlap_errors():
    dd = lib()
    step("factorised overlap errors")
    T, L, bc = 16, 4, -1
    U = random_links(T, L, 0.3, 2401)
    ctx = dd.Context(T, L, bc)
    Ud = dd.pack_links(U)
    for dlt in (-1, 4):  # negative; 8 + 2 * 4 slices is the whole lattice
        with pytest.raises(dd.DDError) as e:
            dd.factorized_propagator(ctx, Ud, 0.13, (3, 1, 2, 0), [(0, 8), (8, 8)], overlap=dlt)
        assert e.value.status == dd.DD_ERR_ARG


def test_domain_action_force_vs_oracle():
    dd = lib()
    step("domain action + force")
    T, L, bc, kappa = 8, 4, 0, 0.13
    U = random_links(T, L, 0.3, 2300)
    phi = gaussian_field(T * L ** 3, 1, 2301)
    S_ref, X_ref, Y_ref = O.domain_action(U, kappa, T, L, bc, None, phi[0])
    g_ref = O.link_grad(T, L, bc, None, X_ref, Y_ref, coeff=1.0)
    ctx = dd.Context(T, L, bc)
    Ud = dd.pack_links(U).requires_grad_(True)
    ph = dd.pack_field(phi).requires_grad_(True)
    p = dd.solver_params(tol=1e-13)
    S = dd.DomainActionFn.apply(Ud, ph, ctx, kappa, None, p)
    S.backward()
    assert abs(S.item() - S_ref) < 1e-10 * S_ref
    assert relerr(dd.unpack_links(Ud.grad), g_ref) < 1e-10
    assert relerr(dd.unpack_field(ph.grad)[0], 2 * X_ref) < 1e-10


def test_error_paths():
    dd = lib()
    step("error paths")
    T, L, bc = 8, 4, -1
    U = random_links(T, L, 0.3, 2400)
    ctx = dd.Context(T, L, bc)
    Ud = dd.pack_links(U)
    b = dd.pack_field(gaussian_field(T * L ** 3, 2, 2401))
    # max_iter = 1 -> no convergence, stats filled
    x, stats = dd.block_solve(ctx, Ud, 0.13, b, None, dd.solver_params(tol=1e-12, max_iter=1), allow_noconv=True)
    with pytest.raises(dd.DDError) as e:
        dd.block_solve(ctx, Ud, 0.13, b, None, dd.solver_params(tol=1e-12, max_iter=1))
    assert e.value.status == dd.DD_ERR_NOCONV
    assert stats["nrhs"] == 2 and max(stats["true_rel_resid"]) > 1e-12
    # NaN in the source
    bn = b.clone()
    bn[0, 0, 3] = complex(float("nan"), 0.0)
    with pytest.raises(dd.DDError) as e:
        dd.block_solve(ctx, Ud, 0.13, bn)
    assert e.value.status == dd.DD_ERR_BREAKDOWN
    # a slab as long as the lattice, slabs that do not partition [0, T), host memory
    with pytest.raises(dd.DDError) as e:
        dd.apply_dirac(ctx, Ud, 0.13, b, dom=(0, T))
    assert e.value.status == dd.DD_ERR_ARG
    with pytest.raises(dd.DDError) as e:
        dd.factorized_propagator(ctx, Ud, 0.13, (0, 0, 0, 0), [(0, 4), (5, 3)])
    assert e.value.status == dd.DD_ERR_ARG
    with pytest.raises(ValueError):
        dd.apply_dirac(ctx, Ud, 0.13, b.cpu())


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("solver", [0, 1])
@pytest.mark.parametrize("T,L,bc,dom", [
    (16, 4, -1, None),      # whole lattice, T and L even: even-odd applies
    (12, 6, -1, (9, 5)),    # odd-length slab across the time wrap
    (8, 4, 0, None),        # Dirichlet time walls
])
def test_even_odd_matches_full_operator(prec, solver, T, L, bc, dom):
    """The even-odd preconditioned solve and the plain one both reach the oracle's
    solution (and so each other)."""
    dd = lib()
    step(f"even-odd {prec} solver={solver} T={T} L={L} bc={bc} dom={dom}")
    kappa = 0.13
    U = random_links(T, L, 0.3, 2500 + T)
    nsite = (T if dom is None else dom[1]) * L ** 3
    b = gaussian_field(nsite, 4, 2501)
    ref, _, _, st = O.solve(U, kappa, T, L, bc, b, dom=dom, tol=1e-13, method=1)
    assert st == 0
    ctx = dd.Context(T, L, bc)
    tol = 1e-12 if prec == "fp64" else 1e-10
    bar = 1e-10 if prec == "fp64" else 1e-6
    got = {}
    for pc in (dd.DD_PRECOND_EO, dd.DD_PRECOND_NONE):
        p = dd.solver_params(tol=tol, prec=dd.DD_FP64 if prec == "fp64" else dd.DD_MIXED, solver=solver, precond=pc)
        x, stats = dd.block_solve(ctx, dd.pack_links(U), kappa, dd.pack_field(b), dom, p)
        assert max(stats["true_rel_resid"]) <= tol
        got[pc] = dd.unpack_field(x)
        assert relerr(got[pc], ref) < bar
    assert relerr(got[dd.DD_PRECOND_EO], got[dd.DD_PRECOND_NONE]) < 2 * bar


@pytest.mark.parametrize("precond", [0, 1])
def test_cgnr_columns_stopping_inside_a_round_keep_their_last_update(precond):
    """CGNR adds alpha p to x at the end of an iteration, together with the new search
    direction; a column whose recursion stops in that iteration must still receive it.
    One round of inner iterations covers the whole FP64 solve (check_every above the
    iteration count), Gaussian and point sources stop at different iterations inside it,
    and every true residual must then meet tol at the single reliable update (a lost
    update would leave a residual of order alpha |M p| and force further rounds)."""
    dd = lib()
    step(f"CGNR stopping columns precond={precond}")
    T, L, bc, dom, kappa = 16, 6, -1, (4, 8), 0.13
    U = random_links(T, L, 0.3, 2900)
    nsite = dom[1] * L ** 3
    b = gaussian_field(nsite, 12, 2901)
    b[6:] = 0
    for j in range(6, 12):
        b[j, (j * 379) % nsite, j] = 1.0
    ctx = dd.Context(T, L, bc)
    p = dd.solver_params(tol=1e-10, prec=dd.DD_FP64, solver=dd.DD_CGNR, check_every=5000, precond=precond)
    x, st = dd.block_solve(ctx, dd.pack_links(U), kappa, dd.pack_field(b), dom, p)
    assert st["updates"] == 1 and st["restarts"] == 0, st
    assert max(st["true_rel_resid"]) <= 1e-10
    ref, _, _, ost = O.solve(U, kappa, T, L, bc, b, dom=dom, tol=1e-13, method=1)
    assert ost == 0
    assert relerr(dd.unpack_field(x), ref) < 1e-8


@pytest.mark.parametrize("solver", [0, 1])
def test_even_odd_launch_shapes_bitwise(solver, tmp_path, monkeypatch):
    """The XCD remap of the half hop only moves work between workgroups, and
    non-temporal output stores only change a cache policy: mixed solves give
    bitwise the same solution.  Columns per thread (the kernel is
    compiled once per count, and the compiler may contract multiply-adds
    differently in each), the chunk length, the tile shape and the order of tiles
    and chunks over the workgroups (all regroup the partial sums) change the
    rounding only: the solutions agree to 1e-8 with the same
    iteration counts within a few.  Gaussian and point sources stop at
    different iterations, so stopped columns share workgroups with running
    ones, whose launches must leave the stopped columns' vectors as they were
    (otherwise the reliable updates lose the search directions)."""
    dd = lib()
    step(f"even-odd launch shapes solver={solver}")
    T, L, bc, dom, kappa = 16, 8, -1, (4, 8), 0.13
    U = random_links(T, L, 0.3, 2700)
    nsite = dom[1] * L ** 3
    b = gaussian_field(nsite, 12, 2701)
    b[6:] = 0
    for j in range(6, 12):
        b[j, (j * 977) % nsite, j] = 1.0
    Ud, bd = dd.pack_links(U), dd.pack_field(b)
    p = dd.solver_params(tol=1e-10, prec=dd.DD_MIXED, solver=solver)
    tail = f"12:{L}:{T}:{dom[1]}:0"
    xs, its = [], []
    # bl: tile flags, bit 0 brick tiles, bit 1 the time chunks of a tile in adjacent workgroups,
    # bit 2 non-temporal output stores (two columns per thread)
    for tc, remap, kc, bl in [(2, 0, 1, 0), (2, 1, 1, 0), (2, 0, 2, 0), (2, 1, 2, 0), (4, 1, 2, 0), (2, 0, 1, 1),
                              (4, 1, 2, 1), (2, 1, 1, 2), (2, 1, 2, 2), (1, 0, 2, 3), (2, 1, 2, 3), (2, 1, 2, 4),
                              (2, 1, 2, 7)]:
        path = tmp_path / f"shapes_{tc}_{remap}_{kc}_{bl}.txt"
        path.write_text(f"eo:0:{tail} 256 {tc} {remap} 1 {bl}\neo:1:{tail} 256 {tc} {remap} {kc} {bl}\n")
        monkeypatch.setenv("DD_TUNE_CACHE", str(path))
        ctx = dd.Context(T, L, bc)
        x, stats = dd.block_solve(ctx, Ud, kappa, bd, dom, p)
        assert max(stats["true_rel_resid"]) <= p.tol
        xs.append(x)
        its.append(stats["iters"])
    assert torch.equal(xs[1], xs[0])
    # non-temporal stores change a cache policy, nothing in the arithmetic
    assert torch.equal(xs[11], xs[3]) and torch.equal(xs[12], xs[10])
    for x, it in zip(xs[2:], its[2:]):
        assert relerr(dd.unpack_field(x), dd.unpack_field(xs[0])) < 1e-8
        assert abs(it - its[0]) <= 4


def test_two_row_links_only_for_su3(tmp_path, monkeypatch):
    """FP32 half hops with two columns per thread read every link as its first
    two rows (the third rebuilt as their conjugated cross product) only when the
    links are SU(3); links scaled by 1.05 are not, keep all nine entries, and
    both mixed solves reach the oracle's solution."""
    dd = lib()
    step("two-row FP32 links")
    T, L, bc, dom, kappa = 16, 8, -1, (4, 8), 0.13
    U = random_links(T, L, 0.3, 2800)
    b = gaussian_field(dom[1] * L ** 3, 4, 2801)
    tail = f"4:{L}:{T}:{dom[1]}:0"
    path = tmp_path / "shapes.txt"
    path.write_text(f"eo:0:{tail} 256 2 0 1 0\neo:1:{tail} 256 2 0 2 0\n")
    monkeypatch.setenv("DD_TUNE_CACHE", str(path))
    for scale in (1.0, 1.05):
        Us = U * scale
        ctx = dd.Context(T, L, bc)
        dd.set_kernel_timing(ctx, True)
        x, st = dd.block_solve(ctx, dd.pack_links(Us), kappa, dd.pack_field(b), dom,
                               dd.solver_params(tol=1e-10, prec=dd.DD_MIXED))
        assert max(st["true_rel_resid"]) <= 1e-10
        names = list(dd.kernel_timing(ctx))
        two_row = [n for n in names if n.startswith("k_eo_hop<float") and n.endswith(", 2, true>")]
        full = [n for n in names if n.startswith("k_eo_hop<float") and n.endswith(", 2, false>")]
        assert (len(two_row) > 0, len(full) > 0) == ((True, False) if scale == 1.0 else (False, True)), names
        ref, _, _, ost = O.solve(Us, kappa, T, L, bc, b, dom=dom, tol=1e-13, method=1)
        assert ost == 0
        assert relerr(dd.unpack_field(x), ref) < 1e-6


def test_even_odd_adjoint_and_fallback():
    """D^+ solves go through the even-odd path too; an odd time extent on a whole
    lattice (not bipartite) falls back to the full operator and still converges."""
    dd = lib()
    step("even-odd adjoint + odd-T fallback")
    T, L, bc, kappa = 8, 4, -1, 0.13
    U = random_links(T, L, 0.3, 2600)
    b = gaussian_field(T * L ** 3, 2, 2601)
    ctx = dd.Context(T, L, bc)
    Ud = dd.pack_links(U)
    p = dd.solver_params(tol=1e-12)
    x, _ = dd.block_solve(ctx, Ud, kappa, dd.pack_field(b), None, p)
    g = gaussian_field(T * L ** 3, 2, 2602)
    gb, _, _ = dd.block_solve_backward(ctx, Ud, kappa, x, dd.pack_field(g), None, p)
    lam = dd.unpack_field(gb)
    assert relerr(O.gamma5(O.apply_dirac(U, kappa, T, L, bc, O.gamma5(lam))), g) < 1e-11
    T2 = 7
    U2 = random_links(T2, L, 0.3, 2603)
    b2 = gaussian_field(T2 * L ** 3, 2, 2604)
    ctx2 = dd.Context(T2, L, bc)
    x2, st2 = dd.block_solve(ctx2, dd.pack_links(U2), kappa, dd.pack_field(b2), None, p)
    assert max(st2["true_rel_resid"]) <= 1e-12
    ref, _, _, _ = O.solve(U2, kappa, T2, L, bc, b2, tol=1e-13, method=1)
    assert relerr(dd.unpack_field(x2), ref) < 1e-10


def test_solves_and_factorised_at_64x32():
    """The bench's configuration (64x32^3, eps 0.15, kappa 0.135, 12 point sources at the
    origin; the pion correlator against a plain sum of |S|^2 per slice): the slab solves on
    [0, 16) in FP64 and mixed precision leave a true residual
    b - D_Lambda x within tol, checked with the full-operator stencil (not the even-odd path
    that solved), and agree with each other; every slab of the four-slab factorised
    propagator satisfies its equation of the chain, D_Lk psi_k = eta on the source slab and
    D_Lk psi_k = -sum_j D_{Lk,Lj} psi_j from the slabs one step closer to the source."""
    from paper_1612_06424_amd.inputs import WORKLOADS
    dd = lib()
    w = WORKLOADS["64x32^3"]
    T, L, kappa = w["T"], w["L"], w["kappa"]
    L3 = L ** 3
    step("solves and factorised propagator 64x32^3")
    U = dd.pack_links(random_links(T, L, w["eps"], w["link_seed"]))
    ctx = dd.Context(T, L, w["bc"])
    dom = (0, 16)
    eta = torch.zeros((12, 12, 16 * L3), dtype=torch.complex128, device="cuda")
    for j in range(12):
        eta[j, j, 0] = 1.0
    xs = {}
    for prec in (dd.DD_FP64, dd.DD_MIXED):
        p = dd.solver_params(tol=w["tol"], max_iter=20000, prec=prec, solver=dd.DD_CGNR)
        x, st = dd.block_solve(ctx, U, kappa, eta, dom, p)
        r = eta - dd.apply_dirac(ctx, U, kappa, x, dom)
        rel = torch.linalg.vector_norm(r.reshape(12, -1), dim=1) / torch.linalg.vector_norm(eta.reshape(12, -1), dim=1)
        assert rel.max().item() <= 2 * w["tol"], (prec, rel.max().item())
        xs[prec] = x
    nx = torch.linalg.vector_norm(xs[dd.DD_FP64])
    assert (torch.linalg.vector_norm(xs[dd.DD_MIXED] - xs[dd.DD_FP64]) / nx).item() < 1e-8
    del xs, eta
    # the factorised propagator and its chain: slab 0 holds the source, slabs 1 and 3 are fed
    # by slab 0 (3 across the antiperiodic time edge), slab 2 by slabs 1 and 3
    doms = w["domains"]
    p = dd.solver_params(tol=w["tol"], max_iter=20000, prec=dd.DD_MIXED, solver=dd.DD_CGNR)
    Sf, _, _ = dd.factorized_propagator(ctx, U, kappa, w["sources"][0], doms, p)
    # the pion correlator of it (source slice 0) against a plain sum of |S|^2 per slice
    C = dd.pion_correlator(ctx, Sf, 0)
    Cref = (Sf.real ** 2 + Sf.imag ** 2).reshape(144, T, L3).sum(dim=(0, 2)).cpu().numpy()
    assert np.abs(C - Cref).max() < 1e-12 * Cref.max()
    psi = [Sf[:, :, t0 * L3:(t0 + nt) * L3].contiguous() for t0, nt in doms]
    del Sf
    feeds = {0: [], 1: [0], 3: [0], 2: [1, 3]}
    for k, (t0, nt) in enumerate(doms):
        r = dd.apply_dirac(ctx, U, kappa, psi[k], doms[k])
        if k == 0:
            b = torch.zeros_like(r)
            for j in range(12):
                b[j, j, 0] = 1.0
            r = r - b
        else:
            b = torch.zeros_like(r)
            for j in feeds[k]:
                dd.frontier_hop(ctx, U, doms[k], doms[j], psi[j], b, -1.0)
            r = r - b
        rel = (torch.linalg.vector_norm(r) / torch.linalg.vector_norm(b)).item()
        assert rel <= 4 * w["tol"], (k, rel)


def test_force_at_32x16():
    """The bench's force workload (32x16^3, Dirichlet time, one Gaussian field): the link
    force from the adjoint solve against a central difference of the action along
    U + h i X U, X a random hermitian traceless field on every link (FP64 solves at tol
    1e-12, h = 1e-4); PyTorch's complex convention makes the derivative
    Re sum conj(grad_U) i X U."""
    from paper_1612_06424_amd.inputs import WORKLOADS
    dd = lib()
    w = WORKLOADS["force-32x16^3"]
    T, L, kappa = w["T"], w["L"], w["kappa"]
    V = T * L ** 3
    step("force 32x16^3")
    U0 = dd.pack_links(random_links(T, L, w["eps"], w["link_seed"]))
    phi = dd.pack_field(gaussian_field(V, 1, w["phi_seed"]))
    ctx = dd.Context(T, L, w["bc"])
    p = dd.solver_params(tol=1e-12, max_iter=20000, prec=dd.DD_FP64, solver=dd.DD_CGNR)
    Ug = U0.clone().requires_grad_(True)
    S = dd.DomainActionFn.apply(Ug, phi, ctx, kappa, None, p)
    S.backward()
    g = Ug.grad
    gen = torch.Generator(device="cuda")
    gen.manual_seed(w["fd_seed"])
    A = torch.randn((V, 4, 3, 3), dtype=torch.complex128, device="cuda", generator=gen)
    X = 0.5 * (A + A.conj().transpose(-1, -2))
    X = X - torch.diagonal(X, dim1=-2, dim2=-1).sum(-1)[..., None, None] / 3 * torch.eye(3, device="cuda")
    Un = U0.permute(2, 0, 1).reshape(V, 4, 3, 3)
    dU = (1j * (X @ Un)).reshape(V, 4, 9).permute(1, 2, 0).contiguous()
    pred = (g.conj() * dU).real.sum().item()
    h = 1e-4
    Sp, _, _, _ = dd.domain_action(ctx, (U0 + h * dU).contiguous(), kappa, phi, None, p)
    Sm, _, _, _ = dd.domain_action(ctx, (U0 - h * dU).contiguous(), kappa, phi, None, p)
    fd = (Sp - Sm) / (2 * h)
    assert abs(pred) > 1e-6 * abs(S.item())
    assert abs(fd - pred) <= 1e-6 * abs(pred), (fd, pred)
