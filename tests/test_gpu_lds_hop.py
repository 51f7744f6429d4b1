"""GPU parity of the LDS-tile form of the FP32 even-odd half hop (dd_eo_lds.h).

The form is chosen through the launch-shape cache (DD_TUNE_CACHE, tile flag bit 3 with kc
columns per workgroup), so each case runs it on purpose: mixed-precision solves with both
methods (CGNR: the Schur operator and its adjoint with the norm epilogue; BiCGStab: the
<r^, v> and <t, s>, |t|^2 epilogues) reach the oracle's solution, on L = 16 and L = 32
fields (whole lattices with antiperiodic and Dirichlet time, slabs, one across the time
edge), with 12, 5 (a ragged last group) and 1 column per workgroup, XCD-remapped or not,
plain or non-temporal stores.  Gaussian and point sources stop at different iterations, so
stopped columns share workgroups with running ones, whose launches must leave the stopped
columns' vectors as they were.  The kernel timing names show that the LDS form ran.
"""
import numpy as np
import pytest

import oracle as O
from helpers import gaussian_field, lib, random_links, relerr, step

pytestmark = pytest.mark.gpu


def _sources(nsite, seed):
    b = gaussian_field(nsite, 12, seed)
    b[6:] = 0
    for j in range(6, 12):
        b[j, (j * 977) % nsite, j] = 1.0
    return b


CASES = [  # T, L, bc, dom, cpw, remap, nts
    (8, 16, -1, (2, 4), 12, 1, 0),
    (8, 16, -1, (6, 4), 5, 0, 1),     # a slab across the time edge
    (4, 16, -1, None, 1, 1, 1),       # whole lattice, antiperiodic
    (6, 16, 0, None, 12, 0, 0),       # whole lattice, Dirichlet time walls
    (4, 32, -1, (1, 2), 12, 1, 1),    # the bench's L = 32 bricks
]


@pytest.mark.parametrize("solver", [0, 1])
@pytest.mark.parametrize("T,L,bc,dom,cpw,remap,nts", CASES)
def test_lds_half_hop_solves_vs_oracle(T, L, bc, dom, cpw, remap, nts, solver, tmp_path, monkeypatch):
    dd = lib()
    step(f"LDS half hop T={T} L={L} bc={bc} dom={dom} cpw={cpw} remap={remap} nts={nts} solver={solver}")
    kappa = 0.13
    U = random_links(T, L, 0.3, 3100 + T + L)
    nt = T if dom is None else dom[1]
    nsite = nt * L ** 3
    b = _sources(nsite, 3101)
    whole = 1 if dom is None else 0
    path = tmp_path / "shapes.txt"
    path.write_text(f"eo:1:12:{L}:{T}:{nt}:{whole} 256 1 {remap} {cpw} {8 | (4 if nts else 0)}\n")
    monkeypatch.setenv("DD_TUNE_CACHE", str(path))
    ctx = dd.Context(T, L, bc)
    dd.set_kernel_timing(ctx, True)
    p = dd.solver_params(tol=1e-10, prec=dd.DD_MIXED, solver=solver)
    x, st = dd.block_solve(ctx, dd.pack_links(U), kappa, dd.pack_field(b), dom, p)
    names = list(dd.kernel_timing(ctx))
    assert any(n.startswith("k_eo_lds<float") for n in names), names
    assert max(st["true_rel_resid"]) <= 1e-10
    cols = list(range(12)) if L < 32 else [0, 5, 6, 11]  # the oracle's time at L = 32
    ref, _, _, ost = O.solve(U, kappa, T, L, bc, b[cols], dom=dom, tol=1e-13, method=0)
    assert ost == 0
    assert relerr(dd.unpack_field(x)[cols], ref) < 1e-6


def test_lds_half_hop_matches_the_time_sweep(tmp_path, monkeypatch):
    """The same mixed solve with the LDS form and with the time-sweep form: the two
    differ only in rounding (both reach tol with iteration counts within a few)."""
    dd = lib()
    T, L, bc, dom = 8, 16, -1, (2, 4)
    step("LDS half hop vs time sweep")
    U = random_links(T, L, 0.3, 3200)
    b = _sources(dom[1] * L ** 3, 3201)
    Ud, bd = dd.pack_links(U), dd.pack_field(b)
    xs, its = [], []
    for entry in ("256 1 1 12 8", "256 2 1 2 4"):
        path = tmp_path / f"s{len(xs)}.txt"
        path.write_text(f"eo:1:12:{L}:{T}:{dom[1]}:0 {entry}\n")
        monkeypatch.setenv("DD_TUNE_CACHE", str(path))
        ctx = dd.Context(T, L, bc)
        x, st = dd.block_solve(ctx, Ud, 0.13, bd, dom, dd.solver_params(tol=1e-10, prec=dd.DD_MIXED))
        assert max(st["true_rel_resid"]) <= 1e-10
        xs.append(dd.unpack_field(x))
        its.append(st["iters"])
    assert relerr(xs[0], xs[1]) < 1e-8
    assert abs(its[0] - its[1]) <= 6, its
