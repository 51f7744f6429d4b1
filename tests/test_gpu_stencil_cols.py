"""Launch shapes of the full Wilson-Dirac stencil: several columns per thread (one link
load serves KC columns; FP32 KC = 1..4, FP64 KC = 1..2), brick tiles and the order of tiles
and chunks.

The shape is forced through the launch-shape cache (DD_TUNE_CACHE: key
"kind:ncol:L:T:nt:whole", then workgroup size, chunk length, XCD remap, KC and tile
flags).  Every site's arithmetic is the same whatever the shape, so the output is bitwise
the same for all of them, and within 1e-13 (FP64) / 2e-6 (FP32) of the oracle's D.  Where L
divides 64 the x hops come from neighbouring lanes unless tile flag bit 2 asks for the
loading form: the same products, but the compiler contracts the last multiply of a loaded
backward hop into the accumulation, which a hop handed over by another lane cannot be, so
the two forms agree to rounding (1e-14 / 1e-6) and each is bitwise the same over the shapes.  Inside
the unpreconditioned solves every epilogue of the stencil runs with columns that stop at
different iterations sharing workgroups with running ones: the solutions and iteration
counts must not change with KC either.
"""
import numpy as np
import pytest
import torch

import oracle as O
from helpers import gaussian_field, lib, random_links, step

pytestmark = pytest.mark.gpu

CASES = [
    # T, L, bc, dom: whole lattices and slabs (one across the time wrap); L^3 = 216 and 125
    # leave a ragged tail in the last 256-site tile; L = 8 and 16 take brick tiles
    (16, 4, -1, None),
    (8, 6, -1, None),
    (16, 4, -1, (12, 8)),
    (10, 5, 0, (3, 4)),
    (8, 8, -1, None),
    (8, 16, -1, (6, 4)),
]
# workgroup size, chunk length, XCD remap, tile flags (bit 0 bricks, bit 1 chunk-adjacent order,
# bit 2 the x hops loaded rather than taken from neighbouring lanes where L divides 64)
SHAPES = [(256, 4, 1, 0), (128, 3, 0, 0), (256, 2, 1, 1), (128, 4, 0, 3), (256, 1, 1, 2), (256, 4, 1, 4),
          (128, 2, 0, 5)]


def _maxrel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


def _cache(tmp_path, monkeypatch, name, lines):
    path = tmp_path / name
    path.write_text("".join(f"{k} {v}\n" for k, v in lines))
    monkeypatch.setenv("DD_TUNE_CACHE", str(path))


def _key(kind, ncol, T, L, dom):
    nt, whole = (T, 1) if dom is None else (dom[1], 0)
    return f"{kind}:{ncol}:{L}:{T}:{nt}:{whole}"


@pytest.mark.parametrize("T,L,bc,dom", CASES)
def test_columns_per_thread_and_tiles_vs_oracle(tmp_path, monkeypatch, T, L, bc, dom):
    """Every launch shape (columns per thread, workgroup size, chunk length, remap, brick
    tiles, chunk-adjacent order) gives bitwise the same D psi, within the oracle's bar."""
    dd = lib()
    ncol = 12
    kappa = 0.1287
    U = random_links(T, L, 0.4, 4100 + T + L)
    nsite = (T if dom is None else dom[1]) * L ** 3
    psi = gaussian_field(nsite, ncol, 4101)
    ref = O.apply_dirac(U, kappa, T, L, bc, psi, dom)
    lanes_ok = L >= 4 and 64 % L == 0
    for kind, dtype, kcs, tol in ((0, torch.complex128, (1, 2), 1e-13), (1, torch.complex64, (1, 2, 3, 4), 2e-6)):
        first = {}
        for kc in kcs:
            for nt, tc, remap, bl in SHAPES:
                step(f"stencil KC={kc} kind={kind} T={T} L={L} dom={dom} shape=({nt},{tc},{remap},{bl})")
                _cache(tmp_path, monkeypatch, f"s_{kind}_{kc}_{nt}_{tc}_{remap}_{bl}.txt",
                       [(_key(kind, ncol, T, L, dom), f"{nt} {tc} {remap} {kc} {bl}")])
                ctx = dd.Context(T, L, bc)
                dd.set_kernel_timing(ctx, True)
                out = dd.apply_dirac(ctx, dd.pack_links(U, dtype), kappa, dd.pack_field(psi, dtype), dom)
                torch.cuda.synchronize()
                names = list(dd.kernel_timing(ctx))
                want = f"k_dslash<{'double' if kind == 0 else 'float'}, 0, 0, {nt}" + (f", {kc}>" if kc > 1 else ">")
                assert names == [want], names
                assert _maxrel(dd.unpack_field(out), ref) < tol
                form = "lanes" if lanes_ok and not (bl & 4) else "loads"
                first.setdefault(form, out)
                assert torch.equal(out, first[form]), (kind, kc, nt, tc, remap, bl)
        if len(first) == 2:
            assert _maxrel(dd.unpack_field(first["lanes"]), dd.unpack_field(first["loads"])) < (1e-14 if kind == 0 else 1e-6)


@pytest.mark.parametrize("solver", ["bicgstab", "cgnr"])
def test_unpreconditioned_solves_do_not_depend_on_columns_per_thread(tmp_path, monkeypatch, solver):
    dd = lib()
    T, L, bc, dom, kappa = 16, 6, -1, (2, 8), 0.125
    ncol = 12
    U = random_links(T, L, 0.3, 4200)
    nsite = dom[1] * L ** 3
    b = gaussian_field(nsite, ncol, 4201)
    b[6:] = 0
    for j in range(6, 12):
        b[j, (j * 577) % nsite, j] = 1.0  # point sources stop at other iterations than Gaussian ones
    Ud, bd = dd.pack_links(U), dd.pack_field(b)
    method = dd.DD_BICGSTAB if solver == "bicgstab" else dd.DD_CGNR
    res = []
    for kc64, kc32 in ((1, 1), (2, 4), (2, 3), (1, 2)):
        step(f"unpreconditioned {solver} KC fp64={kc64} fp32={kc32}")
        _cache(tmp_path, monkeypatch, f"sol_{kc64}_{kc32}.txt",
               [(_key(0, ncol, T, L, dom), f"256 4 1 {kc64} 0"), (_key(1, ncol, T, L, dom), f"256 4 1 {kc32} 0")])
        # (the reductions' grouping depends on the tile shape and order, not on KC)
        ctx = dd.Context(T, L, bc)
        p = dd.solver_params(tol=1e-10, prec=dd.DD_MIXED, solver=method, precond=dd.DD_PRECOND_NONE)
        x, st = dd.block_solve(ctx, Ud, kappa, bd, dom, p)
        assert max(st["true_rel_resid"]) <= 1e-10
        res.append((x, st["iters"], st["updates"]))
    x0 = O.solve(U, kappa, T, L, bc, b, dom=dom, tol=1e-12, method=0)[0]
    assert _maxrel(dd.unpack_field(res[0][0]), x0) < 1e-8
    for x, it, up in res[1:]:
        assert torch.equal(x, res[0][0])
        assert (it, up) == res[0][1:]
