"""GPU parity of the Wilson-Dirac stencil and the frontier block against the oracle.

Element by element on the same seeded inputs: FP64 within 1e-13 (relative, max norm),
FP32 within 2e-6 of the FP64 oracle.  Lattices span several 256-site tiles and end in
ragged tails (L^3 = 216, 125); slabs include one that wraps across the time edge (where
the antiperiodic sign falls inside the slab) and a one-slice slab.
"""
import numpy as np
import pytest
import torch

import oracle as O
from helpers import gaussian_field, lib, random_links, relerr, step

pytestmark = pytest.mark.gpu

CASES = [
    # T, L, bc, dom, ncol
    (16, 4, -1, None, 12),
    (8, 6, -1, None, 3),
    (8, 6, 0, None, 1),
    (8, 6, 1, None, 2),
    (16, 4, -1, (0, 8), 12),
    (16, 4, -1, (12, 8), 5),
    (10, 5, -1, (3, 1), 2),
    (6, 5, 0, (4, 2), 4),
]


def _maxrel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


@pytest.mark.parametrize("T,L,bc,dom,ncol", CASES)
def test_stencil_fp64_fp32_vs_oracle(T, L, bc, dom, ncol):
    dd = lib()
    step(f"stencil T={T} L={L} bc={bc} dom={dom} ncol={ncol}")
    kappa = 0.1312
    U = random_links(T, L, 0.4, 1000 + T + L)
    nsite = (T if dom is None else dom[1]) * L ** 3
    psi = gaussian_field(nsite, ncol, 7)
    ref = O.apply_dirac(U, kappa, T, L, bc, psi, dom)
    ctx = dd.Context(T, L, bc)
    out = dd.apply_dirac(ctx, dd.pack_links(U), kappa, dd.pack_field(psi), dom)
    torch.cuda.synchronize()
    got = dd.unpack_field(out)
    assert _maxrel(got, ref) < 1e-13
    out32 = dd.apply_dirac(ctx, dd.pack_links(U, torch.complex64), kappa, dd.pack_field(psi, torch.complex64), dom)
    torch.cuda.synchronize()
    assert _maxrel(dd.unpack_field(out32), ref) < 2e-6


def test_stencil_is_deterministic_and_linear():
    dd = lib()
    step("stencil determinism")
    T, L, kappa = 8, 6, 0.13
    U = dd.pack_links(random_links(T, L, 0.4, 5))
    ctx = dd.Context(T, L, -1)
    a = dd.pack_field(gaussian_field(T * L ** 3, 2, 8))
    b = dd.pack_field(gaussian_field(T * L ** 3, 2, 9))
    o1 = dd.apply_dirac(ctx, U, kappa, a)
    o2 = dd.apply_dirac(ctx, U, kappa, a)
    oab = dd.apply_dirac(ctx, U, kappa, (a + 2.5 * b).contiguous())
    ob = dd.apply_dirac(ctx, U, kappa, b)
    torch.cuda.synchronize()
    assert torch.equal(o1, o2)
    assert torch.allclose(oab, o1 + 2.5 * ob, rtol=0, atol=1e-12)


@pytest.mark.parametrize("dst,src", [((8, 8), (0, 8)), ((0, 8), (8, 8)), ((4, 6), (10, 6)), ((10, 1), (4, 6))])
def test_frontier_hop_vs_oracle(dst, src):
    dd = lib()
    step(f"frontier dst={dst} src={src}")
    T, L, bc, kappa = 16, 4, -1, 0.13
    U = random_links(T, L, 0.4, 77)
    psi = gaussian_field(src[1] * L ** 3, 3, 78)
    base = gaussian_field(dst[1] * L ** 3, 3, 79)
    ref = base + 0.75 * O.block_apply(U, kappa, T, L, bc, dst, src, psi)
    ctx = dd.Context(T, L, bc)
    out = dd.pack_field(base)
    dd.frontier_hop(ctx, dd.pack_links(U), dst, src, dd.pack_field(psi), out, alpha=0.75)
    torch.cuda.synchronize()
    assert _maxrel(dd.unpack_field(out), ref) < 1e-13


def test_stencil_full_size_64x32():
    """The 64x32^3 lattice of the benchmark, FP64 one column against the oracle in full,
    FP32 twelve columns against the oracle on two of them."""
    dd = lib()
    step("stencil 64x32^3")
    T, L, bc, kappa = 64, 32, -1, 0.135
    U = random_links(T, L, 0.15, 301)
    psi = gaussian_field(T * L ** 3, 1, 302)
    ref = O.apply_dirac(U, kappa, T, L, bc, psi)
    ctx = dd.Context(T, L, bc)
    Ud = dd.pack_links(U)
    out = dd.apply_dirac(ctx, Ud, kappa, dd.pack_field(psi))
    torch.cuda.synchronize()
    assert _maxrel(dd.unpack_field(out), ref) < 1e-13
    del Ud, out
    psi12 = gaussian_field(T * L ** 3, 12, 303)
    out32 = dd.apply_dirac(ctx, dd.pack_links(U, torch.complex64), kappa, dd.pack_field(psi12, torch.complex64))
    torch.cuda.synchronize()
    for col in (0, 11):
        refc = O.apply_dirac(U, kappa, T, L, bc, psi12[col])
        got = out32[col].to(torch.complex128).cpu().numpy().T
        assert _maxrel(got, refc) < 2e-6
