"""GPU parity of the factorised nucleon contraction (Sec. 4.2, Eqs. 22-26) against the oracle:
the baryon blocks (Eq. 25) on one and several site chunks, the contraction (Eqs. 23-24), the
quark-line factors xi and eta (Eq. 26) in FP64 and mixed precision, the chain end to end, error
paths, and sampled blocks at the 32^3 slice size with 120 vectors.

Bars: blocks and contraction on identical inputs within 1e-12 of the largest entry (no solves);
lines and the chain within 1e-10 (FP64) / 1e-6 (mixed) as for the other solves.
"""
import os

import numpy as np
import pytest
import torch

import oracle as O
from helpers import gaussian_field, lib, random_links, relerr, step

pytestmark = pytest.mark.gpu

EPS = np.zeros((3, 3, 3))
for _a, _b, _c in ((0, 1, 2), (1, 2, 0), (2, 0, 1)):
    EPS[_a, _b, _c], EPS[_b, _a, _c] = 1.0, -1.0


def _blocks_to_oracle(B):
    """device [t][k][alpha][i][j] -> oracle (t, i, j, k, alpha)"""
    return B.cpu().numpy().transpose(0, 3, 4, 1, 2)


def _blocks_to_dev(B):
    return torch.as_tensor(np.ascontiguousarray(B.transpose(0, 3, 4, 1, 2))).to("cuda")


@pytest.mark.parametrize("n,nt,L,chunk", [(1, 2, 4, None), (5, 3, 4, None), (13, 2, 4, None), (13, 2, 4, 24),
                                         (7, 1, 6, 50)])
def test_baryon_blocks_vs_oracle(n, nt, L, chunk):
    dd = lib()
    step(f"baryon blocks n={n} nt={nt} L={L} chunk={chunk}")
    ctx = dd.Context(8, L, -1)
    s = gaussian_field(nt * L ** 3, n, 4000 + n)
    ref = O.baryon_blocks(L, s)
    if chunk:
        os.environ["DD_BLOCK_CHUNK"] = str(chunk)
    try:
        B = dd.baryon_blocks(ctx, dd.pack_field(s))
        torch.cuda.synchronize()
    finally:
        os.environ.pop("DD_BLOCK_CHUNK", None)
    got = _blocks_to_oracle(B)
    assert np.abs(got - ref).max() < 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("n,ntx,nty", [(4, 1, 3), (9, 2, 5)])
def test_nucleon_contract_vs_oracle(n, ntx, nty):
    dd = lib()
    step(f"nucleon contract n={n} ntx={ntx} nty={nty}")
    ctx = dd.Context(8, 4, -1)
    rng = np.random.default_rng(4100 + n)
    Bx = rng.standard_normal((ntx, n, n, n, 4)) + 1j * rng.standard_normal((ntx, n, n, n, 4))
    By = rng.standard_normal((nty, n, n, n, 4)) + 1j * rng.standard_normal((nty, n, n, n, 4))
    W1r, W2r, _ = O.nucleon_factorized(4, Bx, By)
    W1, W2 = dd.nucleon_contract(ctx, _blocks_to_dev(Bx), _blocks_to_dev(By))
    scale = max(np.abs(W1r).max(), np.abs(W2r).max())
    assert np.abs(W1 - W1r).max() < 1e-12 * scale
    assert np.abs(W2 - W2r).max() < 1e-12 * scale


CASES = {
    # bc, gbar, gstar, t_phi, x0
    "dirichlet": (0, (0, 10), (8, 8), 7, 2),
    "antiperiodic": (-1, (0, 10), (8, 8), 7, 3),
    "backward": (-1, (6, 10), (0, 6), 6, 12),     # gstar = [0, 6), cut on the slice after it
}


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("case", sorted(CASES))
def test_nucleon_lines_and_chain_vs_oracle(case, prec):
    dd = lib()
    step(f"nucleon lines {case} {prec}")
    T, L, kappa = 16, 4, 0.13
    L3 = L ** 3
    bc, gbar, gstar, t_phi, x0 = CASES[case]
    U = random_links(T, L, 0.3, 4200)
    nvec = 14
    pi = ((t_phi - 2) % T, 5)
    sign = +1 if (t_phi + 1) % T == gstar[0] else -1
    v0 = gaussian_field(5 * L3, nvec, 4201)
    phi, _ = O.projection_basis(U, kappa, T, L, bc, pi, t_phi, sign, v0, 2, tol=1e-13)
    xi_r, eta_r = O.nucleon_lines(U, kappa, T, L, bc, gbar, gstar, t_phi, phi, x0, tol=1e-13)
    ctx = dd.Context(T, L, bc)
    p = dd.solver_params(tol=1e-13 if prec == "fp64" else 1e-10, max_iter=20000,
                         prec=dd.DD_FP64 if prec == "fp64" else dd.DD_MIXED, solver=dd.DD_CGNR)
    bar = 1e-10 if prec == "fp64" else 1e-6
    xi, eta, stats = dd.nucleon_lines(ctx, dd.pack_links(U), kappa, gbar, gstar, t_phi, dd.pack_field(phi), x0, p)
    assert relerr(dd.unpack_field(xi), xi_r) < bar
    assert relerr(dd.unpack_field(eta), eta_r) < bar
    assert all(s["nrhs"] == nvec and s["iters"] > 0 and max(s["true_rel_resid"]) <= p.tol for s in stats)
    # the chain: blocks of xi (one slice) and eta (every slice of gstar), contracted
    W1r, W2r, _ = O.nucleon_factorized(L, O.baryon_blocks(L, xi_r), O.baryon_blocks(L, eta_r))
    W1, W2 = dd.nucleon_contract(ctx, dd.baryon_blocks(ctx, xi), dd.baryon_blocks(ctx, eta))
    scale = max(np.abs(W1r).max(), np.abs(W2r).max())
    assert np.abs(W1 - W1r).max() < bar * scale * 10
    assert np.abs(W2 - W2r).max() < bar * scale * 10


def test_nucleon_errors():
    dd = lib()
    step("nucleon errors")
    T, L = 16, 4
    ctx = dd.Context(T, L, 0)
    U = dd.pack_links(random_links(T, L, 0.3, 4300))
    phi = torch.zeros((4, 12, L ** 3), dtype=torch.complex128, device="cuda")
    for gbar, gstar, t_phi, x0 in (((0, 10), (8, 8), 8, 2),     # t_phi inside gstar
                                   ((0, 10), (9, 7), 5, 2),     # not a neighbour of gstar
                                   ((0, 10), (8, 8), 7, 12),    # x0 outside gbar
                                   ((8, 8), (0, 8), 15, 9)):    # neighbour only across a Dirichlet edge
        with pytest.raises(dd.DDError) as e:
            dd.nucleon_lines(ctx, U, 0.13, gbar, gstar, t_phi, phi, x0)
        assert e.value.status == dd.DD_ERR_ARG
    s = torch.zeros((3, 12, L ** 3), dtype=torch.complex128, device="cuda")
    big = torch.zeros((300, 12, L ** 3), dtype=torch.complex128, device="cuda")
    with pytest.raises(dd.DDError) as e:
        dd.baryon_blocks(ctx, big)
    assert e.value.status == dd.DD_ERR_ARG
    st = dd._lib.dd_baryon_blocks(ctx._h, 3, 1, s.data_ptr(), s.data_ptr())  # B on top of s
    assert st == dd.DD_ERR_ARG


def test_sampled_blocks_at_the_32_cubed_slice():
    """120 vectors on one 32^3 slice (the bench's shape, several site chunks): sampled
    entries against sums the oracle's definition gives one by one, and the (i, j) symmetry."""
    dd = lib()
    step("baryon blocks 120 vectors 32^3")
    L, n = 32, 120
    L3 = L ** 3
    ctx = dd.Context(4, L, 0)
    g = torch.Generator(device="cuda")
    g.manual_seed(4400)
    s = torch.randn((n, 12, L3), dtype=torch.complex128, device="cuda", generator=g)
    B = dd.baryon_blocks(ctx, s)
    torch.cuda.synchronize()
    Bh = B[0]                                          # [k][alpha][i][j]
    assert (torch.linalg.vector_norm(Bh - Bh.transpose(2, 3)) / torch.linalg.vector_norm(Bh)).item() < 1e-12
    q = s.cpu().numpy().reshape(n, 4, 3, L3)           # [vector][spin][colour][site]
    cg5 = O.charge_conjugation() @ O.gamma_matrices()[4]
    rng = np.random.default_rng(4401)
    for _ in range(12):
        i, j, k = (int(v) for v in rng.integers(0, n, 3))
        al = int(rng.integers(0, 4))
        want = np.einsum("abc,rax,rs,sbx,cx->", EPS, q[i], cg5, q[j], q[k, al], optimize=True)
        got = Bh[k, al, i, j].item()
        assert abs(got - want) < 1e-12 * np.sqrt(6 * 16 * L3) * 4, (i, j, k, al, got, want)


def test_the_maximum_vector_count():
    """256 vectors (the largest basis): blocks on one 4^3 slice sampled against sums from the
    definition (the pair index reaches 256 * 257 / 2 - 1 and every (i, j) order is unpacked),
    and the contraction of random 256-vector blocks against the oracle."""
    dd = lib()
    step("nucleon 256 vectors")
    L, n = 4, 256
    L3 = L ** 3
    ctx = dd.Context(8, L, -1)
    s = gaussian_field(L3, n, 4500)
    B = dd.baryon_blocks(ctx, dd.pack_field(s))[0].cpu().numpy()   # [k][alpha][i][j]
    q = s.reshape(n, L3, 4, 3)
    cg5 = O.charge_conjugation() @ O.gamma_matrices()[4]
    rng = np.random.default_rng(4501)
    idx = [tuple(int(v) for v in rng.integers(0, n, 3)) + (int(rng.integers(0, 4)),) for _ in range(16)]
    idx += [(0, n - 1, n - 1, 3), (n - 1, n - 1, 0, 0), (n - 1, 0, n - 2, 1), (n - 2, n - 1, 7, 2)]
    for i, j, k, al in idx:
        want = np.einsum("abc,xra,rs,xsb,xc->", EPS, q[i], cg5, q[j], q[k, :, al, :], optimize=True)
        assert abs(B[k, al, i, j] - want) < 1e-12 * max(1.0, abs(want)) * 10, (i, j, k, al)
    assert np.abs(B - B.transpose(0, 1, 3, 2)).max() < 1e-12 * np.abs(B).max()
    del B
    Bx = rng.standard_normal((1, n, n, n, 4)) + 1j * rng.standard_normal((1, n, n, n, 4))
    By = rng.standard_normal((1, n, n, n, 4)) + 1j * rng.standard_normal((1, n, n, n, 4))
    W1r, W2r, _ = O.nucleon_factorized(L, Bx, By)
    W1, W2 = dd.nucleon_contract(ctx, _blocks_to_dev(Bx), _blocks_to_dev(By))
    scale = max(np.abs(W1r).max(), np.abs(W2r).max())
    assert np.abs(W1 - W1r).max() < 1e-11 * scale and np.abs(W2 - W2r).max() < 1e-11 * scale


def test_the_maximum_vector_count_on_a_32_cubed_slice():
    """256 vectors on one 32^3 slice: the largest pair count (32 896 rows of the block product)
    at the bench's slice size, so the site chunks are short (the diquarks of a chunk stay
    below 2 GiB: 25 chunks of at most 1360 sites, each accumulated onto the previous ones) and
    every row and column tile of the product is full or ragged at its edge.  Sampled entries,
    including the last pairs and the last spin-vector column, against sums from the definition,
    and the (i, j) symmetry."""
    dd = lib()
    step("baryon blocks 256 vectors 32^3")
    L, n = 32, 256
    L3 = L ** 3
    ctx = dd.Context(4, L, 0)
    g = torch.Generator(device="cuda")
    g.manual_seed(4600)
    s = torch.randn((n, 12, L3), dtype=torch.complex128, device="cuda", generator=g)
    B = dd.baryon_blocks(ctx, s)
    torch.cuda.synchronize()
    Bh = B[0]                                          # [k][alpha][i][j]
    rng = np.random.default_rng(4601)
    idx = [tuple(int(v) for v in rng.integers(0, n, 3)) + (int(rng.integers(0, 4)),) for _ in range(10)]
    idx += [(n - 1, n - 1, n - 1, 3), (0, n - 1, n - 2, 2), (n - 2, n - 1, 0, 1)]
    cg5 = O.charge_conjugation() @ O.gamma_matrices()[4]
    for i, j, k, al in idx:
        q = s[[i, j, k]].cpu().numpy().reshape(3, 4, 3, L3)   # [vector][spin][colour][site]
        want = np.einsum("abc,rax,rs,sbx,cx->", EPS, q[0], cg5, q[1], q[2, al], optimize=True)
        got = Bh[k, al, i, j].item()
        assert abs(got - want) < 1e-12 * np.sqrt(6 * 16 * L3) * 4, (i, j, k, al, got, want)
        assert abs(Bh[k, al, j, i].item() - got) < 1e-12 * max(1.0, abs(got))
