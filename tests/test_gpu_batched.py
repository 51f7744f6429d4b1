"""GPU parity of the batched solve of independent domains (each with its own
shape, links, kappa and number of columns) against the oracle, and a
full-size check of the 96-domain workload through the oracle's operator.

Bars: FP64 within 1e-10 of the oracle (relative field norm per domain), mixed
precision within 1e-6.  The batched inner iterations replay a captured HIP
graph many times between eager reliable updates, so every comparison below
also checks those replays.
"""
import numpy as np
import pytest
import torch

import oracle as O
from helpers import gaussian_field, lib, random_links, relerr, step
from paper_1612_06424_amd.inputs import batched_domains

pytestmark = pytest.mark.gpu

# (T, L, time_bc, kappa, ncol, eps): uneven shapes, odd and even extents,
# Dirichlet and (anti)periodic time, 1..12 columns
SMALL_BATCH = [
    (8, 4, 0, 0.125, 3, 0.3),
    (4, 6, 0, 0.13, 12, 0.3),
    (6, 4, -1, 0.128, 1, 0.3),
    (10, 5, 0, 0.132, 5, 0.25),
    (8, 6, 1, 0.12, 2, 0.3),
]
# every domain bipartite (even L; even T or Dirichlet time walls): the batch takes
# the even-odd path unless the parameters ask for the full operator
EO_BATCH = [
    (8, 4, 0, 0.125, 3, 0.3),
    (4, 6, 0, 0.13, 12, 0.3),
    (6, 4, -1, 0.128, 1, 0.3),
    (9, 4, 0, 0.132, 5, 0.25),
    (8, 6, 1, 0.12, 2, 0.3),
]


# bipartite domains whose column counts are all multiples of 4, so that the FP32
# half hop may serve 1, 2 or 4 columns per workgroup
KC_BATCH = [
    (8, 4, 0, 0.125, 4, 0.3),
    (4, 6, 0, 0.13, 12, 0.3),
    (6, 4, -1, 0.128, 4, 0.3),
    (8, 6, 1, 0.12, 8, 0.3),
]


def _items(dd, seed, batch=SMALL_BATCH):
    items, refs = [], []
    for i, (T, L, bc, kappa, ncol, eps) in enumerate(batch):
        U = random_links(T, L, eps, seed + i)
        b = gaussian_field(T * L ** 3, ncol, seed + 100 + i)
        items.append(dict(T=T, L=L, time_bc=bc, U=dd.pack_links(U), kappa=kappa, b=dd.pack_field(b),
                          x=torch.empty((ncol, 12, T * L ** 3), dtype=torch.complex128, device="cuda")))
        refs.append((U, b))
    return items, refs


@pytest.mark.parametrize("batch,precond", [("uneven", 0), ("bipartite", 0), ("bipartite", 1)])
@pytest.mark.parametrize("prec,solver", [("fp64", 1), ("mixed", 1), ("fp64", 0), ("mixed", 0)])
def test_batched_vs_oracle(prec, solver, batch, precond):
    dd = lib()
    step(f"batched {batch} precond={precond} {prec} solver={solver}")
    shapes = SMALL_BATCH if batch == "uneven" else EO_BATCH
    items, refs = _items(dd, 3000, shapes)
    ctx = dd.Context(8, 4, 0)
    p = dd.solver_params(tol=1e-12 if prec == "fp64" else 1e-10, max_iter=20000,
                         prec=dd.DD_FP64 if prec == "fp64" else dd.DD_MIXED, solver=solver, precond=precond)
    stats = dd.block_solve_batched(ctx, items, p)
    for it, (U, b), st, (T, L, bc, kappa, ncol, _) in zip(items, refs, stats, shapes):
        assert st["nrhs"] == ncol
        assert max(st["true_rel_resid"][:ncol]) <= p.tol
        ref, _, _, ost = O.solve(U, kappa, T, L, bc, b, tol=1e-13, method=1)
        assert ost == 0
        got = dd.unpack_field(it["x"])
        assert relerr(got, ref) < (1e-10 if prec == "fp64" else 1e-6), (T, L, bc)
        assert relerr(O.apply_dirac(U, kappa, T, L, bc, got), b) <= 2 * p.tol


@pytest.mark.parametrize("batch", ["uneven", "bipartite"])
def test_batched_repeatable_and_matches_single(batch):
    """Two batched solves give bitwise the same answer (graph replays are
    deterministic), and each domain agrees with its own single-domain solve."""
    dd = lib()
    step(f"batched repeat + single ({batch})")
    shapes = SMALL_BATCH if batch == "uneven" else EO_BATCH
    items, refs = _items(dd, 3100, shapes)
    ctx = dd.Context(8, 4, 0)
    p = dd.solver_params(tol=1e-12, prec=dd.DD_MIXED)
    dd.block_solve_batched(ctx, items, p)
    first = [it["x"].clone() for it in items]
    dd.block_solve_batched(ctx, items, p)
    for a, it in zip(first, items):
        assert torch.equal(a, it["x"])
    for it, (T, L, bc, kappa, ncol, _) in zip(items, shapes):
        sctx = dd.Context(T, L, bc)
        x, _ = dd.block_solve(sctx, it["U"], kappa, it["b"], None, p)
        assert relerr(dd.unpack_field(x), dd.unpack_field(it["x"])) < 1e-9


@pytest.mark.parametrize("solver", [0, 1])
def test_batched_launch_shapes_bitwise(solver, tmp_path, monkeypatch):
    """The XCD remap of the batched half hop gives bitwise the same mixed
    solution; columns per workgroup, the chunk length and the tile shape change
    the rounding only (agreement to 1e-8, iteration counts within a few).  Columns of a
    domain stop at different iterations, so stopped and running columns share
    workgroups."""
    dd = lib()
    step(f"batched launch shapes solver={solver}")
    items, refs = _items(dd, 3200, KC_BATCH)
    sig = "".join(f":{T}x{L}x{ncol}b{bc}" for (T, L, bc, _, ncol, _) in KC_BATCH)
    p = dd.solver_params(tol=1e-10, prec=dd.DD_MIXED, solver=solver)
    results, its = [], []
    for tc, remap, kc, bl in [(2, 0, 1, 0), (2, 1, 1, 0), (2, 0, 2, 0), (2, 1, 2, 0), (4, 1, 2, 0), (2, 0, 1, 1),
                              (4, 1, 2, 1)]:
        path = tmp_path / f"shapes_{tc}_{remap}_{kc}_{bl}.txt"
        path.write_text(f"beo:0{sig} 256 {tc} {remap} 1 {bl}\nbeo:1{sig} 256 {tc} {remap} {kc} {bl}\n")
        monkeypatch.setenv("DD_TUNE_CACHE", str(path))
        ctx = dd.Context(8, 4, 0)
        stats = dd.block_solve_batched(ctx, items, p)
        for st, (_, _, _, _, ncol, _) in zip(stats, KC_BATCH):
            assert max(st["true_rel_resid"][:ncol]) <= p.tol
        results.append([it["x"].clone() for it in items])
        its.append([st["iters"] for st in stats])
    for a, b in zip(results[1], results[0]):
        assert torch.equal(a, b)
    for r, it in zip(results[2:], its[2:]):
        for a, b in zip(r, results[0]):
            assert relerr(dd.unpack_field(a), dd.unpack_field(b)) < 1e-8
        assert max(abs(i - j) for i, j in zip(it, its[0])) <= 4


def test_batched_96_domains_full_size():
    """The 96-domain workload (shapes 8x8^3 .. 16x16^3, own links and kappa, 12
    point sources each), mixed CGNR to 1e-10; sampled domains checked with the
    oracle's operator, every domain with the library's own FP64 residual; a second
    solve on the same inputs agrees with the first to 1e-9."""
    dd = lib()
    step("batched 96 domains")
    doms = batched_domains(96)
    items = []
    for d in doms:
        T, L = d["T"], d["L"]
        U = random_links(T, L, d["eps"], d["link_seed"])
        b = torch.zeros((12, 12, T * L ** 3), dtype=torch.complex128, device="cuda")
        ts, xs, ys, zs = d["source"]
        s = ((ts * L + zs) * L + ys) * L + xs
        for j in range(12):
            b[j, j, s] = 1.0
        items.append(dict(T=T, L=L, time_bc=0, U=dd.pack_links(U), kappa=d["kappa"], b=b, x=torch.empty_like(b),
                          U_nat=U))
    ctx = dd.Context(8, 8, 0)
    p = dd.solver_params(tol=1e-10, prec=dd.DD_MIXED)
    stats = dd.block_solve_batched(ctx, items, p)
    assert all(max(s["true_rel_resid"]) <= 1e-10 for s in stats)
    # the same solve again (tuned shape reused, graph captured anew).  Nearly always bitwise
    # the first; rarely (a few first solves of a context in many) one domain differed at
    # the 1e-11 level with equal iteration counts, cause not found.  The bar below is far
    # above that and far below a launch that raced on the vectors (residuals of 1e-4).
    first = [it["x"].clone() for it in items]
    stats2 = dd.block_solve_batched(ctx, items, p)
    assert all(max(s["true_rel_resid"]) <= 1e-10 for s in stats2)
    same = 0
    for k, (a, it) in enumerate(zip(first, items)):
        same += int(torch.equal(a, it["x"]))
        assert relerr(dd.unpack_field(a), dd.unpack_field(it["x"])) < 1e-9, k
    print(f"[gpu-step] repeat: {same} of {len(items)} domains bitwise equal", flush=True)
    assert max(abs(a["iters"] - b["iters"]) for a, b in zip(stats, stats2)) <= 2
    for k in (0, 17, 95):
        it, d = items[k], doms[k]
        x = dd.unpack_field(it["x"])
        b = dd.unpack_field(it["b"])
        r = O.apply_dirac(it["U_nat"], d["kappa"], d["T"], d["L"], 0, x) - b
        for j in range(12):
            assert np.linalg.norm(r[j]) <= 2e-10 * np.linalg.norm(b[j])


def test_batched_errors():
    dd = lib()
    step("batched errors")
    items, _ = _items(dd, 3200)
    ctx = dd.Context(8, 4, 0)
    bad = dict(items[0])
    bad["U"] = items[0]["U"].cpu()
    with pytest.raises(ValueError):
        dd.block_solve_batched(ctx, [bad], dd.solver_params())
    bad = dict(items[0])
    bad["kappa"] = -0.1
    with pytest.raises(dd.DDError) as e:
        dd.block_solve_batched(ctx, [items[1], bad], dd.solver_params())
    assert e.value.status == dd.DD_ERR_ARG
    bad = dict(items[0])
    bad["time_bc"] = 2
    with pytest.raises(dd.DDError) as e:
        dd.block_solve_batched(ctx, [bad], dd.solver_params())
    assert e.value.status == dd.DD_ERR_ARG
    with pytest.raises(dd.DDError) as e:
        dd.block_solve_batched(ctx, items, dd.solver_params(tol=1e-12, max_iter=2))
    assert e.value.status == dd.DD_ERR_NOCONV
