"""Benchmark of the Wilson-Dirac hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

One step is one pass over every part of the hot path on synthetic inputs
already resident in HBM:
  stencil   D on the whole 64x32^3 lattice (FP64 / FP32, 1 and 12 columns) and
            D_Lambda on a 16x32^3 slab
  solves    12 point sources on the 16x32^3 slab [0,16), even-odd preconditioned
            CGNR in FP64 and in mixed precision (FP32 recursion, FP64 reliable
            updates), both to a true FP64 residual 1e-10; FP64 BiCGStab beside them
  factorised propagator across the four slabs [0,16) [16,32) [32,48) [48,64)
            (mixed solves, frontier hops) and the exact whole-lattice propagator,
            then the pion correlators C_fact(t), C_exact(t)
  overlap   (once, after the timed steps) the same factorised propagator with
            overlap regions of 8 time slices (Sec. 3.2: the slabs that feed a
            frontier are also solved on their extension) and the correction of
            its correlator
  batched   96 independent Dirichlet domains of uneven sizes, 12 sources each
  force     S = phi^+ (D^+ D)^-1 phi on a 32x16^3 Dirichlet domain and its link
            force through the hand-written adjoint (torch.autograd)
The JSON line reports the algorithmic bandwidth of the Wilson-Dirac stencil D on
the whole 64x32^3 lattice (value: bytes over time of its four launches, FP64 and
FP32, 1 and 12 columns), the aggregate over every stencil launch of the step
beside it, the per-part timings (solves with their algorithmic bytes per
iteration), the roofline of the dominant kernel (timed with HIP events on the
library's stream) and the CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6  # MI355X dense FP64 (vector and matrix cores)


def eo_iteration_bytes(nh, ncol, prec, method):
    """Algorithmic bytes of one Krylov iteration of the even-odd preconditioned solve on a field
    of nh even (= odd) sites with ncol columns: every vector read or written once per kernel,
    every link once per half hop (stored as two rows, 12 reals, in the FP32 recursion of a mixed
    solve; 18 reals in FP64).  Per even site and column, in reals:
      CGNR      4 half hops (in + out, + self in the two second halves) 240, r update 3 x 24,
                x and p update 5 x 24: 432;
      BiCGStab  4 half hops with the <r^, v> (aux) and <t, s> epilogues 264, p update 4 x 24,
                s update 3 x 24, x/r update 8 x 24: 624.
    The reliable updates (FP64 residuals every few tens of iterations) are not counted."""
    rb = 4 if prec == "mixed" else 8
    links = 96 if prec == "mixed" else 144
    per_col = 432 if method == "cgnr" else 624
    return nh * (per_col * ncol + 4 * links) * rb


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--parts", default="all", help="comma list of stencil,solve,fact,overlap,batched,force,projection,disconnected,nucleon,"
                    "overlap_study (all = every part but projection, disconnected and nucleon, which take one to a "
                    "few minutes a step; overlap_study runs once, after the timed steps, untimed)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy (10 times), the reference that scales "
                         "the profiler's FETCH_SIZE / WRITE_SIZE counters to bytes")
    return ap.parse_args()


def copy_calibration():
    import torch

    n = 1 << 30
    a = torch.ones(n // 8, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(10):
        b.copy_(a)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / 10
    print(json.dumps({"copy_bytes_read": n, "copy_bytes_written": n, "ms": round(ms, 4),
                      "GBs": round(2 * n / ms / 1e6, 1)}), flush=True)


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (one GPU's share of the "
              "lattice is one time slab; see the design notes on sharding). Run with --gpus 1.", flush=True)
        sys.exit(2)

    if args.copy_calibration:
        copy_calibration()
        return
    # Tuned stencil launch shapes: unless DD_TUNE_CACHE names a file already,
    # start from the shapes stored with the package (a private copy, so that
    # shapes tuned in this run do not change the stored file).
    if not os.environ.get("DD_TUNE_CACHE"):
        import shutil
        import tempfile
        fd, tmp = tempfile.mkstemp(prefix="dd_tune_", suffix=".txt")
        os.close(fd)
        stored = os.path.join(ROOT, "paper_1612_06424_amd", "tune_cache_mi355x.txt")
        if os.path.exists(stored):
            shutil.copyfile(stored, tmp)
        os.environ["DD_TUNE_CACHE"] = tmp

    import torch

    import paper_1612_06424_amd.dd as dd
    from paper_1612_06424_amd.inputs import WORKLOADS, batched_domains, gaussian_field, random_links

    parts = set(args.parts.split(",")) if args.parts != "all" else {"stencil", "solve", "fact", "overlap", "batched",
                                                                     "force", "overlap_study"}
    if args.no_batched:
        parts.discard("batched")
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")

    # ------------------------------------------------------------ inputs
    w = WORKLOADS["64x32^3"]
    T, L, bc, kappa = w["T"], w["L"], w["bc"], w["kappa"]
    V = T * L ** 3
    t0 = time.time()
    U_nat = random_links(T, L, w["eps"], w["link_seed"])
    log(f"links 64x32^3 generated in {time.time() - t0:.1f}s")
    U64 = dd.pack_links(U_nat, torch.complex128)
    U32 = dd.pack_links(U_nat, torch.complex64)
    del U_nat
    ctx = dd.Context(T, L, bc)
    g = torch.Generator(device=dev)
    g.manual_seed(w["stencil_seed"])
    psi12 = torch.randn((12, 12, V), dtype=torch.complex128, device=dev, generator=g)
    psi12_32 = psi12.to(torch.complex64)
    out12 = torch.empty_like(psi12)
    out12_32 = torch.empty_like(psi12_32)
    slab = (16, 16)
    Vs = 16 * L ** 3
    psis = psi12[:, :, :Vs].contiguous()
    outs = torch.empty_like(psis)
    # 12 point sources at the origin of the slab [0,16)
    src = w["sources"][0]
    eta = torch.zeros((12, 12, Vs), dtype=torch.complex128, device=dev)
    s0 = ((src[0] * L + src[3]) * L + src[2]) * L + src[1]
    for j in range(12):
        eta[j, j, s0] = 1.0
    dom0 = (0, 16)
    p64 = dd.solver_params(tol=w["tol"], max_iter=20000, prec=dd.DD_FP64, solver=dd.DD_CGNR)
    pmx = dd.solver_params(tol=w["tol"], max_iter=20000, prec=dd.DD_MIXED, solver=dd.DD_CGNR)
    pbi = dd.solver_params(tol=w["tol"], max_iter=20000, prec=dd.DD_FP64, solver=dd.DD_BICGSTAB)

    if "batched" in parts:
        t0 = time.time()
        bitems = []
        for it in batched_domains(96):
            Ti, Li = it["T"], it["L"]
            Vi = Ti * Li ** 3
            Ub = dd.pack_links(random_links(Ti, Li, it["eps"], it["link_seed"]))
            b = torch.zeros((12, 12, Vi), dtype=torch.complex128, device=dev)
            ts, xs, ys, zs = it["source"]
            si = ((ts * Li + zs) * Li + ys) * Li + xs
            for j in range(12):
                b[j, j, si] = 1.0
            bitems.append(dict(T=Ti, L=Li, time_bc=0, U=Ub, kappa=it["kappa"], b=b, x=torch.empty_like(b)))
        bctx = dd.Context(8, 8, 0)
        # one context per domain shape for the comparison with one solve per domain
        dctx = {(b["T"], b["L"]): None for b in bitems}
        for key in dctx:
            dctx[key] = dd.Context(key[0], key[1], 0)
        log(f"batched inputs: {len(bitems)} domains, {sum(b['b'].shape[2] for b in bitems)} sites "
            f"({time.time() - t0:.1f}s)")
    if "projection" in parts:
        # quark-line projection at the frontier between t = 15 and 16: N_m = 120 vectors, 10
        # inverse iterations on the 16 slices [8, 24) around it, seeded Gaussian start vectors
        proj_pi, proj_t, proj_nvec, proj_iter = (8, 16), 15, 120, 10
        gp = torch.Generator(device=dev)
        gp.manual_seed(w["stencil_seed"] + 1)
        proj_v0 = torch.randn((proj_nvec, 12, proj_pi[1] * L ** 3), dtype=torch.complex128, device=dev,
                              generator=gp)
    if "disconnected" in parts:
        # disconnected pseudoscalar: Dirichlet domains [0, 33) and [33, 64) (the cut between
        # slices 32 and 33), 100 Gaussian volume sources, 8 powers of kappa D_hop
        disc_doms, disc_nsrc, disc_hop = [(0, 33), (33, 31)], 100, 8
        gd = torch.Generator(device=dev)
        gd.manual_seed(w["stencil_seed"] + 2)
        disc_eta = torch.randn((disc_nsrc, 12, V), dtype=torch.complex128, device=dev, generator=gd)
    if "nucleon" in parts:
        # factorised nucleon: the 64x32^3 links with Dirichlet time walls (as the paper's open
        # boundaries), Gbar = [0, 32) (Delta = 8), Gstar = [24, 64), the lines cut on slice 23 by
        # 120 vectors from 10 inverse iterations on [16, 32), source slice x0 = 4
        nctx = dd.Context(T, L, 0)
        nuc_gbar, nuc_gstar, nuc_t, nuc_x0, nuc_n, nuc_iter, nuc_pi = (0, 32), (24, 40), 23, 4, 120, 10, (16, 16)
        gn = torch.Generator(device=dev)
        gn.manual_seed(w["stencil_seed"] + 3)
        nuc_v0 = torch.randn((nuc_n, 12, nuc_pi[1] * L ** 3), dtype=torch.complex128, device=dev, generator=gn)
    if "force" in parts:
        wf = WORKLOADS["force-32x16^3"]
        Uf = dd.pack_links(random_links(wf["T"], wf["L"], wf["eps"], wf["link_seed"]))
        phi = dd.pack_field(gaussian_field(wf["T"] * wf["L"] ** 3, 1, wf["phi_seed"]))
        fctx = dd.Context(wf["T"], wf["L"], wf["bc"])
        pf = dd.solver_params(tol=wf["tol"], prec=dd.DD_MIXED, solver=dd.DD_CGNR)
    torch.cuda.synchronize()

    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731

    def timed_stencil(fn, n=10):
        a, b = ev(), ev()
        a.record()
        for _ in range(n):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / n

    corr_ref = {}  # the exact correlator of the latest step, for the overlap correction
    stencil_acc = {"bytes": 0.0, "ms": 0.0, "timed": False}  # the 64x32^3 D launches of the timed steps

    def overlap8():
        # the four-slab factorised propagator with overlap regions Delta = 8 (the first "next" row):
        # its extended slabs at this kappa need ~1200 CGNR iterations each, so it runs once, after
        # the timed steps, and is not part of a step
        t0 = time.perf_counter()
        Sf, _, fst = dd.factorized_propagator(ctx, U64, kappa, src, w["domains"], pmx, overlap=8)
        Cf = dd.pion_correlator(ctx, Sf, src[0])
        nd = len(w["domains"])
        r = dict(ms=(time.perf_counter() - t0) * 1e3, timed_step=False,
                 slab_iters=[s["iters"] for s in fst[:nd]],
                 max_true_rel_resid=max(max(s["true_rel_resid"]) for s in fst[:nd]))
        if "Ce" in corr_ref:
            Ce = corr_ref["Ce"]
            for t in (0, 8, 16, 32):
                r[f"C_corr[{t}]/C_exact"] = float((Ce[t] - Cf[t]) / Ce[t])
        del Sf
        return r

    def step(record):
        ph = {}
        if "stencil" in parts:
            for name, fn, nsite, ncol, rb in [
                ("D_fp64_1col", lambda: dd.apply_dirac(ctx, U64, kappa, psi12[:1], None, out12[:1]), V, 1, 8),
                ("D_fp64_12col", lambda: dd.apply_dirac(ctx, U64, kappa, psi12, None, out12), V, 12, 8),
                ("D_fp32_1col", lambda: dd.apply_dirac(ctx, U32, kappa, psi12_32[:1], None, out12_32[:1]), V, 1, 4),
                ("D_fp32_12col", lambda: dd.apply_dirac(ctx, U32, kappa, psi12_32, None, out12_32), V, 12, 4),
                ("Dslab_fp64_12col", lambda: dd.apply_dirac(ctx, U64, kappa, psis, slab, outs), Vs, 12, 8),
            ]:
                ms = timed_stencil(fn)
                gbs = nsite * (48 * ncol + 72) * rb / ms / 1e6
                ph[name] = dict(ms=ms, GBs=gbs, frac=gbs / HBM_PEAK_GBS)
                if stencil_acc["timed"] and name.startswith("D_"):
                    stencil_acc["bytes"] += nsite * (48 * ncol + 72) * rb
                    stencil_acc["ms"] += ms
        if "solve" in parts:
            x64, s64 = dd.block_solve(ctx, U64, kappa, eta, dom0, p64)
            xmx, smx = dd.block_solve(ctx, U64, kappa, eta, dom0, pmx)
            xbi, sbi = dd.block_solve(ctx, U64, kappa, eta, dom0, pbi)
            nh = Vs // 2
            for key, s, pr, me in (("solve_fp64", s64, "fp64", "cgnr"), ("solve_mixed", smx, "mixed", "cgnr"),
                                   ("solve_fp64_bicgstab", sbi, "fp64", "bicgstab")):
                bpi = eo_iteration_bytes(nh, 12, pr, me)
                gbs = bpi * s["iters"] / s["ms"] / 1e6
                ph[key] = dict(ms=s["ms"], iters=s["iters"], updates=s["updates"], restarts=s["restarts"],
                               max_true_rel_resid=max(s["true_rel_resid"]), bytes_per_iter=bpi,
                               algorithmic_GBs=gbs, frac=gbs / HBM_PEAK_GBS)
            if record:
                nrm = torch.linalg.vector_norm(x64)
                ph["solve_mixed"]["rel_diff_vs_fp64"] = float((torch.linalg.vector_norm(xmx - x64) / nrm).item())
                ph["solve_fp64_bicgstab"]["rel_diff_vs_fp64"] = float(
                    (torch.linalg.vector_norm(xbi - x64) / nrm).item())
            del x64, xmx, xbi
        if "fact" in parts:
            t0 = time.perf_counter()
            Sf, Se, fst = dd.factorized_propagator(ctx, U64, kappa, src, w["domains"], pmx, exact=True)
            Cf = dd.pion_correlator(ctx, Sf, src[0])
            Ce = dd.pion_correlator(ctx, Se, src[0])
            nd = len(w["domains"])
            ph["factorised"] = dict(ms=(time.perf_counter() - t0) * 1e3,
                                    slab_iters=[s["iters"] for s in fst[:nd]], exact_iters=fst[nd]["iters"],
                                    max_true_rel_resid=max(max(s["true_rel_resid"]) for s in fst[:nd + 1]))
            if record:
                for t in (0, 8, 16, 32):
                    ph["factorised"][f"C_exact[{t}]"] = float(Ce[t])
                    ph["factorised"][f"C_corr[{t}]/C_exact"] = float((Ce[t] - Cf[t]) / Ce[t])
            corr_ref["Ce"] = Ce
            del Sf, Se
        if "projection" in parts:
            t0 = time.perf_counter()
            basis, pst = dd.projection_basis(ctx, U64, kappa, proj_pi, proj_t, +1, proj_v0, proj_iter, pmx)
            t1 = time.perf_counter()
            log(f"projection: basis {t1 - t0:.1f}s")
            Sf, _, fst = dd.factorized_propagator(ctx, U64, kappa, src, w["domains"], pmx,
                                                  projections={proj_t: basis})
            Cf = dd.pion_correlator(ctx, Sf, src[0])
            t2 = time.perf_counter()
            nd = len(w["domains"])
            ph["projection"] = dict(ms=(t2 - t0) * 1e3, ms_basis=(t1 - t0) * 1e3, ms_propagator=(t2 - t1) * 1e3,
                                    nvec=proj_nvec, inverse_iterations=proj_iter, basis_iters=pst["iters"],
                                    basis_max_true_rel_resid=pst["true_rel_resid"][0],
                                    slab_iters=[s["iters"] for s in fst[:nd]])
            if record and "Ce" in corr_ref:
                Ce = corr_ref["Ce"]
                for t in (0, 8, 16, 32):
                    ph["projection"][f"C_corr[{t}]/C_exact"] = float((Ce[t] - Cf[t]) / Ce[t])
            del Sf, basis
        if "disconnected" in parts:
            t0 = time.perf_counter()
            tau_f, dst = dd.disconnected_traces(ctx, U64, kappa, disc_eta, disc_doms, disc_hop, pmx)
            Cf = dd.disconnected_correlator(ctx, tau_f)
            t1 = time.perf_counter()
            log(f"disconnected: domains {t1 - t0:.1f}s")
            tau_w, wst = dd.disconnected_traces(ctx, U64, kappa, disc_eta, None, disc_hop, pmx)
            Cw = dd.disconnected_correlator(ctx, tau_w)
            t2 = time.perf_counter()
            ph["disconnected"] = dict(ms=(t2 - t0) * 1e3, ms_domains=(t1 - t0) * 1e3, ms_whole=(t2 - t1) * 1e3,
                                      nsrc=disc_nsrc, n_hop=disc_hop, domain_iters=[s["iters"] for s in dst],
                                      whole_iters=wst[0]["iters"],
                                      max_true_rel_resid=max(max(s["true_rel_resid"]) for s in dst + wst))
            if record:
                for d in (2, 8, 16, 32):  # x0, y0 equidistant from the cut at 32
                    x0, y0 = 32 - d // 2, 32 + d // 2
                    ph["disconnected"][f"C_f[{d}]"] = float(Cf[y0, x0].real)
                    ph["disconnected"][f"C_full[{d}]"] = float(Cw[y0, x0].real)
            del tau_f, tau_w
        if "nucleon" in parts:
            t0 = time.perf_counter()
            nb, nbs = dd.projection_basis(nctx, U64, kappa, nuc_pi, nuc_t, +1, nuc_v0, nuc_iter, pmx)
            t1 = time.perf_counter()
            log(f"nucleon: basis {t1 - t0:.1f}s")
            # the lines in calls of 24 vectors (two solves of 12 each), reporting as they go
            parts_xi, parts_eta, nls = [], [], [dict(iters=0, true_rel_resid=[0.0]), dict(iters=0, true_rel_resid=[0.0])]
            for a0 in range(0, nuc_n, 24):
                xa, ea, sa = dd.nucleon_lines(nctx, U64, kappa, nuc_gbar, nuc_gstar, nuc_t, nb[a0:a0 + 24].contiguous(),
                                              nuc_x0, pmx)
                parts_xi.append(xa)
                parts_eta.append(ea)
                for q, r in zip(nls, sa):
                    q["iters"] += r["iters"]
                    q["true_rel_resid"] = [max(q["true_rel_resid"] + r["true_rel_resid"])]
                log(f"nucleon: lines {a0 + 24}/{nuc_n} ({time.perf_counter() - t1:.1f}s)")
            nxi, neta = torch.cat(parts_xi), torch.cat(parts_eta)
            del parts_xi, parts_eta
            t2 = time.perf_counter()
            log(f"nucleon: lines {t2 - t1:.1f}s")
            Bx = dd.baryon_blocks(nctx, nxi)
            By = dd.baryon_blocks(nctx, neta)
            torch.cuda.synchronize()
            t3 = time.perf_counter()
            log(f"nucleon: blocks {t3 - t2:.1f}s")
            W1, W2 = dd.nucleon_contract(nctx, Bx, By)
            t4 = time.perf_counter()
            nslice = 1 + nuc_gstar[1]
            # complex GEMM of the blocks over the pairs i <= j, 8 real flops per multiply-add
            flops = 96.0 * (nuc_n * (nuc_n + 1) // 2) * nuc_n * L ** 3 * nslice
            ph["nucleon"] = dict(ms=(t4 - t0) * 1e3, ms_basis=(t1 - t0) * 1e3, ms_lines=(t2 - t1) * 1e3,
                                 ms_blocks=(t3 - t2) * 1e3, ms_contract=(t4 - t3) * 1e3, nvec=nuc_n,
                                 block_slices=nslice, block_TFLOPs=flops / (t3 - t2) / 1e12,
                                 basis_iters=nbs["iters"], line_iters=[q["iters"] for q in nls],
                                 max_true_rel_resid=max(max(q["true_rel_resid"]) for q in nls))
            # the block product runs on the FP64 matrix cores (diquark kernels included in the time)
            tf = flops / (t3 - t2) / 1e12
            ph["nucleon"]["block_roofline"] = dict(bound="mfma", achieved=round(tf, 2), peak=FP64_PEAK_TFLOPS,
                                                   unit="TFLOP/s", frac=round(tf / FP64_PEAK_TFLOPS, 4))
            if record and not args.no_cpu_baseline:
                ph["nucleon"]["block_cpu_baseline"] = nucleon_cpu_baseline()
            if record:
                Cn = (W1[:, 0] - W2[:, 0]) / L ** 3  # C_N^(f)(y0, x0 = 4), y0 = 24 + index
                for y0 in (24, 28, 32, 40, 48):
                    ph["nucleon"][f"C_f[{y0}]"] = float(Cn[y0 - 24].real)
            del nb, nxi, neta, Bx, By
        if "batched" in parts:
            t0 = time.perf_counter()
            bst = dd.block_solve_batched(bctx, bitems, pmx)
            ms_b = (time.perf_counter() - t0) * 1e3
            # the same domains with one solve (of 12 columns) each, in turn
            t1 = time.perf_counter()
            sst = []
            for it in bitems:
                xi, si = dd.block_solve(dctx[(it["T"], it["L"])], it["U"], it["kappa"], it["b"], None, pmx,
                                        x=it["x"])
                sst.append(si)
            ms_s = (time.perf_counter() - t1) * 1e3
            site_it = sum(it["b"].shape[2] * 12 * s["iters"] for it, s in zip(bitems, bst))
            bbytes = sum(eo_iteration_bytes(it["b"].shape[2] // 2, 12, "mixed", "cgnr") * s["iters"]
                         for it, s in zip(bitems, bst))
            ph["batched"] = dict(ms=ms_b, domains=len(bitems), domains_per_s=len(bitems) / ms_b * 1e3,
                                 site_iterations_per_s=site_it / ms_b * 1e3,
                                 algorithmic_GBs=bbytes / ms_b / 1e6, frac=bbytes / ms_b / 1e6 / HBM_PEAK_GBS,
                                 max_true_rel_resid=max(max(s["true_rel_resid"]) for s in bst),
                                 ms_one_solve_per_domain=ms_s, speedup_vs_one_solve_per_domain=ms_s / ms_b,
                                 max_true_rel_resid_one_per_domain=max(max(s["true_rel_resid"]) for s in sst))
        if "force" in parts:
            t0 = time.perf_counter()
            Ug = Uf.clone().requires_grad_(True)
            S = dd.DomainActionFn.apply(Ug, phi, fctx, wf["kappa"], None, pf)
            S.backward()
            torch.cuda.synchronize()
            ph["force"] = dict(ms=(time.perf_counter() - t0) * 1e3, S=float(S.item()))
        return ph

    for i in range(args.warmup):
        log(f"warmup step {i}")
        step(False)
    contexts = [ctx] + ([bctx] + list(dctx.values()) if "batched" in parts else []) + \
        ([fctx] if "force" in parts else [])
    stencil_acc["timed"] = True
    for c in contexts:
        dd.set_kernel_timing(c, True)
    torch.cuda.synchronize()
    log("timed region")
    t0 = time.perf_counter()
    phases = []
    for i in range(args.steps):
        phases.append(step(i == args.steps - 1))
        log(f"step {i}: {json.dumps({k: round(v.get('ms', 0), 2) for k, v in phases[-1].items()})}")
    torch.cuda.synchronize()
    total_ms = (time.perf_counter() - t0) * 1e3
    kt = {}
    for c in contexts:
        for name, (ms, n, b) in dd.kernel_timing(c).items():
            a = kt.setdefault(name, [0.0, 0, 0.0])
            a[0] += ms
            a[1] += n
            a[2] += b
        dd.set_kernel_timing(c, False)
    tot_ms = sum(v[0] for v in kt.values())
    tot_b = sum(v[2] for v in kt.values())
    value_all = tot_b / max(tot_ms, 1e-9) / 1e6  # aggregate algorithmic stencil GB/s over every timed launch
    # the headline: D on the whole 64x32^3 lattice (FP64 / FP32, 1 and 12 columns), bytes over time
    value = stencil_acc["bytes"] / max(stencil_acc["ms"], 1e-9) / 1e6 if stencil_acc["ms"] > 0 else value_all
    dom_name = max(kt, key=lambda k: kt[k][0]) if kt else ""
    dms, dn, db = kt.get(dom_name, (0.0, 0, 0.0))
    achieved = db / max(dms, 1e-9) / 1e6 if dn else 0.0
    last = phases[-1]
    out = {
        "metric": "Dirac-stencil GB/s + 12-source domain solve ms (mixed vs FP64) at 64x32^3",
        "value": round(value, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(total_ms / args.steps, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128+c64",
        "data": "synthetic",
        "config": {"workload": "64x32^3 Wilson-Dirac, antiperiodic time, eps=0.15, kappa=0.135; "
                               "12-source solves on the 16x32^3 slab; 4-slab factorised propagator (overlap 0 timed; overlap 8 once, untimed); "
                               "96 uneven Dirichlet domains; 32x16^3 force",
                   "lattice": [T, L, L, L], "kappa": kappa, "tol": w["tol"],
                   "parts": sorted(parts)},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": dom_name, "launches": dn, "avg_launch_ms": round(dms / max(dn, 1), 5),
                     "bytes_per_launch": round(db / max(dn, 1)),
                     "share_of_stencil_time": round(dms / max(tot_ms, 1e-9), 3)},
        # the five kernel instances with the most time, each against the same peak
        "roofline_top": [{"kernel": k, "share_of_stencil_time": round(v[0] / max(tot_ms, 1e-9), 3),
                          "achieved": round(v[2] / max(v[0], 1e-9) / 1e6, 1),
                          "frac": round(v[2] / max(v[0], 1e-9) / 1e6 / HBM_PEAK_GBS, 4)}
                         for k, v in sorted(kt.items(), key=lambda kv: -kv[1][0])[:5]],
        "stencil_kernels": {k: {"ms": round(v[0], 2), "launches": v[1], "GBs": round(v[2] / max(v[0], 1e-9) / 1e6, 1)}
                            for k, v in sorted(kt.items(), key=lambda kv: -kv[1][0])},
        "value_definition": "algorithmic GB/s of D on the whole 64x32^3 lattice, FP64 and FP32, 1 and 12 "
                            "columns (sum of bytes over sum of time)" if stencil_acc["ms"] > 0 else
                            "aggregate over every stencil launch",
        "stencil_GBs_all_launches": round(value_all, 1),
    }
    if "solve" in parts:
        out["domain_solve_ms_fp64"] = round(last["solve_fp64"]["ms"], 2)
        out["domain_solve_ms_mixed"] = round(last["solve_mixed"]["ms"], 2)
        out["mixed_speedup"] = round(last["solve_fp64"]["ms"] / last["solve_mixed"]["ms"], 3)
        out["domain_solve_frac_mixed"] = round(last["solve_mixed"]["frac"], 4)
        out["domain_solve_frac_fp64"] = round(last["solve_fp64"]["frac"], 4)
    traffic = stencil_traffic(dom_name)
    if traffic is not None:
        out["roofline"]["traffic"] = traffic
        out["roofline"]["traffic_over_algorithmic"] = round(traffic / max(db / max(dn, 1), 1), 3)
    out["parts"] = last
    if "overlap" in parts:
        log("overlap 8 (once, untimed)")
        out["parts"]["factorised_overlap8"] = overlap8()
    if "overlap_study" in parts:
        out["overlap_study"] = overlap_study(dd, ctx, U64, w, pmx)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(T, L, bc, kappa, w)
    print(json.dumps(out), flush=True)


def overlap_study(dd, ctx, U64, w, params):
    """The hierarchy of the factorised pion correlator in the overlap thickness Delta
    (Sec. 3.2, Eqs. 14-15; the expansion of Sec. 6): on the 64x32^3 lattice, source slab
    Gamma = [0, 24) and Gamma* = [24, 64), point source at x0 = (4, 0, 0, 0), the
    factorised correlator C^(i) with Delta = 8, 12, 16 for i = 0, 1, 2, and the exact C.
    Reported per slice t: C, C^(0), C^(1) - C^(0), C^(2) - C^(1) and C^(rest) = C - C^(2),
    at kappa = 0.12 and 0.115 on the workload's links.  The workload's own kappa = 0.135
    lies past the critical value of these smooth links: the propagator does not decay, the
    factorised correlator exceeds the exact one by orders of magnitude at every Delta and the
    solves take thousands of iterations (the study there took 108 s), so it stays out.
    Untimed; mixed-precision solves to the workload's tol."""
    src = (4, 0, 0, 0)
    doms = [(0, 24), (24, 40)]
    deltas = (8, 12, 16)
    show = [4, 8, 16, 20, 24, 28, 32, 36, 40, 48, 56]
    res = {"domains": [list(d) for d in doms], "source": list(src), "deltas": list(deltas), "t": show}
    for kap in (0.12, 0.115):
        t0 = time.perf_counter()
        C = {}
        iters = {}
        for i, dl in enumerate(deltas):
            Sf, Se, st = dd.factorized_propagator(ctx, U64, kap, src, doms, params, overlap=dl, exact=(i == 0))
            C[dl] = dd.pion_correlator(ctx, Sf, src[0])
            iters[dl] = [s["iters"] for s in st]
            if Se is not None:
                C["exact"] = dd.pion_correlator(ctx, Se, src[0])
            del Sf, Se
        Ce, C0, C1, C2 = C["exact"], C[8], C[12], C[16]
        res[f"kappa={kap}"] = {
            "ms": round((time.perf_counter() - t0) * 1e3, 1),
            "solve_iters": {str(k): v for k, v in iters.items()},
            "C": [float(Ce[t]) for t in show],
            "C0": [float(C0[t]) for t in show],
            "C1-C0": [float(C1[t] - C0[t]) for t in show],
            "C2-C1": [float(C2[t] - C1[t]) for t in show],
            "rest": [float(Ce[t] - C2[t]) for t in show],
        }
    return res


def stencil_traffic(kernel):
    """HBM bytes per launch of `kernel` (FETCH_SIZE + WRITE_SIZE, scaled by a plain
    copy) from the profiler summary kept in profiles/, or None when it is missing
    or was taken on other stencil sources than the ones built here."""
    from paper_1612_06424_amd.rocprof_summary import kernel_source_hash

    path = os.path.join(ROOT, "profiles", "stencil_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_hash") != kernel_source_hash():
        return None
    k = rec.get("kernels", {}).get(kernel)
    return k["hbm_bytes"] if k else None


def cpu_baseline(T, L, bc, kappa, w):
    """The FP64 oracle, as it stands, on a bounded sample of the same workload:
    the whole-lattice D apply on 64x32^3 for all 12 columns, repeated until about
    10 s of host time have been spent (at most 8 times), scaled to GB/s with the
    same algorithmic byte count as the GPU."""
    import numpy as np

    sys.path.insert(0, os.path.join(ROOT, "oracle"))
    import oracle as O
    from paper_1612_06424_amd.inputs import gaussian_field, random_links

    U = random_links(T, L, w["eps"], w["link_seed"])
    ncol = 12
    psi = gaussian_field(T * L ** 3, ncol, w["stencil_seed"])
    O.apply_dirac(U, kappa, T, L, bc, psi[0])
    reps, dt = 0, 0.0
    while reps < 8 and dt < 10.0:
        t0 = time.perf_counter()
        O.apply_dirac(U, kappa, T, L, bc, psi)
        dt += time.perf_counter() - t0
        reps += 1
    V = T * L ** 3
    gbs = V * (48 + 72) * 8 * ncol * reps / dt / 1e9  # one column per apply: links re-read per column
    out = {"value": round(gbs, 2), "unit": "GB/s", "cores": O.threads(), "kind": "oracle",
           "sample": f"oracle D apply, whole 64x32^3 lattice, FP64, {ncol} columns one at a time, "
                     f"{reps} times ({dt:.1f} s)"}
    out["solves"] = cpu_solve_baseline(O)
    return out


def cpu_solve_baseline(O):
    """The oracle's 12-column domain solves, as they stand (FP64 BiCGStab on the plain
    operator, to a true residual of 1e-10), on bounded samples:
      32x16^3 workload: the 16x16^3 slab [0,16) with the point source (0, 0, 0, 0), one column
        solved in full, the 12-column time extrapolated (x 12);
      64x32^3 workload: the 16x32^3 slab [0,16) with the point source at the origin, 10
        iterations of one column timed; the 12-column time estimated with the iteration count
        of the same plain-operator FP64 BiCGStab on the GPU (618, measured there), x 12."""
    from paper_1612_06424_amd.inputs import WORKLOADS, point_sources, random_links

    res = {}
    w2 = WORKLOADS["32x16^3"]
    T2, L2 = w2["T"], w2["L"]
    U2 = random_links(T2, L2, w2["eps"], w2["link_seed"])
    b2 = O.slab_extract(T2, L2, point_sources(T2, L2, 0, 0, 0, 0)[:1], (0, 16))
    t0 = time.perf_counter()
    _, it2, rr2, st2 = O.solve(U2, w2["kappa"], T2, L2, w2["bc"], b2, dom=(0, 16), tol=1e-10, method=0)
    d2 = time.perf_counter() - t0
    res["slab_16x16^3_12col_ms"] = round(d2 * 12 * 1e3, 1)
    res["slab_16x16^3_sample"] = (f"one column solved in {d2:.1f} s ({it2[0]} iterations, residual {rr2[0]:.1e}, "
                                  f"status {st2}); 12 columns extrapolated x 12")
    w3 = WORKLOADS["64x32^3"]
    T3, L3 = w3["T"], w3["L"]
    U3 = random_links(T3, L3, w3["eps"], w3["link_seed"])
    b3 = O.slab_extract(T3, L3, point_sources(T3, L3, 0, 0, 0, 0)[:1], (0, 16))
    t0 = time.perf_counter()
    _, it3, _, _ = O.solve(U3, w3["kappa"], T3, L3, w3["bc"], b3, dom=(0, 16), tol=1e-30, maxit=10, method=0)
    d3 = time.perf_counter() - t0
    per_it = d3 / max(it3[0], 1)
    res["slab_16x32^3_12col_ms_estimate"] = round(per_it * 618 * 12 * 1e3, 1)
    res["slab_16x32^3_sample"] = (f"{it3[0]} iterations of one column in {d3:.1f} s; x 618 iterations (the GPU's "
                                  f"plain-operator FP64 BiCGStab count on this system) x 12 columns: an estimate")
    return res


def nucleon_cpu_baseline():
    """The oracle's baryon blocks (Eq. 25), as they stand, on a bounded sample of the nucleon
    block workload: 8 Gaussian vectors on one 16^3 slice (about 10 s of host time), scaled to
    TFLOP/s with the GPU's executed flop count for the same sample (96 P n L^3, P = n(n+1)/2)."""
    sys.path.insert(0, os.path.join(ROOT, "oracle"))
    import oracle as O
    from paper_1612_06424_amd.inputs import gaussian_field

    n, Ls = 8, 16
    s = gaussian_field(Ls ** 3, n, 9)
    t0 = time.perf_counter()
    O.baryon_blocks(Ls, s)
    dt = time.perf_counter() - t0
    flops = 96.0 * (n * (n + 1) // 2) * n * Ls ** 3
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        cores = 1
    return {"value": flops / dt / 1e12, "unit": "TFLOP/s", "cores": cores, "kind": "oracle",
            "sample": f"oracle baryon blocks (numpy einsum, FP64), {n} vectors on one {Ls}^3 slice ({dt:.1f} s)"}


if __name__ == "__main__":
    main()
