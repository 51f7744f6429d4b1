// solver.hip -- Krylov solvers for D x = b on the whole lattice or a Dirichlet
// slab, all columns advancing together (one stencil launch serves every
// column; links are fetched once per launch per site block).
//
// The scalars of each column live on the device (ColState) and are updated by
// one-workgroup finalize kernels, so iterations run without host round trips;
// the host reads the per-column state every `check_every` iterations.
//
// Convergence is always confirmed on the true FP64 residual |b - D x| / |b|.
// BiCGStab cycles restart from the true residual (new shadow residual r^ = r)
// after a breakdown or when the recursive residual has drifted.
//
// DD_MIXED: defect correction.  The outer loop computes r = b - D x in FP64,
// solves D e = r / |r| with FP32 links and FP32 vectors to a relative residual
// inner_tol (inner products accumulated in FP64), and adds |r| e to x in FP64.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

#include "dd_internal.h"

namespace dd {

namespace {

template <typename R>
struct Vecs {
    cpx<R>*r, *rh, *p, *v, *s, *t;
};

template <typename R>
dd_status get_vecs(dd_ctx* c, size_t n, Vecs<R>* w) {
    dd_status st = DD_OK;
    const int base = sizeof(R) == 8 ? W_R : W_R32;
    cpx<R>** ptrs[6] = {&w->r, &w->rh, &w->p, &w->v, &w->s, &w->t};
    for (int i = 0; i < 6; i++) {
        *ptrs[i] = (cpx<R>*)workspace(c, Slot(base + i), n * sizeof(cpx<R>), &st);
        if (st != DD_OK) return st;
    }
    return DD_OK;
}

dd_status ensure_host(dd_ctx* c, int ncol) {
    if (c->host_n >= ncol) return DD_OK;
    if (c->host_state) (void)hipHostFree(c->host_state);
    if (c->host_dots) (void)hipHostFree(c->host_dots);
    c->host_state = nullptr;
    c->host_dots = nullptr;
    c->host_n = 0;
    DD_HIP(c, hipHostMalloc((void**)&c->host_state, sizeof(ColState) * ncol, hipHostMallocDefault));
    DD_HIP(c, hipHostMalloc((void**)&c->host_dots, sizeof(double) * 3 * ncol, hipHostMallocDefault));
    c->host_n = ncol;
    return DD_OK;
}

dd_status pull_state(dd_ctx* c, const ColState* dev, int ncol) {
    DD_HIP(c, hipGetLastError());
    DD_HIP(c, hipMemcpyAsync(c->host_state, dev, sizeof(ColState) * ncol, hipMemcpyDeviceToHost, c->stream));
    DD_HIP(c, hipStreamSynchronize(c->stream));
    return DD_OK;
}

dd_status push_state(dd_ctx* c, ColState* dev, int ncol) {
    DD_HIP(c, hipMemcpyAsync(dev, c->host_state, sizeof(ColState) * ncol, hipMemcpyHostToDevice, c->stream));
    return DD_OK;
}

// |a_col|^2 for every column, read back to host_dots[3*col].
template <typename R>
dd_status norms_to_host(dd_ctx* c, int n, int ncol, const cpx<R>* a, double* partial, double* dots) {
    launch_norm2<R>(c, n, ncol, a, partial);
    launch_finalize(c, FIN_STORE, ncol, (n + kBlock - 1) / kBlock, partial, nullptr, dots);
    DD_HIP(c, hipGetLastError());
    DD_HIP(c, hipMemcpyAsync(c->host_dots, dots, sizeof(double) * 3 * ncol, hipMemcpyDeviceToHost, c->stream));
    DD_HIP(c, hipStreamSynchronize(c->stream));
    return DD_OK;
}

// r = b - A x (FP64) and |r|^2 per column into host_dots[3*col].
dd_status residual_to_host(dd_ctx* c, const Geo& g, const cpx<double>* U, double kappa, int dag, int ncol,
                           const cpx<double>* b, const cpx<double>* x, cpx<double>* r, double* partial,
                           double* dots) {
    launch_dslash<double>(c, g, U, kappa, dag, EPI_RESID, x, r, b, ncol, partial, nullptr);
    launch_finalize(c, FIN_STORE, ncol, site_blocks(g.nsite), partial, nullptr, dots);
    DD_HIP(c, hipGetLastError());
    DD_HIP(c, hipMemcpyAsync(c->host_dots, dots, sizeof(double) * 3 * ncol, hipMemcpyDeviceToHost, c->stream));
    DD_HIP(c, hipStreamSynchronize(c->stream));
    return DD_OK;
}

// BiCGStab iterations for every active column until all are inactive or the
// budget is spent.  Returns the lockstep iteration count in *done.
template <typename R>
dd_status bicgstab_iterate(dd_ctx* c, const Geo& g, const cpx<R>* U, double kappa, int dag, int ncol,
                           cpx<R>* x, const Vecs<R>& w, ColState* st, double* partial, int check_every,
                           int budget, int* done) {
    const int n = 12 * g.nsite;
    const int nsb = site_blocks(g.nsite);
    const int nbe = (n + kBlock - 1) / kBlock;
    int it = 0;
    *done = 0;
    while (it < budget) {
        const int k = std::min(check_every, budget - it);
        for (int j = 0; j < k; j++) {
            launch_bicg_p<R>(c, n, ncol, w.r, w.p, w.v, st);
            launch_dslash<R>(c, g, U, kappa, dag, EPI_DOT_AUX, w.p, w.v, w.rh, ncol, partial, st);
            launch_finalize(c, FIN_ALPHA, ncol, nsb, partial, st, nullptr);
            launch_bicg_s<R>(c, n, ncol, w.r, w.v, w.s, st);
            launch_dslash<R>(c, g, U, kappa, dag, EPI_TS, w.s, w.t, nullptr, ncol, partial, st);
            launch_finalize(c, FIN_OMEGA, ncol, nsb, partial, st, nullptr);
            launch_bicg_xr<R>(c, n, ncol, x, w.r, w.p, w.s, w.t, w.rh, partial, st);
            launch_finalize(c, FIN_RHO, ncol, nbe, partial, st, nullptr);
        }
        it += k;
        dd_status e = pull_state(c, st, ncol);
        if (e != DD_OK) return e;
        int any = 0, mx = 0;
        for (int j = 0; j < ncol; j++) {
            any |= c->host_state[j].active;
            mx = std::max(mx, c->host_state[j].iters);
        }
        *done = mx;
        if (!any) break;
    }
    return DD_OK;
}

// CGNR iterations (CG on A^+ A) for every active column.  Expects r = b - A x,
// z = A^+ r, p = z and zz set.
template <typename R>
dd_status cgnr_iterate(dd_ctx* c, const Geo& g, const cpx<R>* U, double kappa, int dag, int ncol, cpx<R>* x,
                       const Vecs<R>& w, ColState* st, double* partial, int check_every, int budget,
                       int* done) {
    const int n = 12 * g.nsite;
    const int nsb = site_blocks(g.nsite);
    const int nbe = (n + kBlock - 1) / kBlock;
    cpx<R>* r = w.r;
    cpx<R>* p = w.p;
    cpx<R>* wv = w.v;
    cpx<R>* z = w.s;
    int it = 0;
    *done = 0;
    while (it < budget) {
        const int k = std::min(check_every, budget - it);
        for (int j = 0; j < k; j++) {
            launch_dslash<R>(c, g, U, kappa, dag, EPI_NORM, p, wv, nullptr, ncol, partial, st);
            launch_finalize(c, FIN_CG_ALPHA, ncol, nsb, partial, st, nullptr);
            launch_cg_xr<R>(c, n, ncol, x, r, p, wv, partial, st);
            launch_finalize(c, FIN_CG_RR, ncol, nbe, partial, st, nullptr);
            launch_dslash<R>(c, g, U, kappa, 1 - dag, EPI_NORM, r, z, nullptr, ncol, partial, st);
            launch_finalize(c, FIN_CG_BETA, ncol, nsb, partial, st, nullptr);
            launch_cg_p<R>(c, n, ncol, p, z, st);
        }
        it += k;
        dd_status e = pull_state(c, st, ncol);
        if (e != DD_OK) return e;
        int any = 0, mx = 0;
        for (int j = 0; j < ncol; j++) {
            any |= c->host_state[j].active;
            mx = std::max(mx, c->host_state[j].iters);
        }
        *done = mx;
        if (!any) break;
    }
    return DD_OK;
}

// Start a Krylov cycle on the device for the columns flagged active in
// host_state (stop2 holds the relative stopping factor): r already holds the
// system's residual; sets r^ = r, p = v = 0 (BiCGStab) or z = A^+ r, p = z (CGNR).
template <typename R>
dd_status start_cycle(dd_ctx* c, const Geo& g, const cpx<R>* U, double kappa, int dag, int ncol, int kind,
                      const Vecs<R>& w, ColState* st, double* partial) {
    const int n = 12 * g.nsite;
    dd_status e = push_state(c, st, ncol);
    if (e != DD_OK) return e;
    launch_norm2<R>(c, n, ncol, w.r, partial);
    launch_finalize(c, FIN_INIT, ncol, (n + kBlock - 1) / kBlock, partial, st, nullptr);
    if (kind == DD_BICGSTAB) {
        launch_copy_cols<R>(c, n, ncol, w.r, w.rh, st);
        launch_zero<R>(c, (size_t)n * ncol, w.p);
        launch_zero<R>(c, (size_t)n * ncol, w.v);
    } else {
        launch_dslash<R>(c, g, U, kappa, 1 - dag, EPI_NORM, w.r, w.s, nullptr, ncol, partial, st);
        launch_finalize(c, FIN_CG_ZZ, ncol, site_blocks(g.nsite), partial, st, nullptr);
        launch_copy_cols<R>(c, n, ncol, w.s, w.p, st);
    }
    DD_HIP(c, hipGetLastError());
    return DD_OK;
}

void reset_host_state(dd_ctx* c, int ncol) { std::memset(c->host_state, 0, sizeof(ColState) * ncol); }

}  // namespace

// Solve A x = b with A = D_Lambda (dag = 0) or D_Lambda^+ (dag = 1).
dd_status solve(dd_ctx* c, const cpx<double>* U, double kappa, const Geo& g, int ncol, const cpx<double>* b,
                cpx<double>* x, const dd_solver_params& p, dd_solve_stats* stats, int dag) {
    const auto t_start = std::chrono::steady_clock::now();
    const int n = 12 * g.nsite;
    const size_t ntot = (size_t)n * ncol;
    const int check_every = p.check_every > 0 ? p.check_every : 8;
    const int kind = p.solver;
    dd_status e = DD_OK;
    e = ensure_host(c, ncol);
    if (e != DD_OK) return e;

    const size_t npart = (size_t)ncol * ((n + kBlock - 1) / kBlock) * 3;
    double* partial = (double*)workspace(c, W_PART, npart * sizeof(double), &e);
    if (e != DD_OK) return e;
    ColState* st = (ColState*)workspace(c, W_STATE, sizeof(ColState) * ncol, &e);
    if (e != DD_OK) return e;
    double* dots = (double*)workspace(c, W_DOTS, sizeof(double) * 3 * ncol, &e);
    if (e != DD_OK) return e;
    Vecs<double> w64;
    e = get_vecs<double>(c, ntot, &w64);
    if (e != DD_OK) return e;

    Vecs<float> w32{};
    cpx<float>*U32 = nullptr, *x32 = nullptr;
    double *scale_dn = nullptr, *scale_up = nullptr;
    if (p.prec == DD_MIXED) {
        e = get_vecs<float>(c, ntot, &w32);
        if (e != DD_OK) return e;
        const size_t nl = (size_t)36 * g.vlink;
        U32 = (cpx<float>*)workspace(c, W_U32, nl * sizeof(cpx<float>), &e);
        if (e != DD_OK) return e;
        x32 = (cpx<float>*)workspace(c, W_X32, ntot * sizeof(cpx<float>), &e);
        if (e != DD_OK) return e;
        scale_dn = (double*)workspace(c, W_AUX0, sizeof(double) * ncol, &e);
        if (e != DD_OK) return e;
        scale_up = (double*)workspace(c, W_AUX1, sizeof(double) * ncol, &e);
        if (e != DD_OK) return e;
        launch_links_to_f32(c, nl, U, U32);
    }

    // |b|^2 per column
    e = norms_to_host<double>(c, n, ncol, b, partial, dots);
    if (e != DD_OK) return e;
    std::vector<double> bb(ncol), rel(ncol, 0.0);
    for (int j = 0; j < ncol; j++) bb[j] = c->host_dots[3 * j];
    for (int j = 0; j < ncol; j++)
        if (!std::isfinite(bb[j])) return fail(c, DD_ERR_BREAKDOWN, "non-finite values in the right-hand side");
    launch_zero<double>(c, ntot, x);

    int total = 0, outer = 0, restarts = 0;
    bool converged = false, nonfinite = false;
    const double tol = p.tol;
    while (true) {
        // true residual r = b - A x in FP64
        e = residual_to_host(c, g, U, kappa, dag, ncol, b, x, w64.r, partial, dots);
        if (e != DD_OK) return e;
        int nact = 0;
        std::vector<int> act(ncol, 0);
        for (int j = 0; j < ncol; j++) {
            const double rr = c->host_dots[3 * j];
            if (!std::isfinite(rr)) nonfinite = true;
            rel[j] = bb[j] > 0 ? std::sqrt(rr / bb[j]) : 0.0;
            act[j] = (bb[j] > 0 && !(rel[j] <= tol)) ? 1 : 0;
            nact += act[j];
        }
        if (nonfinite) break;
        if (nact == 0) {
            converged = true;
            break;
        }
        if (total >= p.max_iter || (p.prec == DD_MIXED && outer >= p.max_outer)) break;
        reset_host_state(c, ncol);
        if (p.prec != DD_MIXED) {
            // FP64 Krylov cycle from the true residual
            for (int j = 0; j < ncol; j++) {
                c->host_state[j].active = act[j];
                c->host_state[j].bb = bb[j];
                c->host_state[j].stop2 = 0.25 * tol * tol * bb[j] / std::max(c->host_dots[3 * j], 1e-300);
            }
            e = start_cycle<double>(c, g, U, kappa, dag, ncol, kind, w64, st, partial);
            if (e != DD_OK) return e;
            int done = 0;
            if (kind == DD_BICGSTAB)
                e = bicgstab_iterate<double>(c, g, U, kappa, dag, ncol, x, w64, st, partial, check_every,
                                             p.max_iter - total, &done);
            else
                e = cgnr_iterate<double>(c, g, U, kappa, dag, ncol, x, w64, st, partial, check_every,
                                         p.max_iter - total, &done);
            if (e != DD_OK) return e;
            total += done;
            for (int j = 0; j < ncol; j++)
                if (c->host_state[j].breakdown == 2) nonfinite = true;
            if (nonfinite) break;
            restarts += outer > 0 ? 1 : 0;
            outer++;
        } else {
            // defect correction: e = A32^-1 (r / |r|), x += |r| e
            std::vector<double> dn(ncol), up(ncol);
            for (int j = 0; j < ncol; j++) {
                const double rn = std::sqrt(c->host_dots[3 * j]);
                dn[j] = act[j] ? 1.0 / rn : 0.0;
                up[j] = act[j] ? rn : 0.0;
                c->host_state[j].active = act[j];
                c->host_state[j].bb = 1.0;
                c->host_state[j].stop2 = p.inner_tol * p.inner_tol;
            }
            DD_HIP(c, hipMemcpyAsync(scale_dn, dn.data(), sizeof(double) * ncol, hipMemcpyHostToDevice, c->stream));
            DD_HIP(c, hipMemcpyAsync(scale_up, up.data(), sizeof(double) * ncol, hipMemcpyHostToDevice, c->stream));
            launch_to_f32_scaled(c, n, ncol, w64.r, w32.r, scale_dn, nullptr);
            launch_zero<float>(c, ntot, x32);
            e = start_cycle<float>(c, g, U32, kappa, dag, ncol, kind, w32, st, partial);
            if (e != DD_OK) return e;
            int done = 0;
            if (kind == DD_BICGSTAB)
                e = bicgstab_iterate<float>(c, g, U32, kappa, dag, ncol, x32, w32, st, partial, check_every,
                                            p.max_iter - total, &done);
            else
                e = cgnr_iterate<float>(c, g, U32, kappa, dag, ncol, x32, w32, st, partial, check_every,
                                        p.max_iter - total, &done);
            if (e != DD_OK) return e;
            total += done;
            launch_add_f32_scaled(c, n, ncol, x, x32, scale_up, nullptr);
            // The scales live in pageable host vectors: make sure the copies are done.
            DD_HIP(c, hipStreamSynchronize(c->stream));
            outer++;
        }
    }
    if (stats) {
        stats->nrhs = ncol;
        stats->iters = total;
        stats->outer = outer;
        stats->restarts = restarts;
        for (int j = 0; j < DD_MAX_RHS; j++) stats->true_rel_resid[j] = j < ncol ? rel[j] : 0.0;
        stats->ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    }
    if (nonfinite) return fail(c, DD_ERR_BREAKDOWN, "non-finite values in the Krylov iteration");
    if (!converged) {
        double worst = 0;
        for (int j = 0; j < ncol; j++) worst = std::max(worst, rel[j]);
        return fail(c, DD_ERR_NOCONV,
                    "solver stopped after " + std::to_string(total) + " iterations with relative residual " +
                        std::to_string(worst) + " > tol " + std::to_string(tol));
    }
    return DD_OK;
}

}  // namespace dd
