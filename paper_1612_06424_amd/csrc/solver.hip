// solver.hip -- Krylov solvers for D x = b on the whole lattice or a Dirichlet
// slab, all columns advancing together (one stencil launch serves every
// column; links are fetched once per launch per site block).
//
// The scalars of each column live on the device (ColState) and are updated by
// one-workgroup finalize kernels, so iterations run without host round trips;
// the host reads the per-column state every `check_every` iterations.
//
// Both methods (BiCGStab on D, CGNR = CG on D^+ D) use reliable updates: the
// Krylov recursion runs in precision R (FP64, or FP32 links and vectors for
// DD_MIXED with inner products accumulated in FP64), and whenever a column's
// recursive residual has dropped by the factor delta the correction is folded
// into the FP64 solution and the recursive residual is replaced by the true
// FP64 residual b - D x.  Convergence is always decided on that true residual.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <type_traits>

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
    launch_finalize(c, FIN_STORE, ncol, stencil_slots(c, g, 0, ncol), partial, nullptr, dots);
    DD_HIP(c, hipGetLastError());
    DD_HIP(c, hipMemcpyAsync(c->host_dots, dots, sizeof(double) * 3 * ncol, hipMemcpyDeviceToHost, c->stream));
    DD_HIP(c, hipStreamSynchronize(c->stream));
    return DD_OK;
}

void reset_host_state(dd_ctx* c, int ncol) { std::memset(c->host_state, 0, sizeof(ColState) * ncol); }

// BiCGStab with reliable updates (Sleijpen & van der Vorst, Computing 56 (1996)
// 141): the Krylov vectors live in precision R; whenever a column's recursive
// residual has dropped by delta below the largest one seen since its last
// update, or the recursion claims convergence, or it broke down, the host
//   - folds the accumulated correction into the FP64 solution (R = float),
//   - recomputes the true residual r = b - D x in FP64,
//   - finishes the column if |r|/|b| <= tol, otherwise replaces the recursive
//     residual by the true one and continues with the same search directions
//     (a breakdown also takes a fresh shadow residual r^ = r).
// Iteration counts are not inflated by restarts and the answer is checked in
// FP64.  For R = double the correction goes straight into x.
template <typename R>
dd_status bicgstab_reliable(dd_ctx* c, const Geo& g, const cpx<double>* U64, const cpx<R>* UK, double kappa,
                            int dag, int ncol, const cpx<double>* b, cpx<double>* x, const std::vector<double>& bb,
                            const dd_solver_params& p, double delta, const Vecs<R>& w, cpx<R>* xk,
                            cpx<double>* r64, ColState* st, double* partial, double* dots, int* mask_dev,
                            std::vector<double>& rel, int* total_out, int* updates_out, int* restarts_out, bool* nonfinite) {
    const int n = 12 * g.nsite;
    const size_t ntot = (size_t)n * ncol;
    const bool fold = !std::is_same<R, double>::value;
    const int check_every = p.check_every > 0 ? p.check_every : 8;
    const int nsb = stencil_slots(c, g, sizeof(R) == 8 ? 0 : 1, ncol);
    const int nbe = (n + kBlock - 1) / kBlock;
    const double tol = p.tol;
    cpx<R>* xx = fold ? xk : reinterpret_cast<cpx<R>*>(x);
    dd_status e;
    launch_zero<double>(c, ntot, x);
    if (fold) launch_zero<R>(c, ntot, xk);
    e = residual_to_host(c, g, U64, kappa, dag, ncol, b, x, r64, partial, dots);
    if (e != DD_OK) return e;
    std::vector<int> done(ncol, 0), mask(ncol, 0), it_upd(ncol, 0);
    std::vector<double> rrmax(ncol, 0.0), rrupd(ncol, 0.0);
    int ndone = 0;
    reset_host_state(c, ncol);
    for (int j = 0; j < ncol; j++) {
        const double rr = c->host_dots[3 * j];
        if (!std::isfinite(rr)) *nonfinite = true;
        rel[j] = bb[j] > 0 ? std::sqrt(rr / bb[j]) : 0.0;
        done[j] = (bb[j] == 0 || rel[j] <= tol) ? 1 : 0;
        ndone += done[j];
        mask[j] = done[j] ? 0 : 2;
        ColState& s = c->host_state[j];
        s.active = !done[j];
        s.rho_re = rr;
        s.alpha_re = s.omega_re = 1.0;
        s.rr = rr;
        s.rh2 = rr;
        s.bb = bb[j];
        s.stop2 = 0.25 * tol * tol * bb[j];
        rrmax[j] = rr;
        rrupd[j] = rr;
    }
    if (*nonfinite) return DD_OK;
    int total = 0, updates = 0;
    if (ndone < ncol) {
        DD_HIP(c, hipMemcpyAsync(mask_dev, mask.data(), sizeof(int) * ncol, hipMemcpyHostToDevice, c->stream));
        launch_set_resid<R>(c, n, ncol, r64, w.r, mask_dev);
        launch_restart_dirs<R>(c, n, ncol, w.r, w.rh, w.p, w.v, mask_dev);
        e = push_state(c, st, ncol);
        if (e != DD_OK) return e;
        DD_HIP(c, hipStreamSynchronize(c->stream));  // mask.data() is pageable host memory
    }
    while (ndone < ncol && total < p.max_iter) {
        const int k = std::min(check_every, p.max_iter - total);
        for (int it = 0; it < k; it++) {
            launch_bicg_p<R>(c, n, ncol, w.r, w.p, w.v, st);
            launch_dslash<R>(c, g, UK, kappa, dag, EPI_DOT_AUX, w.p, w.v, w.rh, ncol, partial, st);
            launch_finalize(c, FIN_ALPHA, ncol, nsb, partial, st, nullptr);
            launch_bicg_s<R>(c, n, ncol, w.r, w.v, w.s, st);
            launch_dslash<R>(c, g, UK, kappa, dag, EPI_TS, w.s, w.t, nullptr, ncol, partial, st);
            launch_finalize(c, FIN_OMEGA, ncol, nsb, partial, st, nullptr);
            launch_bicg_xr<R>(c, n, ncol, xx, w.r, w.p, w.s, w.t, w.rh, partial, st);
            launch_finalize(c, FIN_RHO, ncol, nbe, partial, st, nullptr);
        }
        e = pull_state(c, st, ncol);
        if (e != DD_OK) return e;
        int mx = 0, ntrig = 0;
        for (int j = 0; j < ncol; j++) {
            mx = std::max(mx, c->host_state[j].iters);
            mask[j] = 0;
            if (done[j]) continue;
            const ColState& s = c->host_state[j];
            if (s.breakdown == 2) {
                *nonfinite = true;
                break;
            }
            // A low-precision recursion can lose bi-orthogonality and drift up or
            // stall; such a column restarts (fresh shadow residual) from the true
            // residual: 100x above the last update, or 400 iterations with less
            // than a factor 2 of progress.
            const bool diverged = s.rr > 1e4 * rrupd[j];
            const bool stalled = s.iters - it_upd[j] > 400 && s.rr > 0.25 * rrupd[j];
            if (s.breakdown || diverged || stalled) {
                mask[j] = 2;
                (*restarts_out)++;
            }
            else if (!s.active || s.rr <= delta * delta * rrmax[j]) mask[j] = 1;
            else rrmax[j] = std::max(rrmax[j], s.rr);
            ntrig += mask[j] != 0;
        }
        total = std::max(total + 1, mx);
        if (*nonfinite) break;
        if (ntrig == 0) continue;
        // reliable update of the triggered columns
        updates++;
        static const bool dbg = std::getenv("DD_DEBUG") != nullptr;
        DD_HIP(c, hipMemcpyAsync(mask_dev, mask.data(), sizeof(int) * ncol, hipMemcpyHostToDevice, c->stream));
        if (fold) launch_fold_x<R>(c, n, ncol, x, xk, mask_dev);
        e = residual_to_host(c, g, U64, kappa, dag, ncol, b, x, r64, partial, dots);
        if (e != DD_OK) return e;
        for (int j = 0; j < ncol; j++) {
            if (!mask[j]) continue;
            const double rr = c->host_dots[3 * j];
            ColState& s = c->host_state[j];
            if (!std::isfinite(rr)) {
                *nonfinite = true;
                break;
            }
            rel[j] = std::sqrt(rr / bb[j]);
            if (dbg)
                std::fprintf(stderr, "[dd] it %d col %d update type %d: recursive %.3e true %.3e (rrmax %.3e)\n", total, j,
                             mask[j], std::sqrt(s.rr / bb[j]), rel[j], std::sqrt(rrmax[j] / bb[j]));
            if (rel[j] <= tol) {
                done[j] = 1;
                ndone++;
                s.active = 0;
                mask[j] = 0;
                continue;
            }
            s.active = 1;
            s.rr = rr;
            rrmax[j] = rr;
            rrupd[j] = rr;
            it_upd[j] = s.iters;
            if (mask[j] == 2) {  // breakdown / drift: fresh shadow residual, directions reset
                s.breakdown = 0;
                s.rho_re = rr;
                s.rho_im = 0;
                s.rh2 = rr;
                s.alpha_re = s.omega_re = 1.0;
                s.alpha_im = s.omega_im = 0.0;
                s.beta_re = s.beta_im = 0.0;
            }
        }
        if (*nonfinite) break;
        DD_HIP(c, hipMemcpyAsync(mask_dev, mask.data(), sizeof(int) * ncol, hipMemcpyHostToDevice, c->stream));
        launch_set_resid<R>(c, n, ncol, r64, w.r, mask_dev);
        launch_restart_dirs<R>(c, n, ncol, w.r, w.rh, w.p, w.v, mask_dev);
        e = push_state(c, st, ncol);
        if (e != DD_OK) return e;
        DD_HIP(c, hipStreamSynchronize(c->stream));
    }
    // whatever the exit, x must hold the full correction and rel the true residuals
    if (fold) {
        for (int j = 0; j < ncol; j++) mask[j] = 1;
        DD_HIP(c, hipMemcpyAsync(mask_dev, mask.data(), sizeof(int) * ncol, hipMemcpyHostToDevice, c->stream));
        launch_fold_x<R>(c, n, ncol, x, xk, mask_dev);
    }
    e = residual_to_host(c, g, U64, kappa, dag, ncol, b, x, r64, partial, dots);
    if (e != DD_OK) return e;
    for (int j = 0; j < ncol; j++) {
        const double rr = c->host_dots[3 * j];
        if (!std::isfinite(rr)) *nonfinite = true;
        rel[j] = bb[j] > 0 ? std::sqrt(rr / bb[j]) : 0.0;
    }
    *total_out = total;
    *updates_out = updates;
    return DD_OK;
}


// CGNR (CG on A^+ A x = A^+ b) with reliable updates: the Krylov vectors live in
// precision R; when a column's residual has dropped by delta, or the recursion
// stopped, the host folds the correction into the FP64 solution, recomputes the
// true FP64 residual r = b - A x, replaces the recursive r, recomputes
// z = A^+ r and shifts the search direction by the change of z
// (p <- p + z_new - z_old, which keeps its conjugate history).
template <typename R>
dd_status cgnr_reliable(dd_ctx* c, const Geo& g, const cpx<double>* U64, const cpx<R>* UK, double kappa, int dag,
                        int ncol, const cpx<double>* b, cpx<double>* x, const std::vector<double>& bb,
                        const dd_solver_params& p, double delta, const Vecs<R>& w, cpx<R>* xk, cpx<double>* r64,
                        ColState* st, double* partial, double* dots, int* mask_dev, std::vector<double>& rel,
                        int* total_out, int* updates_out, int* restarts_out, bool* nonfinite) {
    const int n = 12 * g.nsite;
    const size_t ntot = (size_t)n * ncol;
    const bool fold = !std::is_same<R, double>::value;
    const int check_every = p.check_every > 0 ? p.check_every : 8;
    const int nsb = stencil_slots(c, g, sizeof(R) == 8 ? 0 : 1, ncol);
    const int nbe = (n + kBlock - 1) / kBlock;
    const double tol = p.tol;
    cpx<R>* xx = fold ? xk : reinterpret_cast<cpx<R>*>(x);
    cpx<R>* r = w.r;
    cpx<R>* pp = w.p;
    cpx<R>* wv = w.v;
    cpx<R>* z = w.s;
    cpx<R>* tz = w.t;
    dd_status e;
    launch_zero<double>(c, ntot, x);
    if (fold) launch_zero<R>(c, ntot, xk);
    e = residual_to_host(c, g, U64, kappa, dag, ncol, b, x, r64, partial, dots);
    if (e != DD_OK) return e;
    std::vector<int> done(ncol, 0), mask(ncol, 0);
    std::vector<double> rrmax(ncol, 0.0);
    int ndone = 0;
    reset_host_state(c, ncol);
    for (int j = 0; j < ncol; j++) {
        const double rr = c->host_dots[3 * j];
        if (!std::isfinite(rr)) *nonfinite = true;
        rel[j] = bb[j] > 0 ? std::sqrt(rr / bb[j]) : 0.0;
        done[j] = (bb[j] == 0 || rel[j] <= tol) ? 1 : 0;
        ndone += done[j];
        mask[j] = !done[j];
        ColState& s = c->host_state[j];
        s.active = !done[j];
        s.rr = rr;
        s.bb = bb[j];
        s.stop2 = 0.25 * tol * tol * bb[j];
        rrmax[j] = rr;
    }
    if (*nonfinite) return DD_OK;
    int total = 0, updates = 0;
    if (ndone < ncol) {
        DD_HIP(c, hipMemcpyAsync(mask_dev, mask.data(), sizeof(int) * ncol, hipMemcpyHostToDevice, c->stream));
        launch_set_resid<R>(c, n, ncol, r64, r, mask_dev);
        e = push_state(c, st, ncol);
        if (e != DD_OK) return e;
        launch_dslash<R>(c, g, UK, kappa, 1 - dag, EPI_NORM, r, z, nullptr, ncol, partial, st);
        launch_finalize(c, FIN_CG_ZZ, ncol, nsb, partial, st, nullptr);
        launch_copy_cols<R>(c, n, ncol, z, pp, st);
        DD_HIP(c, hipStreamSynchronize(c->stream));
    }
    while (ndone < ncol && total < p.max_iter) {
        const int k = std::min(check_every, p.max_iter - total);
        for (int it = 0; it < k; it++) {
            launch_dslash<R>(c, g, UK, kappa, dag, EPI_NORM, pp, wv, nullptr, ncol, partial, st);
            launch_finalize(c, FIN_CG_ALPHA, ncol, nsb, partial, st, nullptr);
            launch_cg_xr<R>(c, n, ncol, xx, r, pp, wv, partial, st);
            launch_finalize(c, FIN_CG_RR, ncol, nbe, partial, st, nullptr);
            launch_dslash<R>(c, g, UK, kappa, 1 - dag, EPI_NORM, r, z, nullptr, ncol, partial, st);
            launch_finalize(c, FIN_CG_BETA, ncol, nsb, partial, st, nullptr);
            launch_cg_p<R>(c, n, ncol, pp, z, st);
        }
        e = pull_state(c, st, ncol);
        if (e != DD_OK) return e;
        int mx = 0, ntrig = 0;
        for (int j = 0; j < ncol; j++) {
            mx = std::max(mx, c->host_state[j].iters);
            mask[j] = 0;
            if (done[j]) continue;
            const ColState& s = c->host_state[j];
            if (s.breakdown == 2) {
                *nonfinite = true;
                break;
            }
            if (s.breakdown) (*restarts_out)++;
            if (s.breakdown || !s.active || s.rr <= delta * delta * rrmax[j]) mask[j] = 1;
            else rrmax[j] = std::max(rrmax[j], s.rr);
            ntrig += mask[j];
        }
        total = std::max(total + 1, mx);
        if (*nonfinite) break;
        if (ntrig == 0) continue;
        updates++;
        DD_HIP(c, hipMemcpyAsync(mask_dev, mask.data(), sizeof(int) * ncol, hipMemcpyHostToDevice, c->stream));
        if (fold) launch_fold_x<R>(c, n, ncol, x, xk, mask_dev);
        e = residual_to_host(c, g, U64, kappa, dag, ncol, b, x, r64, partial, dots);
        if (e != DD_OK) return e;
        std::vector<int> keep_active(ncol, 0);
        for (int j = 0; j < ncol; j++) {
            ColState& s = c->host_state[j];
            keep_active[j] = (!done[j] && !mask[j]) ? s.active : 0;
            if (!mask[j]) continue;
            const double rr = c->host_dots[3 * j];
            if (!std::isfinite(rr)) {
                *nonfinite = true;
                break;
            }
            rel[j] = std::sqrt(rr / bb[j]);
            if (rel[j] <= tol) {
                done[j] = 1;
                ndone++;
                mask[j] = 0;
                s.active = 0;
                continue;
            }
            s.rr = rr;
            s.breakdown = 0;
            rrmax[j] = rr;
        }
        if (*nonfinite) break;
        // recompute z = A^+ r for the updated columns only: mark them active
        for (int j = 0; j < ncol; j++) c->host_state[j].active = mask[j];
        DD_HIP(c, hipMemcpyAsync(mask_dev, mask.data(), sizeof(int) * ncol, hipMemcpyHostToDevice, c->stream));
        launch_set_resid<R>(c, n, ncol, r64, r, mask_dev);
        e = push_state(c, st, ncol);
        if (e != DD_OK) return e;
        launch_dslash<R>(c, g, UK, kappa, 1 - dag, EPI_NORM, r, tz, nullptr, ncol, partial, st);
        launch_finalize(c, FIN_CG_ZZ, ncol, nsb, partial, st, nullptr);
        launch_cg_shift<R>(c, n, ncol, pp, z, tz, mask_dev);
        e = pull_state(c, st, ncol);  // picks up the new zz
        if (e != DD_OK) return e;
        for (int j = 0; j < ncol; j++) c->host_state[j].active = mask[j] ? 1 : keep_active[j];
        e = push_state(c, st, ncol);
        if (e != DD_OK) return e;
        DD_HIP(c, hipStreamSynchronize(c->stream));
    }
    if (fold) {
        for (int j = 0; j < ncol; j++) mask[j] = 1;
        DD_HIP(c, hipMemcpyAsync(mask_dev, mask.data(), sizeof(int) * ncol, hipMemcpyHostToDevice, c->stream));
        launch_fold_x<R>(c, n, ncol, x, xk, mask_dev);
    }
    e = residual_to_host(c, g, U64, kappa, dag, ncol, b, x, r64, partial, dots);
    if (e != DD_OK) return e;
    for (int j = 0; j < ncol; j++) {
        const double rr = c->host_dots[3 * j];
        if (!std::isfinite(rr)) *nonfinite = true;
        rel[j] = bb[j] > 0 ? std::sqrt(rr / bb[j]) : 0.0;
    }
    *total_out = total;
    *updates_out = updates;
    return DD_OK;
}

}  // namespace

// Solve A x = b with A = D_Lambda (dag = 0) or D_Lambda^+ (dag = 1).
dd_status solve(dd_ctx* c, const cpx<double>* U, double kappa, const Geo& g, int ncol, const cpx<double>* b,
                cpx<double>* x, const dd_solver_params& p, dd_solve_stats* stats, int dag) {
    const auto t_start = std::chrono::steady_clock::now();
    const int n = 12 * g.nsite;
    const size_t ntot = (size_t)n * ncol;
    const int kind = p.solver;
    dd_status e = DD_OK;
    e = ensure_host(c, ncol);
    if (e != DD_OK) return e;

    // partial-sum slots: the larger of the vector kernels' and the stencils' counts
    int slots = (n + kBlock - 1) / kBlock;
    slots = std::max(slots, stencil_slots(c, g, 0, ncol));
    if (p.prec == DD_MIXED) slots = std::max(slots, stencil_slots(c, g, 1, ncol));
    const size_t npart = (size_t)ncol * slots * 3;
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
    if (p.prec == DD_MIXED) {
        e = get_vecs<float>(c, ntot, &w32);
        if (e != DD_OK) return e;
        const size_t nl = (size_t)36 * g.vlink;
        U32 = (cpx<float>*)workspace(c, W_U32, nl * sizeof(cpx<float>), &e);
        if (e != DD_OK) return e;
        x32 = (cpx<float>*)workspace(c, W_X32, ntot * sizeof(cpx<float>), &e);
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

    int total = 0, updates = 0, restarts = 0;
    bool converged = false, nonfinite = false;
    const double tol = p.tol;
    {
        int* mask_dev = (int*)workspace(c, W_AUX4, sizeof(int) * ncol, &e);
        if (e != DD_OK) return e;
        cpx<double>* r64 = (cpx<double>*)workspace(c, W_RES64, ntot * sizeof(cpx<double>), &e);
        if (e != DD_OK) return e;
        const double delta = p.delta > 0 ? p.delta : (p.prec == DD_MIXED ? 0.01 : 0.1);
        if (kind == DD_BICGSTAB && p.prec == DD_MIXED)
            e = bicgstab_reliable<float>(c, g, U, U32, kappa, dag, ncol, b, x, bb, p, delta, w32, x32, r64, st, partial,
                                         dots, mask_dev, rel, &total, &updates, &restarts, &nonfinite);
        else if (kind == DD_BICGSTAB)
            e = bicgstab_reliable<double>(c, g, U, U, kappa, dag, ncol, b, x, bb, p, delta, w64, nullptr, r64, st,
                                          partial, dots, mask_dev, rel, &total, &updates, &restarts, &nonfinite);
        else if (p.prec == DD_MIXED)
            e = cgnr_reliable<float>(c, g, U, U32, kappa, dag, ncol, b, x, bb, p, delta, w32, x32, r64, st, partial,
                                     dots, mask_dev, rel, &total, &updates, &restarts, &nonfinite);
        else
            e = cgnr_reliable<double>(c, g, U, U, kappa, dag, ncol, b, x, bb, p, delta, w64, nullptr, r64, st, partial,
                                      dots, mask_dev, rel, &total, &updates, &restarts, &nonfinite);
        if (e != DD_OK) return e;
        converged = !nonfinite;
        for (int j = 0; j < ncol; j++)
            if (!(rel[j] <= tol)) converged = false;
    }
    if (stats) {
        stats->nrhs = ncol;
        stats->iters = total;
        stats->updates = updates;
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
