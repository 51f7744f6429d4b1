// solver.hip -- Krylov solvers for M x = b, every segment (column of one
// lattice or slab, or column of one domain of a batch) advancing together: one
// stencil launch serves every segment and the vector kernels cover them all.
//
// The scalars of each segment live on the device (ColState) and are updated by
// one-workgroup-per-segment finalize kernels, so iterations run without host
// round trips; the host reads the per-segment state every `check_every`
// iterations.  A System may ask for those inner iterations to be captured
// once into a HIP graph and replayed.
//
// Both methods (BiCGStab on D, CGNR = CG on D^+ D) use reliable updates: the
// Krylov recursion runs in precision R (FP64, or FP32 links and vectors for
// DD_MIXED with inner products accumulated in FP64), and whenever a segment's
// recursive residual has dropped by the factor delta the correction is folded
// into the FP64 solution and the recursive residual is replaced by the true
// FP64 residual b - D x.  Convergence is decided on that true residual only.
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

dd_status ensure_host(dd_ctx* c, int n) {
    if (c->host_n >= n) return DD_OK;
    if (c->host_state) (void)hipHostFree(c->host_state);
    if (c->host_dots) (void)hipHostFree(c->host_dots);
    c->host_state = nullptr;
    c->host_dots = nullptr;
    c->host_n = 0;
    DD_HIP(c, hipHostMalloc((void**)&c->host_state, sizeof(ColState) * n, hipHostMallocDefault));
    DD_HIP(c, hipHostMalloc((void**)&c->host_dots, sizeof(double) * 3 * n, hipHostMallocDefault));
    c->host_n = n;
    return DD_OK;
}

dd_status pull_state(dd_ctx* c, const ColState* dev, int n) {
    DD_HIP(c, hipGetLastError());
    DD_HIP(c, hipMemcpyAsync(c->host_state, dev, sizeof(ColState) * n, hipMemcpyDeviceToHost, c->stream));
    DD_HIP(c, hipStreamSynchronize(c->stream));
    return DD_OK;
}

dd_status push_state(dd_ctx* c, ColState* dev, int n) {
    DD_HIP(c, hipMemcpyAsync(dev, c->host_state, sizeof(ColState) * n, hipMemcpyHostToDevice, c->stream));
    return DD_OK;
}

void reset_host_state(dd_ctx* c, int n) { std::memset(c->host_state, 0, sizeof(ColState) * n); }

// Kernel timing bills the columns the host mirror shows active (exact for the masked
// launches of the reliable updates; for a round of inner iterations the share at its start,
// so a column that stops inside a round is billed until the round ends).
void bill_active(dd_ctx* c, int ns) {
    int n = 0;
    for (int j = 0; j < ns; j++) n += c->host_state[j].active != 0;
    c->bill_frac = ns > 0 ? (double)n / ns : 1.0;
}

// Copy a per-segment mask from (pageable) host memory and wait for the copy.
dd_status push_mask(dd_ctx* c, int* dev, const std::vector<int>& mask) {
    DD_HIP(c, hipMemcpyAsync(dev, mask.data(), sizeof(int) * mask.size(), hipMemcpyHostToDevice, c->stream));
    DD_HIP(c, hipStreamSynchronize(c->stream));
    return DD_OK;
}

// |a_seg|^2 for every segment, read back to host_dots[3*seg].
template <typename R>
dd_status norms_to_host(System& S, const cpx<R>* a, double* partial, double* dots) {
    dd_ctx* c = S.c;
    launch_norm2<R>(c, S.seg, a, partial);
    launch_finalize(c, FIN_STORE, S.nseg, S.seg.eb0, partial, nullptr, dots);
    DD_HIP(c, hipGetLastError());
    DD_HIP(c, hipMemcpyAsync(c->host_dots, dots, sizeof(double) * 3 * S.nseg, hipMemcpyDeviceToHost, c->stream));
    DD_HIP(c, hipStreamSynchronize(c->stream));
    return DD_OK;
}

// r = b - M x (FP64) and |r|^2 per segment into host_dots[3*seg].
dd_status residual_to_host(System& S, const cpx<double>* b, const cpx<double>* x, cpx<double>* r,
                           double* partial, double* dots) {
    dd_ctx* c = S.c;
    c->bill_frac = 1.0;  // every column
    S.apply64(0, EPI_RESID, x, r, b, partial, nullptr);
    launch_finalize(c, FIN_STORE, S.nseg, S.sp0[0], partial, nullptr, dots);
    DD_HIP(c, hipGetLastError());
    DD_HIP(c, hipMemcpyAsync(c->host_dots, dots, sizeof(double) * 3 * S.nseg, hipMemcpyDeviceToHost, c->stream));
    DD_HIP(c, hipStreamSynchronize(c->stream));
    return DD_OK;
}

// Runs `k` inner iterations, either by direct launches or, when the System
// asks for it and k is the usual round length, by replaying a HIP graph
// captured from the first such round (the launches' arguments do not change
// during a solve).  Kernel timing is off while capturing.
class InnerRounds {
  public:
    InnerRounds(System& S, int round) : S_(S), round_(round) {}
    ~InnerRounds() {
        if (exec_) (void)hipGraphExecDestroy(exec_);
        if (graph_) (void)hipGraphDestroy(graph_);
    }
    InnerRounds(const InnerRounds&) = delete;
    InnerRounds& operator=(const InnerRounds&) = delete;
    template <typename F>
    dd_status run(int k, F&& body) {
        dd_ctx* c = S_.c;
        if (!S_.graph || k != round_) {
            for (int it = 0; it < k; it++) body();
            return DD_OK;
        }
        if (!exec_) {
            const int saved = c->timing;
            c->timing = 0;
            DD_HIP(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
            for (int it = 0; it < k; it++) body();
            const hipError_t e = hipStreamEndCapture(c->stream, &graph_);
            c->timing = saved;
            DD_HIP(c, e);
            DD_HIP(c, hipGraphInstantiate(&exec_, graph_, nullptr, nullptr, 0));
        }
        DD_HIP(c, hipGraphLaunch(exec_, c->stream));
        return DD_OK;
    }

  private:
    System& S_;
    int round_;
    hipGraph_t graph_ = nullptr;
    hipGraphExec_t exec_ = nullptr;
};

struct Work {
    ColState* st;
    double* partial;
    double* dots;
    int* mask_dev;
    cpx<double>* r64;
};

// BiCGStab with reliable updates (Sleijpen & van der Vorst, Computing 56 (1996)
// 141): whenever a segment's recursive residual has dropped by delta below the
// largest one seen since its last update, or the recursion claims
// convergence, or it broke down, the host
//   - folds the accumulated correction into the FP64 solution (R = float),
//   - recomputes the true residual r = b - D x in FP64,
//   - finishes the segment if |r|/|b| <= tol, otherwise replaces the recursive
//     residual by the true one and continues with the same search directions
//     (a breakdown or a stalled recursion also takes a fresh shadow residual).
// For R = double the correction goes straight into x.
template <typename R>
dd_status bicgstab_reliable(System& S, const cpx<double>* b, cpx<double>* x, const std::vector<double>& bb,
                            const dd_solver_params& p, double delta, const Vecs<R>& w, cpx<R>* xk, const Work& W,
                            SolveResult* res, bool* nonfinite) {
    dd_ctx* c = S.c;
    const int ns = S.nseg;
    const bool fold = !std::is_same<R, double>::value;
    const int check_every = p.check_every > 0 ? p.check_every : 8;
    const int kind = sizeof(R) == 8 ? 0 : 1;
    const double tol = p.tol;
    cpx<R>* xx = fold ? xk : reinterpret_cast<cpx<R>*>(x);
    ColState* st = W.st;
    double* partial = W.partial;
    dd_status e;
    if (!p.x0) launch_zero<double>(c, S.nelem, x);  // else x holds the caller's guess
    if (fold) launch_zero<R>(c, S.nelem, xk);
    e = residual_to_host(S, b, x, W.r64, partial, W.dots);
    if (e != DD_OK) return e;
    std::vector<int> done(ns, 0), mask(ns, 0), it_upd(ns, 0);
    std::vector<double> rrmax(ns, 0.0), rrupd(ns, 0.0);
    int ndone = 0;
    reset_host_state(c, ns);
    for (int j = 0; j < ns; j++) {
        const double rr = c->host_dots[3 * j];
        if (!std::isfinite(rr)) *nonfinite = true;
        res->rel[j] = bb[j] > 0 ? std::sqrt(rr / bb[j]) : 0.0;
        done[j] = (bb[j] == 0 || res->rel[j] <= tol) ? 1 : 0;
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
    int total = 0;
    if (ndone < ns) {
        e = push_mask(c, W.mask_dev, mask);
        if (e != DD_OK) return e;
        launch_set_resid<R>(c, S.seg, W.r64, w.r, W.mask_dev);
        launch_restart_dirs<R>(c, S.seg, w.r, w.rh, w.p, w.v, W.mask_dev);
        e = push_state(c, st, ns);
        if (e != DD_OK) return e;
    }
    InnerRounds rounds(S, check_every);
    auto iteration = [&]() {
        launch_bicg_p<R>(c, S.seg, w.r, w.p, w.v, st);
        S.apply(0, EPI_DOT_AUX, w.p, w.v, w.rh, partial, st);
        launch_finalize(c, FIN_ALPHA, ns, S.sp0[kind], partial, st, nullptr);
        launch_bicg_s<R>(c, S.seg, w.r, w.v, w.s, st);
        S.apply(0, EPI_TS, w.s, w.t, (const cpx<R>*)nullptr, partial, st);
        launch_finalize(c, FIN_OMEGA, ns, S.sp0[kind], partial, st, nullptr);
        launch_bicg_xr<R>(c, S.seg, xx, w.r, w.p, w.s, w.t, w.rh, partial, st);
        launch_finalize(c, FIN_RHO, ns, S.seg.eb0, partial, st, nullptr);
    };
    static const bool dbg = std::getenv("DD_DEBUG") != nullptr;
    while (ndone < ns && total < p.max_iter) {
        const int k = std::min(check_every, p.max_iter - total);
        bill_active(c, ns);
        e = rounds.run(k, iteration);
        if (e != DD_OK) return e;
        e = pull_state(c, st, ns);
        if (e != DD_OK) return e;
        int mx = 0, ntrig = 0;
        for (int j = 0; j < ns; j++) {
            mx = std::max(mx, c->host_state[j].iters);
            mask[j] = 0;
            if (done[j]) continue;
            const ColState& s = c->host_state[j];
            // A breakdown (an exact zero, or a non-finite alpha, omega or rho: the
            // finalize kernel stops the segment before its solution is updated) takes
            // a fresh start from the true residual of the last finite iterate; only a
            // non-finite true residual is an error.
            // A low-precision recursion can lose bi-orthogonality and drift up or
            // stall; such a segment restarts (fresh shadow residual) from the true
            // residual: 100x above the last update, or 400 iterations with less
            // than a factor 2 of progress.
            const bool diverged = s.rr > 1e4 * rrupd[j];
            const bool stalled = s.iters - it_upd[j] > 400 && s.rr > 0.25 * rrupd[j];
            if (s.breakdown || diverged || stalled) {
                mask[j] = 2;
                res->restarts++;
            } else if (!s.active || s.rr <= delta * delta * rrmax[j]) {
                mask[j] = 1;
            } else {
                rrmax[j] = std::max(rrmax[j], s.rr);
            }
            ntrig += mask[j] != 0;
        }
        total = std::max(total + 1, mx);
        if (*nonfinite) break;
        if (ntrig == 0) continue;
        res->updates++;
        e = push_mask(c, W.mask_dev, mask);
        if (e != DD_OK) return e;
        if (fold) launch_fold_x<R>(c, S.seg, x, xk, W.mask_dev);
        e = residual_to_host(S, b, x, W.r64, partial, W.dots);
        if (e != DD_OK) return e;
        for (int j = 0; j < ns; j++) {
            if (!mask[j]) continue;
            const double rr = c->host_dots[3 * j];
            ColState& s = c->host_state[j];
            if (!std::isfinite(rr)) {
                *nonfinite = true;
                break;
            }
            res->rel[j] = std::sqrt(rr / bb[j]);
            if (dbg)
                std::fprintf(stderr, "[dd] it %d seg %d update type %d: recursive %.3e true %.3e (rrmax %.3e)\n",
                             total, j, mask[j], std::sqrt(s.rr / bb[j]), res->rel[j], std::sqrt(rrmax[j] / bb[j]));
            if (res->rel[j] <= tol) {
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
            if (mask[j] == 2) {
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
        e = push_mask(c, W.mask_dev, mask);
        if (e != DD_OK) return e;
        launch_set_resid<R>(c, S.seg, W.r64, w.r, W.mask_dev);
        launch_restart_dirs<R>(c, S.seg, w.r, w.rh, w.p, w.v, W.mask_dev);
        e = push_state(c, st, ns);
        if (e != DD_OK) return e;
    }
    res->iters = total;
    return DD_OK;
}

// CGNR (CG on D^+ D x = D^+ b) with reliable updates: when a segment's residual
// has dropped by delta, or the recursion stopped, the host folds the correction
// into the FP64 solution, recomputes the true FP64 residual r = b - D x,
// replaces the recursive r, recomputes z = D^+ r and shifts the search
// direction by the change of z (p <- p + z_new - z_old, which keeps its
// conjugate history).
template <typename R>
dd_status cgnr_reliable(System& S, const cpx<double>* b, cpx<double>* x, const std::vector<double>& bb,
                        const dd_solver_params& p, double delta, const Vecs<R>& w, cpx<R>* xk, const Work& W,
                        SolveResult* res, bool* nonfinite) {
    dd_ctx* c = S.c;
    const int ns = S.nseg;
    const bool fold = !std::is_same<R, double>::value;
    const int check_every = p.check_every > 0 ? p.check_every : 8;
    const int kind = sizeof(R) == 8 ? 0 : 1;
    const double tol = p.tol;
    cpx<R>* xx = fold ? xk : reinterpret_cast<cpx<R>*>(x);
    cpx<R>* r = w.r;
    cpx<R>* pp = w.p;
    cpx<R>* wv = w.v;
    cpx<R>* z = w.s;
    cpx<R>* tz = w.t;
    ColState* st = W.st;
    double* partial = W.partial;
    dd_status e;
    if (!p.x0) launch_zero<double>(c, S.nelem, x);  // else x holds the caller's guess
    if (fold) launch_zero<R>(c, S.nelem, xk);
    e = residual_to_host(S, b, x, W.r64, partial, W.dots);
    if (e != DD_OK) return e;
    std::vector<int> done(ns, 0), mask(ns, 0);
    std::vector<double> rrmax(ns, 0.0);
    int ndone = 0;
    reset_host_state(c, ns);
    for (int j = 0; j < ns; j++) {
        const double rr = c->host_dots[3 * j];
        if (!std::isfinite(rr)) *nonfinite = true;
        res->rel[j] = bb[j] > 0 ? std::sqrt(rr / bb[j]) : 0.0;
        done[j] = (bb[j] == 0 || res->rel[j] <= tol) ? 1 : 0;
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
    int total = 0;
    if (ndone < ns) {
        e = push_mask(c, W.mask_dev, mask);
        if (e != DD_OK) return e;
        launch_set_resid<R>(c, S.seg, W.r64, r, W.mask_dev);
        e = push_state(c, st, ns);
        if (e != DD_OK) return e;
        bill_active(c, ns);
        S.apply(1, EPI_NORM, r, z, (const cpx<R>*)nullptr, partial, st);
        launch_finalize(c, FIN_CG_ZZ, ns, S.sp0[kind], partial, st, nullptr);
        launch_copy_segs<R>(c, S.seg, z, pp, st);
    }
    InnerRounds rounds(S, check_every);
    auto iteration = [&]() {
        S.apply(0, EPI_NORM, pp, wv, (const cpx<R>*)nullptr, partial, st);
        launch_finalize(c, FIN_CG_ALPHA, ns, S.sp0[kind], partial, st, nullptr);
        launch_cg_r<R>(c, S.seg, r, wv, partial, st);
        launch_finalize(c, FIN_CG_RR, ns, S.seg.eb0, partial, st, nullptr);
        S.apply(1, EPI_NORM, r, z, (const cpx<R>*)nullptr, partial, st);
        launch_finalize(c, FIN_CG_BETA, ns, S.sp0[kind], partial, st, nullptr);
        launch_cg_px<R>(c, S.seg, xx, pp, z, st);  // x += alpha p (also as a column stops), p = z + beta p
    };
    while (ndone < ns && total < p.max_iter) {
        const int k = std::min(check_every, p.max_iter - total);
        bill_active(c, ns);
        e = rounds.run(k, iteration);
        if (e != DD_OK) return e;
        e = pull_state(c, st, ns);
        if (e != DD_OK) return e;
        int mx = 0, ntrig = 0;
        for (int j = 0; j < ns; j++) {
            mx = std::max(mx, c->host_state[j].iters);
            mask[j] = 0;
            if (done[j]) continue;
            const ColState& s = c->host_state[j];
            if (s.breakdown == 2) {
                *nonfinite = true;
                break;
            }
            if (s.breakdown) res->restarts++;
            if (s.breakdown || !s.active || s.rr <= delta * delta * rrmax[j]) mask[j] = 1;
            else rrmax[j] = std::max(rrmax[j], s.rr);
            ntrig += mask[j];
        }
        total = std::max(total + 1, mx);
        if (*nonfinite) break;
        if (ntrig == 0) continue;
        res->updates++;
        e = push_mask(c, W.mask_dev, mask);
        if (e != DD_OK) return e;
        if (fold) launch_fold_x<R>(c, S.seg, x, xk, W.mask_dev);
        e = residual_to_host(S, b, x, W.r64, partial, W.dots);
        if (e != DD_OK) return e;
        std::vector<int> keep_active(ns, 0);
        for (int j = 0; j < ns; j++) {
            ColState& s = c->host_state[j];
            keep_active[j] = (!done[j] && !mask[j]) ? s.active : 0;
            if (!mask[j]) continue;
            const double rr = c->host_dots[3 * j];
            if (!std::isfinite(rr)) {
                *nonfinite = true;
                break;
            }
            res->rel[j] = std::sqrt(rr / bb[j]);
            if (res->rel[j] <= tol) {
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
        // recompute z = D^+ r for the updated segments only: mark them active
        for (int j = 0; j < ns; j++) c->host_state[j].active = mask[j];
        e = push_mask(c, W.mask_dev, mask);
        if (e != DD_OK) return e;
        launch_set_resid<R>(c, S.seg, W.r64, r, W.mask_dev);
        e = push_state(c, st, ns);
        if (e != DD_OK) return e;
        bill_active(c, ns);
        S.apply(1, EPI_NORM, r, tz, (const cpx<R>*)nullptr, partial, st);
        launch_finalize(c, FIN_CG_ZZ, ns, S.sp0[kind], partial, st, nullptr);
        launch_cg_shift<R>(c, S.seg, pp, z, tz, W.mask_dev);
        e = pull_state(c, st, ns);  // picks up the new zz
        if (e != DD_OK) return e;
        for (int j = 0; j < ns; j++) c->host_state[j].active = mask[j] ? 1 : keep_active[j];
        e = push_state(c, st, ns);
        if (e != DD_OK) return e;
    }
    res->iters = total;
    return DD_OK;
}

// The columns of one lattice or slab: segments are the ncol columns, the
// stencil is the time-sweep kernel of dirac.hip with its tuned schedule.
struct SingleSystem : System {
    Geo g{};
    const cpx<double>* U64 = nullptr;
    const cpx<float>* U32 = nullptr;
    double kappa = 0;
    int dag = 0;
    int ncol = 0;
    void apply64(int d, int epi, const cpx<double>* in, cpx<double>* out, const cpx<double>* aux, double* partial,
                 const ColState* st) override {
        launch_dslash<double>(c, g, U64, kappa, d ^ dag, epi, in, out, aux, ncol, partial, st);
    }
    void apply32(int d, int epi, const cpx<float>* in, cpx<float>* out, const cpx<float>* aux, double* partial,
                 const ColState* st) override {
        launch_dslash<float>(c, g, U32, kappa, d ^ dag, epi, in, out, aux, ncol, partial, st);
    }
};

}  // namespace

dd_status SegLayout::upload(dd_ctx* c, Slot slot, System* S) {
    const int ns = (int)off.size();
    // FP32 half fields pair their components (dd_eo.h), which segments must not split
    for (int k = 0; k < ns; k++)
        if ((off[k] & 1) != 0 || (len[k] & 1) != 0) return fail(c, DD_ERR_ARG, "segments must have even offsets and lengths");
    eb0.assign(ns + 1, 0);
    const int per = kBlock * kElems;  // elements per elementwise workgroup
    for (int k = 0; k < ns; k++) eb0[k + 1] = eb0[k] + (len[k] + per - 1) / per;
    const int neb = eb0[ns];
    eseg.resize(neb);
    for (int k = 0; k < ns; k++)
        for (int b = eb0[k]; b < eb0[k + 1]; b++) eseg[b] = k;
    // one allocation: off | len | eb0 | sp0[0] | sp0[1] | eseg
    const size_t n_off = (size_t)ns * sizeof(long long);
    const size_t n_int = (size_t)ns + (size_t)(ns + 1) * 3 + neb;
    dd_status e = DD_OK;
    char* base = (char*)workspace(c, slot, n_off + n_int * sizeof(int), &e);
    if (e != DD_OK) return e;
    std::vector<int> ints;
    ints.reserve(n_int);
    ints.insert(ints.end(), len.begin(), len.end());
    ints.insert(ints.end(), eb0.begin(), eb0.end());
    ints.insert(ints.end(), sp0[0].begin(), sp0[0].end());
    ints.insert(ints.end(), sp0[1].begin(), sp0[1].end());
    ints.insert(ints.end(), eseg.begin(), eseg.end());
    DD_HIP(c, hipMemcpyAsync(base, off.data(), n_off, hipMemcpyHostToDevice, c->stream));
    DD_HIP(c, hipMemcpyAsync(base + n_off, ints.data(), n_int * sizeof(int), hipMemcpyHostToDevice, c->stream));
    DD_HIP(c, hipStreamSynchronize(c->stream));  // the host vectors are pageable
    const int* ip = (const int*)(base + n_off);
    S->seg.off = (const long long*)base;
    S->seg.len = ip;
    S->seg.eb0 = ip + ns;
    S->sp0[0] = ip + ns + (ns + 1);
    S->sp0[1] = ip + ns + 2 * (ns + 1);
    S->seg.eseg = ip + ns + 3 * (ns + 1);
    S->seg.nseg = ns;
    S->seg.neb = neb;
    S->seg.paired = S->pair32 ? 1 : 0;
    S->nseg = ns;
    S->nslots = std::max(S->nslots, (size_t)neb);
    S->nslots = std::max(S->nslots, (size_t)sp0[0][ns]);
    S->nslots = std::max(S->nslots, (size_t)sp0[1][ns]);
    return DD_OK;
}

dd_status solve_system(System& S, const cpx<double>* b, cpx<double>* x, const dd_solver_params& p,
                       SolveResult* res) {
    dd_ctx* c = S.c;
    const int ns = S.nseg;
    dd_status e = ensure_host(c, ns);
    if (e != DD_OK) return e;
    Work W{};
    W.partial = (double*)workspace(c, W_PART, S.nslots * 3 * sizeof(double), &e);
    if (e != DD_OK) return e;
    W.st = (ColState*)workspace(c, W_STATE, sizeof(ColState) * ns, &e);
    if (e != DD_OK) return e;
    W.dots = (double*)workspace(c, W_DOTS, sizeof(double) * 3 * ns, &e);
    if (e != DD_OK) return e;
    W.mask_dev = (int*)workspace(c, W_AUX4, sizeof(int) * ns, &e);
    if (e != DD_OK) return e;
    W.r64 = (cpx<double>*)workspace(c, W_RES64, S.nelem * sizeof(cpx<double>), &e);
    if (e != DD_OK) return e;

    res->rel.assign(ns, 0.0);
    res->seg_iters.assign(ns, 0);
    e = norms_to_host<double>(S, b, W.partial, W.dots);
    if (e != DD_OK) return e;
    std::vector<double> bb(ns);
    for (int j = 0; j < ns; j++) bb[j] = c->host_dots[3 * j];
    for (int j = 0; j < ns; j++)
        if (!std::isfinite(bb[j])) return fail(c, DD_ERR_BREAKDOWN, "non-finite values in the right-hand side");
    // a zero source column has the zero solution, whatever guess x held
    if (p.x0) {
        std::vector<int> zmask(ns, 0);
        bool any = false;
        for (int j = 0; j < ns; j++) any = any || (zmask[j] = bb[j] == 0);
        if (any) {
            e = push_mask(c, W.mask_dev, zmask);
            if (e != DD_OK) return e;
            launch_zero_segs(c, S.seg, x, W.mask_dev);
        }
    }
    // relative residuals refer to |b|^2, or to the norm the System names (the
    // original source of a preconditioned system); a zero source stays done
    if (S.ref_norm2 != nullptr)
        for (int j = 0; j < ns; j++)
            if (bb[j] > 0) bb[j] = S.ref_norm2[j];

    const bool mixed = p.prec == DD_MIXED;
    if (mixed && !S.has32) return fail(c, DD_ERR_ARG, "DD_MIXED needs FP32 links");
    const double delta = p.delta > 0 ? p.delta : (mixed ? 0.01 : 0.1);
    bool nonfinite = false;
    cpx<float>* xk = nullptr;
    if (mixed) {
        Vecs<float> w;
        e = get_vecs<float>(c, S.nelem, &w);
        if (e != DD_OK) return e;
        xk = (cpx<float>*)workspace(c, W_X32, S.nelem * sizeof(cpx<float>), &e);
        if (e != DD_OK) return e;
        e = p.solver == DD_BICGSTAB ? bicgstab_reliable<float>(S, b, x, bb, p, delta, w, xk, W, res, &nonfinite)
                                    : cgnr_reliable<float>(S, b, x, bb, p, delta, w, xk, W, res, &nonfinite);
    } else {
        Vecs<double> w;
        e = get_vecs<double>(c, S.nelem, &w);
        if (e != DD_OK) return e;
        e = p.solver == DD_BICGSTAB ? bicgstab_reliable<double>(S, b, x, bb, p, delta, w, nullptr, W, res, &nonfinite)
                                    : cgnr_reliable<double>(S, b, x, bb, p, delta, w, nullptr, W, res, &nonfinite);
    }
    c->bill_frac = 1.0;
    if (e != DD_OK) return e;

    // whatever the exit, x holds the full correction: report the true residuals
    if (mixed) {
        e = push_mask(c, W.mask_dev, std::vector<int>(ns, 1));
        if (e != DD_OK) return e;
        launch_fold_x<float>(c, S.seg, x, xk, W.mask_dev);
    }
    e = residual_to_host(S, b, x, W.r64, W.partial, W.dots);
    if (e != DD_OK) return e;
    bool converged = !nonfinite;
    for (int j = 0; j < ns; j++) {
        const double rr = c->host_dots[3 * j];
        if (!std::isfinite(rr)) nonfinite = true;
        res->rel[j] = bb[j] > 0 ? std::sqrt(rr / bb[j]) : 0.0;
        res->seg_iters[j] = c->host_state[j].iters;
        if (!(res->rel[j] <= p.tol)) converged = false;
    }
    if (nonfinite) return fail(c, DD_ERR_BREAKDOWN, "non-finite values in the Krylov iteration");
    if (!converged) {
        double worst = 0;
        for (int j = 0; j < ns; j++) worst = std::max(worst, res->rel[j]);
        return fail(c, DD_ERR_NOCONV,
                    "solver stopped after " + std::to_string(res->iters) + " iterations with relative residual " +
                        std::to_string(worst) + " > tol " + std::to_string(p.tol));
    }
    return DD_OK;
}

dd_status segment_norms(dd_ctx* c, const std::vector<long long>& off, const std::vector<int>& len,
                        const cpx<double>* a, std::vector<double>* out) {
    struct NoStencil : System {
        void apply64(int, int, const cpx<double>*, cpx<double>*, const cpx<double>*, double*,
                     const ColState*) override {}
        void apply32(int, int, const cpx<float>*, cpx<float>*, const cpx<float>*, double*,
                     const ColState*) override {}
    } S;
    S.c = c;
    const int ns = (int)off.size();
    SegLayout lay;
    lay.off = off;
    lay.len = len;
    lay.sp0[0].assign(ns + 1, 0);
    lay.sp0[1].assign(ns + 1, 0);
    dd_status e = lay.upload(c, W_SEGN, &S);  // own slot: a System's tables may be live in W_SEGS
    if (e != DD_OK) return e;
    e = ensure_host(c, ns);
    if (e != DD_OK) return e;
    double* partial = (double*)workspace(c, W_PART, S.nslots * 3 * sizeof(double), &e);
    if (e != DD_OK) return e;
    double* dots = (double*)workspace(c, W_DOTS, sizeof(double) * 3 * ns, &e);
    if (e != DD_OK) return e;
    e = norms_to_host<double>(S, a, partial, dots);
    if (e != DD_OK) return e;
    out->resize(ns);
    for (int k = 0; k < ns; k++) (*out)[k] = c->host_dots[3 * k];
    return DD_OK;
}

dd_status column_norms(dd_ctx* c, int n, int ncol, const cpx<double>* a, std::vector<double>* out) {
    std::vector<long long> off(ncol);
    std::vector<int> len(ncol, n);
    for (int k = 0; k < ncol; k++) off[k] = (long long)k * n;
    return segment_norms(c, off, len, a, out);
}

// Solve M x = b on one lattice or slab for ncol columns (M = D, or D^+ for dag).
dd_status solve(dd_ctx* c, const cpx<double>* U, double kappa, const Geo& g, int ncol, const cpx<double>* b,
                cpx<double>* x, const dd_solver_params& p, dd_solve_stats* stats, int dag) {
    if (p.precond == DD_PRECOND_EO && eo_applicable(g)) return solve_eo(c, U, kappa, g, ncol, b, x, p, stats, dag);
    const auto t_start = std::chrono::steady_clock::now();
    SingleSystem S;
    S.c = c;
    S.g = g;
    S.U64 = U;
    S.kappa = kappa;
    S.dag = dag;
    S.ncol = ncol;
    const int n = 12 * g.nsite;
    S.nelem = (size_t)n * ncol;
    dd_status e = DD_OK;
    if (p.prec == DD_MIXED) {
        const size_t nl = (size_t)36 * g.vlink;
        cpx<float>* U32 = (cpx<float>*)workspace(c, W_U32, nl * sizeof(cpx<float>), &e);
        if (e != DD_OK) return e;
        launch_links_to_f32(c, nl, U, U32);
        S.U32 = U32;
        S.has32 = true;
    }
    SegLayout lay;
    lay.off.resize(ncol);
    lay.len.assign(ncol, n);
    for (int k = 0; k < ncol; k++) lay.off[k] = (long long)k * n;
    for (int kind = 0; kind < 2; kind++) {
        const int per = (kind == 1 && !S.has32) ? 0 : stencil_slots(c, g, kind, ncol);
        lay.sp0[kind].resize(ncol + 1);
        for (int k = 0; k <= ncol; k++) lay.sp0[kind][k] = k * per;
    }
    e = lay.upload(c, W_SEGS, &S);
    if (e != DD_OK) return e;
    SolveResult res;
    const dd_status st = solve_system(S, b, x, p, &res);
    if (stats && (st == DD_OK || st == DD_ERR_NOCONV || st == DD_ERR_BREAKDOWN)) {
        stats->nrhs = ncol;
        stats->iters = res.iters;
        stats->updates = res.updates;
        stats->restarts = res.restarts;
        for (int j = 0; j < DD_MAX_RHS; j++)
            stats->true_rel_resid[j] = (j < ncol && j < (int)res.rel.size()) ? res.rel[j] : 0.0;
        stats->ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    }
    return st;
}

}  // namespace dd
