/*
 * dd.h -- C ABI of the MI355X (gfx950) Wilson-Dirac library for the factorised
 * (domain-decomposed) quark propagator of M. Ce, L. Giusti, S. Schaefer,
 * "Domain decomposition and multilevel integration for fermions",
 * PoS LATTICE2016, arXiv:1612.06424.
 *
 * Every compute step runs in hand-written HIP kernels in libdd.so.
 *
 * ---------------------------------------------------------------- layouts
 * Lattice T x L^3, site s = ((t*L + z)*L + y)*L + x (time slowest, x fastest);
 * mu = 0 is time, mu = 1,2,3 are x,y,z.  Space is periodic; the time edge
 * (hop between t = T-1 and t = 0) carries the factor time_bc.
 *
 * Links U: device array of complex numbers (interleaved re, im), structure of
 *   arrays [4][9][V]: element (mu, k, s) is entry k = 3*row + col of U_mu(s).
 *   complex128 for DD_FP64 / DD_MIXED entry points, complex64 for DD_FP32.
 * Spinor fields: device array [ncol][12][nsite] of complex, component
 *   c = 3*spin + colour, site fastest.  On a time slab (dd_domain) [t0, t0+nt)
 *   (mod T) the field is compact: nsite = nt*L^3, local site
 *   ((t - t0) mod T) * L^3 + spatial index.  On the whole lattice nsite = V.
 * Propagators: 12 source columns j = 3*spin + colour, i.e. [12][12][nsite].
 * Gamma matrices: chiral basis gamma_0 = [[0,-1],[-1,0]],
 *   gamma_k = [[0,-i sigma_k],[i sigma_k,0]] (2x2 blocks), gamma_5 = diag(1,1,-1,-1).
 *
 * The operator (Sec. 5 fixes 2 kappa D = 1 - kappa D_hop; the projector form
 * is the standard Wilson one):
 *   D psi(x) = psi(x)/(2 kappa) - 1/2 sum_mu [ (1-gamma_mu) U_mu(x) psi(x+mu)
 *                                            + (1+gamma_mu) U_mu(x-mu)^+ psi(x-mu) ].
 * The Dirichlet slab block D_Lambda = P_Lambda D P_Lambda (Sec. 3, Eq. 10;
 * Sec. 5: Dirichlet conditions on the block operators) drops every hop that
 * leaves the slab.
 *
 * ---------------------------------------------------------------- contract
 * Ownership: every field / link pointer is device memory owned by the caller;
 *   the library never frees or retains it past the call.  The context owns a
 *   lazily grown device workspace, released by dd_destroy.  Host pointers
 *   (stats, correlator output) are owned by the caller.
 * Streams: all work is enqueued on the context's stream.  dd_apply_dirac,
 *   dd_frontier_hop and dd_link_force return without synchronising; the
 *   solvers, the propagators and the correlator synchronise before returning.
 * Errors: a negative dd_status; the message is in dd_last_error(ctx).  No
 *   exception crosses the ABI.  Arguments are validated: null or misaligned
 *   (16 B) pointers, pointers not on the context's device, sizes, slabs
 *   outside [0,T) or, for propagators, slabs that do not partition [0,T).
 * Threads: one context per host thread.
 */
#ifndef DD_H
#define DD_H

#ifdef __cplusplus
extern "C" {
#endif

#define DD_MAX_RHS 12

typedef struct dd_ctx dd_ctx;

typedef enum {
    DD_OK = 0,
    DD_ERR_ARG = -1,         /* invalid argument (pointer, size, slab, parameter) */
    DD_ERR_HIP = -2,         /* a HIP runtime call failed */
    DD_ERR_NOMEM = -3,       /* workspace allocation failed */
    DD_ERR_NOCONV = -4,      /* solver hit max_iter; x holds the last iterate */
    DD_ERR_BREAKDOWN = -5,   /* non-finite values (NaN/Inf) in the iteration, or dependent vectors */
    DD_ERR_UNSUPPORTED = -6  /* valid request this build does not implement */
} dd_status;

typedef enum {
    DD_FP64 = 0,   /* complex128 everywhere */
    DD_FP32 = 1,   /* complex64 (stencil entry points only) */
    DD_MIXED = 2   /* solves: FP32 Krylov recursion, FP64 solution and reliable updates */
} dd_precision;

typedef enum {
    DD_BICGSTAB = 0,  /* BiCGStab on D_Lambda x = b */
    DD_CGNR = 1       /* CG on D^+ D x = D^+ b (converges wherever D is invertible) */
} dd_solver_kind;

typedef enum {
    DD_PRECOND_EO = 0,   /* even-odd: solve the even-site Schur complement m - H_eo H_oe / (4m)
                            where the lattice is bipartite (L even; T even for a whole lattice),
                            otherwise no preconditioning */
    DD_PRECOND_NONE = 1  /* always solve with the full operator */
} dd_precond;

typedef struct {
    int T, L;      /* lattice extent T x L^3, L >= 2, T >= 2 */
    int time_bc;   /* -1 antiperiodic, +1 periodic, 0 Dirichlet walls at t = 0 and T-1 */
} dd_lattice;

typedef struct {
    int t0, nt;    /* time slab [t0, t0+nt) mod T, 1 <= nt < T */
} dd_domain;

/*
 * Krylov solves (both methods, both precisions) run the recursion in the
 * working precision and keep the solution in FP64.  A column takes a reliable
 * update when its recursive residual has dropped by the factor delta since
 * the last one (or the recursion stopped): the correction is folded into the
 * FP64 solution and the recursive residual is replaced by the true FP64
 * residual b - D x.  Convergence is decided on that true residual only.
 */
typedef struct {
    double tol;        /* stop when |b - D x| / |b| <= tol (true residual, FP64) per column */
    int max_iter;      /* cap on Krylov iterations (lockstep over the columns) */
    int prec;          /* DD_FP64 or DD_MIXED */
    int solver;        /* dd_solver_kind */
    double delta;      /* reliable-update threshold in (0, 1); 0: 0.1 (DD_FP64), 0.01 (DD_MIXED) */
    int check_every;   /* iterations between host-side convergence reads (0: 8) */
    int precond;       /* dd_precond (single-lattice solves; batched solves use the full operator) */
    int x0;            /* dd_block_solve only: 0 start from x = 0 (x is output only), 1 x holds an
                          initial guess on entry; every other entry point requires 0 */
} dd_solver_params;

typedef struct {
    int nrhs;                           /* columns solved */
    int iters;                          /* Krylov iterations (lockstep over the columns) */
    int updates;                        /* rounds of reliable updates */
    int restarts;                       /* columns restarted after a breakdown or a stalled recursion */
    double true_rel_resid[DD_MAX_RHS];  /* final |b - D x| / |b| per column, FP64 */
    double ms;                          /* wall time of the call on the host clock */
} dd_solve_stats;

/* Create a context for lattice *lat on HIP stream `stream` (hipStream_t; NULL =
 * the default stream) of the current device.  The workspace grows on demand. */
dd_status dd_create(const dd_lattice* lat, void* stream, dd_ctx** out);
void dd_destroy(dd_ctx* ctx);
/* Last error message of this context ("" if none).  Valid until the next call. */
const char* dd_last_error(const dd_ctx* ctx);

/*
 * out = D in (dom NULL) or D_Lambda in (slab dom), for nrhs columns.
 * Sec. 5 (normalisation 2 kappa D = 1 - kappa D_hop), Sec. 3 Eq. 10 (blocks).
 * prec DD_FP64: U, in, out complex128; DD_FP32: all complex64.  in and out
 * must not overlap.  1 <= nrhs <= 4*DD_MAX_RHS.  Asynchronous.
 */
dd_status dd_apply_dirac(dd_ctx* ctx, const void* U, double kappa, const dd_domain* dom,
                         int nrhs, const void* in, void* out, int prec);

/*
 * out += alpha * P_dst D P_src in: the off-diagonal frontier block between two
 * disjoint slabs (D_dGamma / D_dGamma* of Sec. 3, Eq. 10).  Only time hops
 * across the shared frontier slices contribute; the half-spinor projected
 * message is 6 complex numbers per frontier site (Sec. 3.3).  in lives on
 * src, out on dst (compact layouts).  FP64.  Asynchronous.
 */
dd_status dd_frontier_hop(dd_ctx* ctx, const void* U, const dd_domain* dst, const dd_domain* src,
                          int nrhs, const void* in, void* out, double alpha);

/*
 * x = D_Lambda^-1 b (dom = slab) or D^-1 b (dom NULL), nrhs <= DD_MAX_RHS
 * columns solved together (the "solutions of the Dirac equation" of Sec. 5).
 * U, b, x complex128, b and x distinct.  With params->x0 = 0 x is output only
 * (the solve starts from zero); with x0 = 1 x holds an initial guess on entry
 * (a column whose source is zero gets the zero solution whatever its guess).
 * Returns DD_ERR_NOCONV with x = last iterate if a column misses tol.
 * stats may be NULL.  Synchronises.
 */
dd_status dd_block_solve(dd_ctx* ctx, const void* U, double kappa, const dd_domain* dom, int nrhs,
                         const void* b, void* x, const dd_solver_params* params,
                         dd_solve_stats* stats);

/*
 * Factorised point-to-all propagator from the 12 spin-colour point sources at
 * src = {t, x, y, z} across time slabs doms[0..ndom-1], which partition
 * [0, T) with src in doms[0]:
 *   psi_0 = D_L0^-1 eta                                   (Sec. 3.1, Eq. 13)
 *   psi_k = -D_Lk^-1 sum_{j: d(j) = d(k)-1} D_{Lk,Lj} h_j   (Sec. 3.2, Eq. 14,
 *            chained outward by block distance d on the graph of non-zero
 *            blocks of D)
 *   S_fact = sum_k psi_k.
 * h_j is what crosses the frontier: psi_j for overlap = 0; for overlap =
 * Delta > 0 the solution of slab j's equation (same source) on slab j grown by
 * Delta time slices on both sides (Gamma-bar, the overlap region of Sec. 3.2),
 * restricted to slab j.  Every slab with a slab beyond it must satisfy
 * nt + 2 Delta < T (else DD_ERR_ARG).
 * S_fact (and S_exact = D^-1 eta if not NULL) are complex128 [12][12][V].
 * stats: NULL or ndom + 1 entries (per slab, then the whole-lattice solve; a
 * slab's entry adds the iterations and time of its extended solve, and its
 * residuals are the larger of the two solves').  Synchronises.
 */
dd_status dd_factorized_propagator(dd_ctx* ctx, const void* U, double kappa, const int src[4],
                                   const dd_domain* doms, int ndom, int overlap,
                                   const dd_solver_params* params, void* S_fact, void* S_exact,
                                   dd_solve_stats* stats);

/*
 * Quark-line projection vectors (Sec. 3.3, Eqs. 16-17): an orthonormal basis
 * phi_1..phi_nvec of the field on the time slice t_slice (global time, inside
 * the slab pi) that a frontier hop reads, for the hop leaving the slice forward
 * (sign = +1: towards t_slice + 1, spin projector (1 + gamma_0)/2) or backward
 * (sign = -1: (1 - gamma_0)/2).
 *   V <- v0, orthonormalised; n_iter times V <- orthonormalise(D_pi^-1 V)
 *   (inverse iteration on the slab pi, DD_MAX_RHS columns per solve);
 *   phi = orthonormalise((1 + sign gamma_0)/2 (V on slice t_slice)).
 * Orthonormalisation is Cholesky QR applied twice, in FP64.
 * v0: complex128 [nvec][12][pi->nt L^3] (device, read only); phi: complex128
 * [nvec][12][L^3] (device, output).  1 <= nvec <= min(256, 6 L^3),
 * n_iter >= 0.  Returns DD_ERR_BREAKDOWN if the vectors are linearly dependent
 * in FP64 (e.g. nvec above the rank of the projected slice), DD_ERR_NOCONV if a
 * solve missed tol (phi is still written).  stats (may be NULL): summed
 * iterations and time, nrhs = nvec, true_rel_resid[0] = the largest final
 * residual of all solves.  Synchronises.
 */
dd_status dd_projection_basis(dd_ctx* ctx, const void* U, double kappa, const dd_domain* pi,
                              int t_slice, int sign, int nvec, int n_iter, const void* v0, void* phi,
                              const dd_solver_params* params, dd_solve_stats* stats);

/*
 * dd_factorized_propagator with the quark line cut on nproj time slices
 * (Sec. 3.3, Eqs. 16-17): the field that crosses the frontiers, h_j, has its
 * slice proj_t[i] replaced by P_L h_j = sum_a phi_a (phi_a^+ h_j) over the
 * proj_nvec[i] orthonormal vectors proj_phi[i] (complex128 [nvec][12][L^3],
 * device; e.g. from dd_projection_basis).  S_fact on each slab stays that
 * slab's unprojected solution.  proj_t, proj_nvec and proj_phi are host
 * arrays of nproj entries; slices are distinct, 1 <= proj_nvec[i] <=
 * min(256, 6 L^3).  nproj = 0 is dd_factorized_propagator.  Synchronises.
 */
dd_status dd_factorized_propagator_projected(dd_ctx* ctx, const void* U, double kappa, const int src[4],
                                             const dd_domain* doms, int ndom, int overlap, int nproj,
                                             const int* proj_t, const int* proj_nvec,
                                             const void* const* proj_phi, const dd_solver_params* params,
                                             void* S_fact, void* S_exact, dd_solve_stats* stats);

/*
 * Stochastic traces of the disconnected pseudoscalar contraction (Sec. 4.1,
 * Eqs. 18-19, with the estimator of Sec. 5, Eq. 27):
 *   tau[i][t] = sum_xvec eta_i^+(x) [(kappa D_hop)^n_hop D_Lambda^-1 gamma5 eta_i](x),
 * x_0 = t, for every source i and every slice t of the slabs doms[0..ndom-1]
 * (disjoint; D_Lambda is the Dirichlet block of the slab holding t and
 * kappa D_hop = 1 - 2 kappa D_Lambda), or of the whole lattice with D when
 * doms = NULL and ndom = 0.  For n_hop <= 8 its mean over Gaussian sources is
 * sum_xvec tr{gamma5 D_Lambda^-1(x, x)} (the paper uses n_hop = 8).
 * eta: complex128 [nsrc][12][V] whole-lattice sources (device, read only);
 * tau: complex128 [nsrc][T] (device, output; zero on slices no slab covers).
 * Sources are solved DD_MAX_RHS at a time.  0 <= n_hop <= 16.  stats: NULL or
 * max(ndom, 1) entries, one per domain, summed over its solves
 * (true_rel_resid[j] = the largest over sources j mod DD_MAX_RHS).  Returns
 * DD_ERR_NOCONV if a solve missed tol (tau still written).  Synchronises.
 */
dd_status dd_disconnected_traces(dd_ctx* ctx, const void* U, double kappa, const dd_domain* doms, int ndom,
                                 int nsrc, const void* eta, int n_hop, const dd_solver_params* params,
                                 void* tau, dd_solve_stats* stats);

/*
 * Two-trace product of the disconnected contraction over distinct sources
 * (W_Pd of Eq. 4 summed over xvec and yvec; its factorised term W_Pd^(f) of
 * Eq. 19 when tau comes from slabs holding x_0 and y_0):
 *   C_host[y0][x0] = 1/(nsrc (nsrc - 1) L^3) sum_{i != j} tau[i][x0] tau[j][y0],
 * complex (2 T^2 doubles, host, output).  tau: complex128 [nsrc][T] (device),
 * nsrc >= 2.  Synchronises.
 */
dd_status dd_disconnected_correlator(dd_ctx* ctx, int nsrc, const void* tau, double* C_host);

/*
 * The two factors of the quark lines of the factorised nucleon (Sec. 4.2,
 * Eq. 26), cut by nvec orthonormal vectors phi_i on the time slice t_phi
 * (complex128 [nvec][12][L^3], device; e.g. from dd_projection_basis):
 *   xi_i^T(x) = [phi_i^+ D_gbar^-1](x) on the slice x0 of gbar, returned as
 *     xi (complex128 [nvec][12][L^3]: xi_i(x) = conj([D_gbar^-1+ phi_i](x))),
 *   eta_i(y) = [D_gstar^-1 D_{gstar, dgstar} phi_i](y) on the slab gstar
 *     (complex128 [nvec][12][gstar->nt L^3]),
 * so that D^-1(y, x) ~ -sum_i eta_i(y) xi_i^T(x) (Eq. 17).  t_phi and x0 lie in
 * gbar, t_phi is a time neighbour of gstar outside it (the slice the frontier
 * hop into gstar reads).  1 <= nvec <= min(256, 6 L^3).  stats: NULL or 2
 * entries (the gbar solves with D^+, then the gstar solves).  Returns
 * DD_ERR_NOCONV if a solve missed tol.  Synchronises.
 */
dd_status dd_nucleon_lines(dd_ctx* ctx, const void* U, double kappa, const dd_domain* gbar,
                           const dd_domain* gstar, int t_phi, int nvec, const void* phi, int x0, void* xi,
                           void* eta, const dd_solver_params* params, dd_solve_stats* stats);

/*
 * Colourless spinors of Eq. 25 summed over each time slice of nt slices:
 *   B[t][k][alpha][i][j] = sum_xvec eps^{abc} (s_i^{aT} C gamma5 s_j^b)(x) s_k^c_alpha(x),
 * C = gamma_0 gamma_2 in the library's chiral basis.  s: complex128
 * [nvec][12][nt L^3] (device, read only); B: complex128 [nt][nvec][4][nvec][nvec]
 * (device, output; must not overlap s).  1 <= nvec <= 256.  FP64 (the
 * product over sites runs on the FP64 matrix cores in the library's own GEMM
 * kernel, in chunks of sites whose diquarks stay below 2 GiB; the environment
 * variable DD_BLOCK_CHUNK caps the sites per chunk).  Asynchronous.
 */
dd_status dd_baryon_blocks(dd_ctx* ctx, int nvec, int nt, const void* s, void* B);

/*
 * The factorised nucleon Wick contractions summed over xvec and yvec
 * (Eqs. 22-24), from blocks Bx of the xi lines on ntx source slices and By of
 * the eta lines on nty sink slices (layout of dd_baryon_blocks):
 *   W1[y][x] = -sum_{ijk} Bx[x](j, i, k)^T P_+ By[y](i, j, k),
 *   W2[y][x] = -sum_{ijk} Bx[x](k, i, j)^T P_+ By[y](i, j, k),
 * P_+ = (1 + gamma_0)/2: the text's gamma5 P_- read for this basis and operator
 * (a quark propagating forward in time carries (1 + gamma_0)/2 here, and with
 * gamma5 the forward signal vanishes at leading order in kappa);
 * C_N^(f)(y0, x0) = (W1 - W2) / L^3.  W_host: host,
 * 2 x nty x ntx complex (W1 then W2, 4 nty ntx doubles).  Sums in a fixed order.
 * Synchronises.
 */
dd_status dd_nucleon_contract(dd_ctx* ctx, int nvec, int ntx, const void* Bx, int nty, const void* By,
                              double* W_host);

/*
 * Pion two-point function of a whole-lattice propagator S (complex128
 * [ncol][12][V]) from a source on time slice t_src (Eq. 4, connected W_Pc):
 *   C_host[t] = sum_xvec sum_{c,j} |S_cj((t_src + t) mod T, xvec)|^2, t = 0..T-1,
 * summed in FP64 in a fixed order (bitwise reproducible).  Synchronises.
 */
dd_status dd_pion_correlator(dd_ctx* ctx, const void* S, int ncol, int t_src, double* C_host);

/*
 * dd_pion_correlator for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same kernels and the same result, bitwise, with their partial sums in a
 * static device array of 2^18 doubles (2 MiB, one per GPU, held until the
 * process ends) instead of the context's workspace.  No allocation of any kind.
 * Limit: 36 T ncol + T <= 2^18 (e.g. T = 64 with 48 columns); larger requests
 * return DD_ERR_ARG.  Every call on one GPU shares that array: calls that
 * overlap on one GPU (different contexts, streams or threads) race.
 * Synchronises.
 */
dd_status dd_pion_correlator_noalloc(dd_ctx* ctx, const void* S, int ncol, int t_src, double* C_host);

/*
 * Adjoint of x = D_Lambda^-1 b for a real loss with gradient grad_x
 * (PyTorch convention g = dL/dRe + i dL/dIm): solves D_Lambda^+ lambda = grad_x
 * (one extra solve, through gamma_5-hermiticity) and returns grad_b = lambda
 * and grad_U += the link gradient -Re<lambda, dD x> (layout of U, complex128;
 * links outside the slab or crossing its walls are left untouched).
 * Synchronises.
 */
dd_status dd_block_solve_backward(dd_ctx* ctx, const void* U, double kappa, const dd_domain* dom,
                                  int nrhs, const void* x, const void* grad_x, void* grad_b,
                                  void* grad_U, const dd_solver_params* params,
                                  dd_solve_stats* stats);

/*
 * Pseudofermion action of one slab and what its force needs:
 *   Y = D_Lambda^-+ phi, X = D_Lambda^-1 Y, S = phi^+ (D^+ D)^-1 phi = |Y|^2.
 * phi, X, Y complex128 [nrhs][12][nsite]; *S_host receives the sum over
 * columns.  Synchronises.
 */
dd_status dd_domain_action(dd_ctx* ctx, const void* U, double kappa, const dd_domain* dom, int nrhs,
                           const void* phi, void* X, void* Y, double* S_host,
                           const dd_solver_params* params, dd_solve_stats* stats);

/*
 * Backward of S = phi^+ (D_Lambda^+ D_Lambda)^-1 phi (dd_domain_action) for a
 * loss with dL/dS = g_S, from the X, Y of the forward call; no further solve:
 *   grad_U += g_S * (the link force of dd_link_force with coeff 1),
 *   grad_phi = 2 g_S X  (PyTorch convention dL/dRe phi + i dL/dIm phi; S is
 *   real and dS/d conj(phi) = (D^+ D)^-1 phi = X).
 * X, Y, grad_phi complex128 [nrhs][12][nsite] (grad_phi overwritten), grad_U
 * like U (accumulated).  The fermion force that local updates of a region need
 * (Sec. 5 gives D^+ through gamma_5-hermiticity).  Asynchronous.
 */
dd_status dd_domain_action_backward(dd_ctx* ctx, const dd_domain* dom, int nrhs, const void* X, const void* Y,
                                    double g_S, void* grad_U, void* grad_phi);

/*
 * grad_U += coeff * g with g the link gradient of F(U) = -2 Re<Y, D_Lambda(U) X>
 * at fixed X, Y (PyTorch convention), per link
 *   g_mu(x) = ph sum_spin [ ((1-gamma_mu) Y(x)) X(x+mu)^+ + X(x) ((1+gamma_mu) Y(x+mu))^+ ]
 * (ph = time_bc on the time-edge link).  For S = |Y|^2 of dd_domain_action the
 * force is coeff = 1.  X, Y complex128 [nrhs][12][nsite]; grad_U like U.
 * Asynchronous.
 */
dd_status dd_link_force(dd_ctx* ctx, const dd_domain* dom, int nrhs, const void* X, const void* Y,
                        double coeff, void* grad_U);

/* One independent lattice of a batched solve (time_bc is normally 0: a
 * Dirichlet domain standing on its own). */
typedef struct {
    dd_lattice lat;
    const void* U;   /* complex128 [4][9][V_i] */
    double kappa;
    int nrhs;        /* <= DD_MAX_RHS */
    const void* b;   /* complex128 [nrhs][12][V_i] */
    void* x;         /* complex128 [nrhs][12][V_i], output */
} dd_batch_item;

/*
 * Solve every item of an uneven batch of independent domains (each item is
 * its own lattice with its own links, kappa, time boundary and 1..12
 * columns: many local Dirichlet problems of the decomposition of Sec. 3
 * solved at once).  Every column of every item is
 * advanced together: one launch of the multi-domain stencil and of each
 * vector kernel covers all domains still iterating, the tile shape is tuned
 * on the batch (and cached in the context for the same batch signature), and
 * the inner iterations are captured once into a HIP graph and replayed on a
 * library-owned stream that is ordered after ctx's stream.  Both methods and
 * both precisions of dd_solver_params apply; convergence is per column on the
 * true FP64 residual.  The context's own lattice is not used.
 * items[i].U, .b, .x: device memory of the context's device, complex128,
 * 16-byte aligned; b is not modified.  stats: NULL or n entries (iters: the
 * most iterations of the item's columns; updates, restarts, ms: of the whole
 * batch).  Returns DD_ERR_NOCONV if any column missed tol (all x written).
 * Synchronises.
 */
dd_status dd_block_solve_batched(dd_ctx* ctx, int n, const dd_batch_item* items,
                                 const dd_solver_params* params, dd_solve_stats* stats);

/*
 * Stencil launch shapes are tuned per context on first use; with the
 * environment variable DD_TUNE_CACHE naming a file, contexts load the shapes
 * stored there and append new ones, so that separate processes launch the
 * same kernels.
 *
 * Kernel timing on the context stream.  With enable != 0 every stencil
 * launch made by the library is bracketed by HIP events recorded on the
 * context stream; enabling or disabling resets the counters.  Launches are
 * accumulated per kernel instance, named as a profiler names the template
 * instance, e.g. "k_dslash<float, 1, 4, 128>" (real type, dagger, fused
 * epilogue, work-group size).  For each instance dd_kernel_timing returns the
 * summed milliseconds, the launch count and the summed algorithmic bytes
 *     V * ((48 + e) * ncol * f + 72) * sizeof(real)   per launch,
 * with e = 24 for the epilogues that read one more field and f the share of
 * the launch's columns that are live (inside solves the share the host saw
 * active when it launched; the workgroups of a stopped column return at once;
 * 1 elsewhere).  index runs over
 * [0, count) from dd_kernel_timing_count, in first-launch order; name
 * receives at most name_len - 1 characters and a terminating zero.  Reading
 * the counters waits for the context stream.
 */
dd_status dd_set_kernel_timing(dd_ctx* ctx, int enable);
dd_status dd_kernel_timing_count(dd_ctx* ctx, int* count);
dd_status dd_kernel_timing(dd_ctx* ctx, int index, char* name, int name_len, double* ms, long long* launches,
                           double* bytes);

#ifdef __cplusplus
}
#endif

#endif /* DD_H */
