/*
 * dd_oracle.c -- plain FP64 CPU oracle for the Wilson-Dirac hot path of the
 * factorised (domain-decomposed) quark propagator of
 *   M. Ce, L. Giusti, S. Schaefer, "Domain decomposition and multilevel
 *   integration for fermions", PoS LATTICE2016, arXiv:1612.06424.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark load this library.  It shares no code,
 * header, table or helper with the HIP library; the product path never calls
 * it.  It is deliberately slow and literal:
 *   - fields use the natural site-major layout psi[site][spin][colour]
 *     (the HIP library uses a structure-of-arrays layout instead);
 *   - (1 -/+ gamma_mu) are applied as full 4x4 matrices, no half-spinor tricks;
 *   - the block operator P_dst D P_src is evaluated exactly as its definition:
 *     every hop whose end point lies outside the source block is dropped.
 *
 * Conventions (the paper fixes only the normalisation of D):
 *   site  s = ((t*L + z)*L + y)*L + x, time slowest; mu = 0 is time, 1..3 = x,y,z
 *   spinor component c = 3*spin + colour
 *   link  U[site][mu][row][col]
 *   D psi(x) = psi(x)/(2 kappa)
 *            - 1/2 sum_mu [ (1 - gamma_mu) U_mu(x) psi(x+mu)
 *                         + (1 + gamma_mu) U_mu(x-mu)^dagger psi(x-mu) ]
 *   which is 2 kappa D = 1 - kappa D_hop (Sec. 5, the definition given with
 *   the stochastic estimator, Eq. 27).  Space is periodic; the hop across the
 *   time edge T-1 <-> 0 carries the factor bc (-1 antiperiodic, +1 periodic,
 *   0 = dropped, i.e. Dirichlet walls at t = 0 and t = T-1).
 *   Chiral gamma basis: gamma_0 = [[0,-1],[-1,0]], gamma_k = [[0,-i s_k],[i s_k,0]]
 *   (2x2 blocks), so gamma_5 = gamma_0 gamma_1 gamma_2 gamma_3 = diag(1,1,-1,-1).
 *
 * A time slab (domain) is [t0, t0+nt) modulo T.  Fields on a slab are stored
 * compactly with local site index ((t - t0) mod T) * L^3 + spatial index.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

static cplx GAMMA[4][4][4]; /* gamma_mu, mu = 0..3 */
static cplx GAMMA5[4][4];
static int gamma_ready = 0;

/* Fill the chiral-basis gamma matrices from the 2x2 Pauli blocks. */
static void init_gamma(void)
{
    if (gamma_ready) return;
    const cplx sig[3][2][2] = {
        {{0, 1}, {1, 0}},
        {{0, -I}, {I, 0}},
        {{1, 0}, {0, -1}},
    };
    memset(GAMMA, 0, sizeof(GAMMA));
    for (int a = 0; a < 2; a++) {
        GAMMA[0][a][2 + a] = -1;
        GAMMA[0][2 + a][a] = -1;
    }
    for (int k = 0; k < 3; k++)
        for (int a = 0; a < 2; a++)
            for (int b = 0; b < 2; b++) {
                GAMMA[k + 1][a][2 + b] = -I * sig[k][a][b];
                GAMMA[k + 1][2 + a][b] = I * sig[k][a][b];
            }
    /* gamma_5 = gamma_0 gamma_1 gamma_2 gamma_3 computed, not typed in */
    cplx tmp[4][4], acc[4][4];
    memcpy(acc, GAMMA[0], sizeof(acc));
    for (int mu = 1; mu < 4; mu++) {
        for (int i = 0; i < 4; i++)
            for (int j = 0; j < 4; j++) {
                cplx s = 0;
                for (int k = 0; k < 4; k++) s += acc[i][k] * GAMMA[mu][k][j];
                tmp[i][j] = s;
            }
        memcpy(acc, tmp, sizeof(acc));
    }
    memcpy(GAMMA5, acc, sizeof(acc));
    gamma_ready = 1;
}

/* Exported for the tests of the Clifford algebra: g[mu][4][4], mu=0..3, 4 = gamma_5. */
/* Number of host threads the parallel loops below use. */
int ora_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void ora_gamma(cplx *g)
{
    init_gamma();
    memcpy(g, GAMMA, sizeof(GAMMA));
    memcpy(g + 64, GAMMA5, sizeof(GAMMA5));
}

static int mod(int a, int n) { return ((a % n) + n) % n; }

/* offset of time slice t inside the slab [t0, t0+nt), or -1 if outside */
static int slab_pos(int t, int t0, int nt, int T)
{
    int d = mod(t - t0, T);
    return d < nt ? d : -1;
}

/*
 * out = P_dst D P_src in, for slabs dst = [dt0, dt0+dnt), src = [st0, st0+snt).
 * With dst = src this is the Dirichlet block D_Lambda (Sec. 3, Eq. 10; Sec. 5,
 * Dirichlet conditions on the block operators); with disjoint slabs it is an
 * off-diagonal frontier block (D_dGamma, D_dGamma* of Eq. 10); with
 * dst = src = [0,T) it is D itself.
 * in: [snt*L^3][12], out: [dnt*L^3][12] (overwritten).
 */
void ora_block_apply(int T, int L, int bc, const cplx *U, double kappa,
                     int dt0, int dnt, int st0, int snt,
                     const cplx *in, cplx *out)
{
    init_gamma();
    const long L3 = (long)L * L * L;
    const long nsite = (long)dnt * L3;
    const double mass = 1.0 / (2.0 * kappa);

#pragma omp parallel for schedule(static)
    for (long i = 0; i < nsite; i++) {
        const int t = mod(dt0 + (int)(i / L3), T);
        const long sp = i % L3;
        const int c[4] = {t, (int)(sp % L), (int)((sp / L) % L), (int)(sp / ((long)L * L))};
        const int n[4] = {T, L, L, L};
        const long s = (long)t * L3 + sp;
        cplx res[4][3];
        memset(res, 0, sizeof(res));

        /* mass term, only if the site itself belongs to the source block */
        int pos = slab_pos(t, st0, snt, T);
        if (pos >= 0) {
            const cplx *p = in + ((long)pos * L3 + sp) * 12;
            for (int a = 0; a < 4; a++)
                for (int b = 0; b < 3; b++) res[a][b] += mass * p[3 * a + b];
        }

        for (int mu = 0; mu < 4; mu++) {
            for (int dir = +1; dir >= -1; dir -= 2) {
                int cn[4] = {c[0], c[1], c[2], c[3]};
                cn[mu] = mod(c[mu] + dir, n[mu]);
                double ph = 1.0;
                if (mu == 0 && ((dir > 0 && t == T - 1) || (dir < 0 && t == 0))) ph = (double)bc;
                if (ph == 0.0) continue;
                int npos = slab_pos(cn[0], st0, snt, T);
                if (npos < 0) continue; /* hop leaves the source block: dropped */
                const long nsp = ((long)cn[3] * L + cn[2]) * L + cn[1];
                const cplx *q = in + ((long)npos * L3 + nsp) * 12;
                /* colour matrix: U_mu(x) forward, U_mu(x-mu)^dagger backward */
                cplx W[3][3];
                if (dir > 0) {
                    const cplx *u = U + (s * 4 + mu) * 9;
                    for (int a = 0; a < 3; a++)
                        for (int b = 0; b < 3; b++) W[a][b] = u[3 * a + b];
                } else {
                    const long sn = (long)cn[0] * L3 + nsp;
                    const cplx *u = U + (sn * 4 + mu) * 9;
                    for (int a = 0; a < 3; a++)
                        for (int b = 0; b < 3; b++) W[a][b] = conj(u[3 * b + a]);
                }
                /* h = W q (colour), then res -= 1/2 ph (1 -/+ gamma_mu) h (spin) */
                cplx h[4][3];
                for (int sp4 = 0; sp4 < 4; sp4++)
                    for (int a = 0; a < 3; a++) {
                        cplx acc = 0;
                        for (int b = 0; b < 3; b++) acc += W[a][b] * q[3 * sp4 + b];
                        h[sp4][a] = acc;
                    }
                const double sg = (dir > 0) ? -1.0 : 1.0; /* 1 - gamma fwd, 1 + gamma bwd */
                for (int a = 0; a < 4; a++)
                    for (int col = 0; col < 3; col++) {
                        cplx proj = h[a][col];
                        for (int b = 0; b < 4; b++) proj += sg * GAMMA[mu][a][b] * h[b][col];
                        res[a][col] -= 0.5 * ph * proj;
                    }
            }
        }
        cplx *o = out + i * 12;
        for (int a = 0; a < 4; a++)
            for (int b = 0; b < 3; b++) o[3 * a + b] = res[a][b];
    }
}

/* out = gamma_5 in, site by site (n sites); in and out may alias. */
void ora_gamma5(long n, const cplx *in, cplx *out)
{
    init_gamma();
#pragma omp parallel for schedule(static)
    for (long i = 0; i < n; i++) {
        cplx res[12];
        for (int a = 0; a < 4; a++)
            for (int b = 0; b < 3; b++) {
                cplx acc = 0;
                for (int k = 0; k < 4; k++) acc += GAMMA5[a][k] * in[i * 12 + 3 * k + b];
                res[3 * a + b] = acc;
            }
        memcpy(out + i * 12, res, sizeof(res));
    }
}

/* ---------------------------------------------------------------- BLAS-1 */

static cplx dot(long n, const cplx *a, const cplx *b) /* sum conj(a) b */
{
    double re = 0, im = 0;
#pragma omp parallel for reduction(+ : re, im) schedule(static)
    for (long i = 0; i < n; i++) {
        cplx p = conj(a[i]) * b[i];
        re += creal(p);
        im += cimag(p);
    }
    return re + I * im;
}

static double norm2(long n, const cplx *a) { return creal(dot(n, a, a)); }

/* ---------------------------------------------------------------- solvers */

typedef struct {
    int T, L, bc, t0, nt;
    const cplx *U;
    double kappa;
} op_t;

static void op_apply(const op_t *A, const cplx *in, cplx *out)
{
    ora_block_apply(A->T, A->L, A->bc, A->U, A->kappa, A->t0, A->nt, A->t0, A->nt, in, out);
}

/* A^dagger = gamma_5 A gamma_5 for the Wilson operator and its slab blocks */
static void op_apply_dag(const op_t *A, const cplx *in, cplx *out, cplx *tmp, long n)
{
    ora_gamma5(n / 12, in, tmp);
    op_apply(A, tmp, out);
    ora_gamma5(n / 12, out, out);
}

static double true_relres(const op_t *A, const cplx *b, const cplx *x, cplx *tmp, long n, double bnorm)
{
    op_apply(A, x, tmp);
    double r2 = 0;
    for (long i = 0; i < n; i++) {
        cplx d = b[i] - tmp[i];
        r2 += creal(d) * creal(d) + cimag(d) * cimag(d);
    }
    return sqrt(r2) / bnorm;
}

/*
 * BiCGStab (van der Vorst 1992) for A x = b, A = the Dirichlet slab block.
 * x0 = 0, shadow residual r^ = r0 = b.  Stops when the recursive residual is
 * below tol*|b| and the true residual |b - A x|/|b| confirms it; otherwise
 * restarts from the true residual.  A breakdown (rho or <r^,v> vanishing, or
 * omega = 0) restarts with r^ = r.  Returns 0 converged, 1 not converged,
 * 2 non-finite values.
 */
static int bicgstab(const op_t *A, const cplx *b, cplx *x, double tol, int maxit,
                    int *iters, double *relres)
{
    const long n = (long)A->nt * A->L * A->L * A->L * 12;
    cplx *r = malloc(n * sizeof(cplx)), *rh = malloc(n * sizeof(cplx));
    cplx *p = malloc(n * sizeof(cplx)), *v = malloc(n * sizeof(cplx));
    cplx *s = malloc(n * sizeof(cplx)), *t = malloc(n * sizeof(cplx));
    const double bnorm = sqrt(norm2(n, b));
    int status = 1, it = 0;
    memset(x, 0, n * sizeof(cplx));
    if (bnorm == 0.0) {
        *iters = 0;
        *relres = 0.0;
        status = 0;
        goto done;
    }
    if (!isfinite(bnorm)) {
        status = 2;
        goto done;
    }
    int restart = 1;
    double rhn2 = 0;
    cplx rho = 1, alpha = 1, omega = 1;
    while (it < maxit) {
        if (restart) {
            op_apply(A, x, t);
            for (long i = 0; i < n; i++) r[i] = b[i] - t[i];
            memcpy(rh, r, n * sizeof(cplx));
            rhn2 = norm2(n, rh);
            memset(p, 0, n * sizeof(cplx));
            memset(v, 0, n * sizeof(cplx));
            rho = alpha = omega = 1;
            restart = 0;
        }
        cplx rho_new = dot(n, rh, r);
        if (cabs(rho_new) < 1e-30 * sqrt(norm2(n, r) * rhn2)) {
            memcpy(rh, r, n * sizeof(cplx)); /* breakdown: new shadow residual */
            rhn2 = norm2(n, rh);
            rho_new = dot(n, rh, r);
            memset(p, 0, n * sizeof(cplx));
            memset(v, 0, n * sizeof(cplx));
            rho = alpha = omega = 1;
        }
        cplx beta = (rho_new / rho) * (alpha / omega);
        for (long i = 0; i < n; i++) p[i] = r[i] + beta * (p[i] - omega * v[i]);
        op_apply(A, p, v);
        cplx rv = dot(n, rh, v);
        if (cabs(rv) < 1e-30 * sqrt(norm2(n, v) * rhn2)) {
            restart = 1;
            it++;
            continue;
        }
        alpha = rho_new / rv;
        for (long i = 0; i < n; i++) s[i] = r[i] - alpha * v[i];
        op_apply(A, s, t);
        double tt = norm2(n, t);
        omega = (tt > 0) ? dot(n, t, s) / tt : 0;
        for (long i = 0; i < n; i++) {
            x[i] += alpha * p[i] + omega * s[i];
            r[i] = s[i] - omega * t[i];
        }
        rho = rho_new;
        it++;
        double rr = sqrt(norm2(n, r));
        if (!isfinite(rr)) {
            status = 2;
            break;
        }
        if (omega == 0) restart = 1;
        if (rr <= tol * bnorm) {
            double tr = true_relres(A, b, x, t, n, bnorm);
            if (tr <= tol) {
                status = 0;
                break;
            }
            restart = 1;
        }
    }
    *iters = it;
    *relres = true_relres(A, b, x, t, n, bnorm);
done:
    free(r); free(rh); free(p); free(v); free(s); free(t);
    return status;
}

/*
 * CGNR: conjugate gradients on A^dagger A x = A^dagger b.  Always convergent
 * for invertible A; used where BiCGStab stagnates.  Same stopping rule on the
 * true residual of A x = b.
 */
static int cgnr(const op_t *A, const cplx *b, cplx *x, double tol, int maxit, int *iters, double *relres)
{
    const long n = (long)A->nt * A->L * A->L * A->L * 12;
    cplx *r = malloc(n * sizeof(cplx)), *z = malloc(n * sizeof(cplx));
    cplx *p = malloc(n * sizeof(cplx)), *w = malloc(n * sizeof(cplx));
    cplx *tmp = malloc(n * sizeof(cplx));
    const double bnorm = sqrt(norm2(n, b));
    int status = 1, it = 0;
    memset(x, 0, n * sizeof(cplx));
    if (bnorm == 0.0) {
        *iters = 0;
        *relres = 0;
        status = 0;
        goto done;
    }
    memcpy(r, b, n * sizeof(cplx));           /* r = b - A x */
    op_apply_dag(A, r, z, tmp, n);            /* z = A^dag r */
    memcpy(p, z, n * sizeof(cplx));
    double zz = norm2(n, z);
    while (it < maxit) {
        op_apply(A, p, w);
        double ww = norm2(n, w);
        if (ww == 0) break;
        double al = zz / ww;
        for (long i = 0; i < n; i++) {
            x[i] += al * p[i];
            r[i] -= al * w[i];
        }
        it++;
        double rr = sqrt(norm2(n, r));
        if (!isfinite(rr)) {
            status = 2;
            break;
        }
        if (rr <= tol * bnorm) {
            double tr = true_relres(A, b, x, tmp, n, bnorm);
            if (tr <= tol) {
                status = 0;
                break;
            }
            op_apply(A, x, tmp);
            for (long i = 0; i < n; i++) r[i] = b[i] - tmp[i];
        }
        op_apply_dag(A, r, z, tmp, n);
        double zz_new = norm2(n, z);
        double be = zz_new / zz;
        zz = zz_new;
        for (long i = 0; i < n; i++) p[i] = z[i] + be * p[i];
    }
    *iters = it;
    *relres = true_relres(A, b, x, tmp, n, bnorm);
done:
    free(r); free(z); free(p); free(w); free(tmp);
    return status;
}

/*
 * Solve the slab block D_Lambda x = b for ncol columns (each [nt*L^3][12],
 * columns contiguous).  method 0 = BiCGStab, 1 = CGNR.  iters/relres per column.
 * Returns the worst column status.
 */
int ora_solve(int T, int L, int bc, const cplx *U, double kappa, int t0, int nt,
              int ncol, const cplx *b, cplx *x, double tol, int maxit, int method,
              int *iters, double *relres)
{
    init_gamma();
    op_t A = {T, L, bc, t0, nt, U, kappa};
    const long n = (long)nt * L * L * L * 12;
    int worst = 0;
    for (int j = 0; j < ncol; j++) {
        int st = method == 1 ? cgnr(&A, b + j * n, x + j * n, tol, maxit, &iters[j], &relres[j])
                             : bicgstab(&A, b + j * n, x + j * n, tol, maxit, &iters[j], &relres[j]);
        if (st > worst) worst = st;
    }
    return worst;
}

/*
 * Pion two-point function from a point-to-all propagator (Eq. 4, W_Pc):
 * C(t) = sum_xvec sum_{c,j} |S_cj(x)|^2 at x0 = (t_src + t) mod T, i.e.
 * tr{ S(x,x_s) S(x,x_s)^dagger } summed over the sink time slice.
 * S: ncol columns, each a whole-lattice field [V][12].
 */
void ora_pion(int T, int L, int ncol, const cplx *S, int t_src, double *C)
{
    const long L3 = (long)L * L * L, V = (long)T * L3;
    for (int t = 0; t < T; t++) {
        const int ts = mod(t_src + t, T);
        double acc = 0;
#pragma omp parallel for reduction(+ : acc) schedule(static)
        for (long sp = 0; sp < L3; sp++)
            for (int j = 0; j < ncol; j++)
                for (int c = 0; c < 12; c++) {
                    cplx z = S[(long)j * V * 12 + ((long)ts * L3 + sp) * 12 + c];
                    acc += creal(z) * creal(z) + cimag(z) * cimag(z);
                }
        C[t] = acc;
    }
}

/*
 * Link gradient of F(U) = -2 Re<Y, D_Lambda(U) X> at fixed X, Y, as one colour
 * matrix per link in the PyTorch convention for a real function of complex
 * variables, g = dF/dRe U + i dF/dIm U.  grad += coeff * g.
 * Only links inside the slab whose hop stays inside the slab enter D_Lambda;
 * every other link gets exactly zero.  Derivation: U_mu(x) appears in
 * (D psi)(x) as -1/2 ph (1-gamma_mu) U_mu(x) psi(x+mu) and in (D psi)(x+mu) as
 * -1/2 ph (1+gamma_mu) U_mu(x)^dagger psi(x), so
 *   -2 Re<Y, dD X> = ph Re tr[ dU ( sum_s X_s(x+mu) a_s^dagger + b_s X_s(x)^dagger ) ]
 with a = (1-gamma_mu) Y(x), b = (1+gamma_mu) Y(x+mu), hence
 *   g = ph sum_s [ a_s X_s(x+mu)^dagger + X_s(x) b_s^dagger ].
 * grad uses the natural link layout [V][4][9].
 * X, Y: compact slab fields [nt*L^3][12], ncol columns each.
 */
void ora_link_grad(int T, int L, int bc, int t0, int nt, int ncol,
                   const cplx *X, const cplx *Y, double coeff, cplx *grad)
{
    init_gamma();
    const long L3 = (long)L * L * L;
    const long nsite = (long)nt * L3;
#pragma omp parallel for schedule(static)
    for (long i = 0; i < nsite; i++) {
        const int t = mod(t0 + (int)(i / L3), T);
        const long sp = i % L3;
        const int c[4] = {t, (int)(sp % L), (int)((sp / L) % L), (int)(sp / ((long)L * L))};
        const int n[4] = {T, L, L, L};
        const long s = (long)t * L3 + sp;
        for (int mu = 0; mu < 4; mu++) {
            int cn[4] = {c[0], c[1], c[2], c[3]};
            cn[mu] = mod(c[mu] + 1, n[mu]);
            double ph = 1.0;
            if (mu == 0 && t == T - 1) ph = (double)bc;
            if (ph == 0.0) continue;
            int npos = slab_pos(cn[0], t0, nt, T);
            if (npos < 0) continue;
            const long j_loc = (long)npos * L3 + ((long)cn[3] * L + cn[2]) * L + cn[1];
            cplx g[3][3];
            memset(g, 0, sizeof(g));
            for (int col = 0; col < ncol; col++) {
                const cplx *Xx = X + (long)col * nsite * 12 + i * 12;
                const cplx *Xn = X + (long)col * nsite * 12 + j_loc * 12;
                const cplx *Yx = Y + (long)col * nsite * 12 + i * 12;
                const cplx *Yn = Y + (long)col * nsite * 12 + j_loc * 12;
                cplx a[4][3], b[4][3];
                for (int s4 = 0; s4 < 4; s4++)
                    for (int k = 0; k < 3; k++) {
                        cplx pa = Yx[3 * s4 + k], pb = Yn[3 * s4 + k];
                        for (int q = 0; q < 4; q++) {
                            pa -= GAMMA[mu][s4][q] * Yx[3 * q + k];
                            pb += GAMMA[mu][s4][q] * Yn[3 * q + k];
                        }
                        a[s4][k] = pa;
                        b[s4][k] = pb;
                    }
                for (int s4 = 0; s4 < 4; s4++)
                    for (int r = 0; r < 3; r++)
                        for (int k = 0; k < 3; k++)
                            g[r][k] += a[s4][r] * conj(Xn[3 * s4 + k]) + Xx[3 * s4 + r] * conj(b[s4][k]);
            }
            cplx *gout = grad + (s * 4 + mu) * 9;
            for (int r = 0; r < 3; r++)
                for (int k = 0; k < 3; k++) gout[3 * r + k] += coeff * ph * g[r][k];
        }
    }
}
