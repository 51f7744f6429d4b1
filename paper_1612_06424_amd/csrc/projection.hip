// projection.hip -- quark-line projection (Sec. 3.3, Eqs. 16-17).
//
// The factorised propagator crosses a frontier through the field on one time
// slice (the slice the frontier hop reads).  Projecting that field on N_m
// orthonormal vectors phi_i, P_L = sum_i phi_i phi_i^+, cuts the quark line.
// The vectors come from inverse iteration of the Dirac operator of a slab Pi
// around the frontier, V <- orthonormalize(D_Pi^-1 V), restricted to the slice,
// spin-projected with the projector (1 +- gamma_0)/2 that the hop applies, and
// orthonormalised again.
//
// Orthonormalisation is Cholesky QR applied twice: G = V^+ V (N_m x N_m), G =
// R^+ R, V <- V R^-1.  Vectors are [N_m][n] complex128 (n = 12 x sites of the
// field, components outermost as in every field of the library).  The Gram
// matrix is summed from fixed per-workgroup partials in a fixed order, so the
// result is reproducible run to run.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

#include "dd_internal.h"
#include "dd_wilson.h"

namespace dd {

namespace {

constexpr int kGT = 16;       // Gram tile: kGT x kGT outputs per workgroup (256 threads)
constexpr int kGR = 64;       // rows staged in LDS per step
constexpr int kGChunk = 8192; // rows per workgroup (one partial)
constexpr int kCB = 16;       // output columns per workgroup of the combine kernel

__device__ inline cpx<double> cj(cpx<double> a) { return {a.re, -a.im}; }

// Gp[chunk][a][b] = sum over the chunk's rows i of conj(A[a][i]) B[b][i]
// (tile (ta, tb) of kGT x kGT; with sym only the tiles ta <= tb).
__global__ __launch_bounds__(256) void k_xgram_partial(int na, int nb, long long n, const cpx<double>* __restrict__ A,
                                                       const cpx<double>* __restrict__ B, int sym,
                                                       cpx<double>* __restrict__ Gp) {
    const int ta = blockIdx.x, tb = blockIdx.y, chunk = blockIdx.z;
    if (sym && ta > tb) return;  // uniform over the workgroup
    __shared__ cpx<double> sa[kGT][kGR + 1], sb[kGT][kGR + 1];
    const int tid = threadIdx.x;
    const int ia = tid / kGT, ib = tid % kGT;
    const long long r0 = (long long)chunk * kGChunk;
    const long long r1 = std::min(n, r0 + kGChunk);
    cpx<double> acc = {0.0, 0.0};
    for (long long base = r0; base < r1; base += kGR) {
        // stage kGT rows of A and of B, kGR entries each (zeros past the ends)
        for (int e = tid; e < kGT * kGR; e += 256) {
            const int v = e / kGR, r = e % kGR;
            const long long i = base + r;
            const int a = ta * kGT + v, b = tb * kGT + v;
            sa[v][r] = (a < na && i < r1) ? A[(size_t)a * n + i] : cpx<double>{0.0, 0.0};
            sb[v][r] = (b < nb && i < r1) ? B[(size_t)b * n + i] : cpx<double>{0.0, 0.0};
        }
        __syncthreads();
#pragma unroll 8
        for (int r = 0; r < kGR; r++) acc = acc + cj(sa[ia][r]) * sb[ib][r];
        __syncthreads();
    }
    const int a = ta * kGT + ia, b = tb * kGT + ib;
    if (a < na && b < nb) Gp[((size_t)chunk * na + a) * nb + b] = acc;
}

// G[a][b] = sum of the partials in chunk order; with sym the lower triangle is
// the conjugate of the upper one.
__global__ __launch_bounds__(256) void k_xgram_reduce(int na, int nb, int nchunk, int sym,
                                                      const cpx<double>* __restrict__ Gp, cpx<double>* __restrict__ G) {
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= na * nb) return;
    const int a = e / nb, b = e % nb;
    const int ua = sym && a > b ? b : a, ub = sym && a > b ? a : b;
    cpx<double> s = {0.0, 0.0};
    for (int c = 0; c < nchunk; c++) s = s + Gp[((size_t)c * na + ua) * nb + ub];
    G[e] = (sym && a > b) ? cj(s) : s;
}

// R entries written by other threads of the workgroup are read around the
// vector L1 cache (volatile: from L2), after the barrier that orders the writes.
__device__ inline cpx<double> ldv(const cpx<double>* p) {
    const volatile double* q = (const volatile double*)p;
    return {q[0], q[1]};
}

// One workgroup: G = R^+ R (R upper triangular, positive real diagonal), then
// Rinv = R^-1 (upper triangular, zeros below the diagonal).  flag = 1 if a pivot
// is not positive and finite (the vectors are linearly dependent in FP64).
__global__ __launch_bounds__(256) void k_chol_inv(int n, const cpx<double>* __restrict__ G, cpx<double>* R,
                                                  cpx<double>* __restrict__ Rinv, int* __restrict__ flag) {
    const int tid = threadIdx.x;
    __shared__ double piv;
    __shared__ int bad;
    if (tid == 0) bad = 0;
    for (int e = tid; e < n * n; e += 256) R[e] = cpx<double>{0.0, 0.0};
    __syncthreads();
    for (int k = 0; k < n; k++) {
        if (tid == 0) {
            double d = G[(size_t)k * n + k].re;
            for (int j = 0; j < k; j++) {
                const cpx<double> r = ldv(&R[(size_t)j * n + k]);
                d -= r.re * r.re + r.im * r.im;
            }
            if (!(d > 0.0) || !std::isfinite(d)) {
                bad = 1;
                d = 1.0;
            }
            piv = sqrt(d);
            R[(size_t)k * n + k] = cpx<double>{piv, 0.0};
        }
        __syncthreads();
        for (int b = k + 1 + tid; b < n; b += 256) {
            cpx<double> s = G[(size_t)k * n + b];
            for (int j = 0; j < k; j++) s = s - cj(ldv(&R[(size_t)j * n + k])) * ldv(&R[(size_t)j * n + b]);
            R[(size_t)k * n + b] = cpx<double>{s.re / piv, s.im / piv};
        }
        __syncthreads();
    }
    // back substitution, one column of Rinv per thread
    for (int j = tid; j < n; j += 256) {
        for (int i = n - 1; i >= 0; i--) {
            if (i > j) {
                Rinv[(size_t)i * n + j] = cpx<double>{0.0, 0.0};
                continue;
            }
            cpx<double> s = {i == j ? 1.0 : 0.0, 0.0};
            for (int k = i + 1; k <= j; k++) s = s - ldv(&R[(size_t)i * n + k]) * Rinv[(size_t)k * n + j];
            const double d = ldv(&R[(size_t)i * n + i]).re;
            Rinv[(size_t)i * n + j] = cpx<double>{s.re / d, s.im / d};
        }
    }
    __syncthreads();
    if (tid == 0 && bad) flag[0] = 1;
}

// out[b][i] = sum_a A[a][i] M[a][b] for the kCB columns b of this workgroup;
// M (na x nb) staged in LDS.
__global__ __launch_bounds__(256) void k_combine(int na, int nb, long long n, const cpx<double>* __restrict__ A,
                                                 const cpx<double>* __restrict__ M, cpx<double>* __restrict__ out) {
    __shared__ cpx<double> sm[kMaxProjVec][kCB];
    const int b0 = blockIdx.y * kCB;
    for (int e = threadIdx.x; e < na * kCB; e += 256) {
        const int a = e / kCB, j = e % kCB;
        sm[a][j] = (b0 + j < nb) ? M[(size_t)a * nb + b0 + j] : cpx<double>{0.0, 0.0};
    }
    __syncthreads();
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    cpx<double> acc[kCB];
#pragma unroll
    for (int j = 0; j < kCB; j++) acc[j] = cpx<double>{0.0, 0.0};
    for (int a = 0; a < na; a++) {
        const cpx<double> v = A[(size_t)a * n + i];
#pragma unroll
        for (int j = 0; j < kCB; j++) acc[j] = acc[j] + v * sm[a][j];
    }
#pragma unroll
    for (int j = 0; j < kCB; j++)
        if (b0 + j < nb) out[(size_t)(b0 + j) * n + i] = acc[j];
}

// W[a][c][s] = ((1 + SGN gamma_0)/2 V[a] on slice k of the slab)_c(s)
template <int SGN>
__global__ __launch_bounds__(256) void k_slice_project(int nvec, int L3, int nsite, int k,
                                                       const cpx<double>* __restrict__ V, cpx<double>* __restrict__ W) {
    const int s = blockIdx.x * 256 + threadIdx.x;
    const int a = blockIdx.y;
    if (s >= L3 || a >= nvec) return;
    cpx<double> p[12], h[6], o[12];
#pragma unroll
    for (int c = 0; c < 12; c++) {
        p[c] = V[((size_t)a * 12 + c) * nsite + (size_t)k * L3 + s];
        o[c] = cpx<double>{0.0, 0.0};
    }
    project<double, 0, SGN>(p, h);
    accum<double, 0, SGN>(o, h);
#pragma unroll
    for (int c = 0; c < 12; c++) W[((size_t)a * 12 + c) * L3 + s] = cpx<double>{0.5 * o[c].re, 0.5 * o[c].im};
}

int gram_chunks(long long n) { return (int)((n + kGChunk - 1) / kGChunk); }

// G = A^+ B (na x nb); Gp: nchunk x na x nb scratch
void launch_xgram(dd_ctx* c, int na, int nb, long long n, const cpx<double>* A, const cpx<double>* B, bool sym,
                  cpx<double>* Gp, cpx<double>* G) {
    const int nchunk = gram_chunks(n);
    const dim3 grid((unsigned)((na + kGT - 1) / kGT), (unsigned)((nb + kGT - 1) / kGT), (unsigned)nchunk);
    hipLaunchKernelGGL(k_xgram_partial, grid, dim3(256), 0, c->stream, na, nb, n, A, B, sym ? 1 : 0, Gp);
    hipLaunchKernelGGL(k_xgram_reduce, dim3((unsigned)((na * nb + 255) / 256)), dim3(256), 0, c->stream, na, nb,
                       nchunk, sym ? 1 : 0, Gp, G);
}

void launch_combine(dd_ctx* c, int na, int nb, long long n, const cpx<double>* A, const cpx<double>* M,
                    cpx<double>* out) {
    const dim3 grid((unsigned)((n + 255) / 256), (unsigned)((nb + kCB - 1) / kCB));
    hipLaunchKernelGGL(k_combine, grid, dim3(256), 0, c->stream, na, nb, n, A, M, out);
}

struct OrthoWork {
    cpx<double>* Gp;
    cpx<double>* G;
    cpx<double>* R;
    cpx<double>* Rinv;
    int* flag;
};

dd_status ortho_work(dd_ctx* c, int nvec, long long n, OrthoWork* w) {
    dd_status e = DD_OK;
    const size_t nn = (size_t)nvec * nvec;
    w->Gp = (cpx<double>*)workspace(c, W_PROJ_G, (size_t)gram_chunks(n) * nn * sizeof(cpx<double>), &e);
    if (e != DD_OK) return e;
    cpx<double>* m = (cpx<double>*)workspace(c, W_PROJ_R, (3 * nn + 1) * sizeof(cpx<double>), &e);
    if (e != DD_OK) return e;
    w->G = m;
    w->R = m + nn;
    w->Rinv = m + 2 * nn;
    w->flag = (int*)(m + 3 * nn);
    return DD_OK;
}

// out = V R^-1 twice (Cholesky QR 2); V and tmp are overwritten
void orthonormalize(dd_ctx* c, int nvec, long long n, cpx<double>* V, cpx<double>* tmp, const OrthoWork& w) {
    for (int pass = 0; pass < 2; pass++) {
        cpx<double>* src = pass == 0 ? V : tmp;
        cpx<double>* dst = pass == 0 ? tmp : V;
        launch_xgram(c, nvec, nvec, n, src, src, true, w.Gp, w.G);
        hipLaunchKernelGGL(k_chol_inv, dim3(1), dim3(256), 0, c->stream, nvec, w.G, w.R, w.Rinv, w.flag);
        launch_combine(c, nvec, nvec, n, src, w.Rinv, dst);
    }
}

}  // namespace

// Quark-line projection vectors of the frontier hop that leaves slice k of the
// slab g (the region Pi around the frontier) forward (sign = +1) or backward
// (-1): inverse iteration from v0 ([nvec][12][|Pi|]), n_iter solves of 12
// columns at a time, Cholesky QR 2 after each, then restriction to slice k,
// spin projection and Cholesky QR 2 into phi ([nvec][12][L^3]).
dd_status projection_basis(dd_ctx* c, const cpx<double>* U, double kappa, const Geo& g, int k, int sign, int nvec,
                           int n_iter, const cpx<double>* v0, cpx<double>* phi, const dd_solver_params& p,
                           dd_solve_stats* stats) {
    const auto t_start = std::chrono::steady_clock::now();
    dd_status e = DD_OK;
    const int L3 = g.L3, npi = g.nsite;
    const long long n = 12LL * npi, ns = 12LL * L3;
    cpx<double>* V = (cpx<double>*)workspace(c, W_PROJ_V, 2 * (size_t)nvec * n * sizeof(cpx<double>), &e);
    if (e != DD_OK) return e;
    cpx<double>* Vt = V + (size_t)nvec * n;
    OrthoWork w;
    if ((e = ortho_work(c, nvec, n, &w)) != DD_OK) return e;
    DD_HIP(c, hipMemsetAsync(w.flag, 0, sizeof(int), c->stream));
    DD_HIP(c, hipMemcpyAsync(V, v0, (size_t)nvec * n * sizeof(cpx<double>), hipMemcpyDeviceToDevice, c->stream));
    orthonormalize(c, nvec, n, V, Vt, w);
    DD_HIP(c, hipGetLastError());
    int flag = 0;
    DD_HIP(c, hipMemcpyAsync(&flag, w.flag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    DD_HIP(c, hipStreamSynchronize(c->stream));
    if (flag) return fail(c, DD_ERR_BREAKDOWN, "start vectors linearly dependent in FP64");
    dd_solve_stats tot;
    std::memset(&tot, 0, sizeof(tot));
    tot.nrhs = nvec;
    dd_status worst = DD_OK;
    for (int it = 0; it < n_iter; it++) {
        // V <- D_Pi^-1 V, DD_MAX_RHS columns per solve
        for (int a0 = 0; a0 < nvec; a0 += DD_MAX_RHS) {
            const int nc = std::min(DD_MAX_RHS, nvec - a0);
            dd_solve_stats st;
            e = solve(c, U, kappa, g, nc, V + (size_t)a0 * n, Vt + (size_t)a0 * n, p, &st, 0);
            if (e != DD_OK && e != DD_ERR_NOCONV) return e;
            if (e == DD_ERR_NOCONV) worst = e;
            tot.iters += st.iters;
            tot.updates += st.updates;
            tot.restarts += st.restarts;
            for (int j = 0; j < nc; j++) tot.true_rel_resid[0] = std::max(tot.true_rel_resid[0], st.true_rel_resid[j]);
        }
        std::swap(V, Vt);
        orthonormalize(c, nvec, n, V, Vt, w);
        DD_HIP(c, hipGetLastError());
    }
    const dim3 sg((unsigned)((L3 + 255) / 256), (unsigned)nvec);
    if (sign > 0)
        hipLaunchKernelGGL(k_slice_project<1>, sg, dim3(256), 0, c->stream, nvec, L3, npi, k, V, phi);
    else
        hipLaunchKernelGGL(k_slice_project<-1>, sg, dim3(256), 0, c->stream, nvec, L3, npi, k, V, phi);
    orthonormalize(c, nvec, ns, phi, Vt, w);
    DD_HIP(c, hipGetLastError());
    DD_HIP(c, hipMemcpyAsync(&flag, w.flag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    DD_HIP(c, hipStreamSynchronize(c->stream));
    tot.ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    if (stats) *stats = tot;
    if (flag) return fail(c, DD_ERR_BREAKDOWN, "projection vectors linearly dependent in FP64");
    if (worst != DD_OK) return fail(c, worst, "an inverse-iteration solve did not converge: " + c->err);
    return DD_OK;
}

// field (ncol columns of a slab of nt slices, [ncol][12][nt L3]): slice k replaced by
// P_L of it, P_L = sum_i phi_i phi_i^+ with phi [nvec][12][L3] orthonormal
dd_status project_slice(dd_ctx* c, int L3, int nt, int k, int ncol, cpx<double>* field, int nvec,
                        const cpx<double>* phi) {
    dd_status e = DD_OK;
    const long long ns = 12LL * L3;
    cpx<double>* buf = (cpx<double>*)workspace(c, W_PROJ_V, 2 * (size_t)ncol * ns * sizeof(cpx<double>), &e);
    if (e != DD_OK) return e;
    cpx<double>* out = buf + (size_t)ncol * ns;
    OrthoWork w;
    if ((e = ortho_work(c, std::max(nvec, ncol), ns, &w)) != DD_OK) return e;
    launch_slab_embed(c, L3, nt, k, 1, ncol, buf, field, 1);        // the slice, [ncol][12][L3]
    launch_xgram(c, nvec, ncol, ns, phi, buf, false, w.Gp, w.G);    // C = phi^+ field (nvec x ncol)
    launch_combine(c, nvec, ncol, ns, phi, w.G, out);                // phi C
    launch_slab_embed(c, L3, nt, k, 1, ncol, out, field, 0);
    DD_HIP(c, hipGetLastError());
    return DD_OK;
}

}  // namespace dd
