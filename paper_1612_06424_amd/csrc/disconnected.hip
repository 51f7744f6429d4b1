// disconnected.hip -- the disconnected contraction of the isospin-singlet
// pseudoscalar (Sec. 4.1, Eqs. 18-19) with the stochastic estimator of Sec. 5
// (Eq. 27):
//   tau_i(t) = sum_xvec eta_i^+(x) [(kappa D_hop)^n D_Lambda^-1 gamma5 eta_i](x),  x_0 = t,
// per volume source eta_i and time slice, with D_Lambda the Dirichlet block of
// the domain holding t (or D on the whole lattice).  2 kappa D = 1 - kappa D_hop
// gives D^-1 = 2 kappa sum_{k<n} (kappa D_hop)^k + (kappa D_hop)^n D^-1, and the
// gamma5 trace of (kappa D_hop)^k vanishes on every site for k < 8, so for
// n <= 8 the estimator is unbiased for sum_xvec tr{gamma5 D_Lambda^-1(x, x)}
// while the powers of the hop cut its noise.
//
// Per domain and per group of up to 12 sources: gather eta onto the domain and
// apply gamma5 (one kernel), solve, apply kappa D_hop n times (the stencil with
// the hop-only epilogue), then contract slice by slice.  The contraction reads
// gamma5 eta, the right-hand side the solve needed anyway, and puts the sign
// of gamma5 back (gamma5 is diag(1, 1, -1, -1) in spin: components 6..11 flip).
#include <algorithm>
#include <chrono>
#include <cstring>

#include "dd_internal.h"

namespace dd {

namespace {

constexpr int kTB = 256;

// (re, im) summed over the workgroup in a fixed order; valid in thread 0
__device__ inline void block_sum2(double& re, double& im) {
    __shared__ double sh[kTB / kWave][2];
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
        re += __shfl_xor(re, off, kWave);
        im += __shfl_xor(im, off, kWave);
    }
    const int w = threadIdx.x / kWave, l = threadIdx.x % kWave;
    if (l == 0) {
        sh[w][0] = re;
        sh[w][1] = im;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        re = 0;
        im = 0;
        for (int k = 0; k < kTB / kWave; k++) {
            re += sh[k][0];
            im += sh[k][1];
        }
    }
}

// part[col][c][s] = gamma5 whole[col][c][site of slice (t0 + s / L3) mod T]
// (the slab [t0, t0 + nt) of a whole-lattice field, gamma5 applied)
__global__ __launch_bounds__(kTB) void k_gather_g5(int T, int L3, int t0, int nt, const cpx<double>* __restrict__ whole,
                                                   cpx<double>* __restrict__ part) {
    const int n = nt * L3;
    const int s = blockIdx.x * kTB + threadIdx.x;
    const int cc = blockIdx.y;  // col * 12 + component
    if (s >= n) return;
    const int c = cc % 12;
    const int tl = s / L3, sp = s - tl * L3;
    const int t = (t0 + tl) % T;
    const cpx<double> v = whole[(size_t)cc * T * L3 + (size_t)t * L3 + sp];
    part[(size_t)cc * n + s] = c < 6 ? v : cpx<double>{-v.re, -v.im};
}

// tau[(col0 + col) T + (t0 + k) mod T] = sum over slice k and the 12 components of
// conj(gamma5 g5e) y, one workgroup per (slice, column)
__global__ __launch_bounds__(kTB) void k_trace_slices(int T, int L3, int t0, int nt, int col0,
                                                      const cpx<double>* __restrict__ g5e,
                                                      const cpx<double>* __restrict__ y,
                                                      cpx<double>* __restrict__ tau) {
    const int k = blockIdx.x, col = blockIdx.y;
    const size_t nsite = (size_t)nt * L3;
    const size_t base = (size_t)col * 12 * nsite + (size_t)k * L3;
    double re = 0, im = 0;
    for (int c = 0; c < 12; c++) {
        const double sg = c < 6 ? 1.0 : -1.0;
        const cpx<double>* e = g5e + base + (size_t)c * nsite;
        const cpx<double>* v = y + base + (size_t)c * nsite;
        double cr = 0, ci = 0;
        for (int s = threadIdx.x; s < L3; s += kTB) {
            const cpx<double> a = e[s], b = v[s];
            cr += a.re * b.re + a.im * b.im;
            ci += a.re * b.im - a.im * b.re;
        }
        re += sg * cr;
        im += sg * ci;
    }
    block_sum2(re, im);
    if (threadIdx.x == 0) tau[(size_t)(col0 + col) * T + (t0 + k) % T] = cpx<double>{re, im};
}

// C[y0][x0] = 1/(n (n - 1) L^3) sum_i tau_i(x0) (S(y0) - tau_i(y0)), S = sum_i tau_i:
// the product over distinct sources i != j
__global__ __launch_bounds__(kTB) void k_disc_corr(int T, int n, double scale, const cpx<double>* __restrict__ tau,
                                                   cpx<double>* __restrict__ C) {
    const int e = blockIdx.x * kTB + threadIdx.x;
    if (e >= T * T) return;
    const int y0 = e / T, x0 = e % T;
    cpx<double> S = {0.0, 0.0};
    for (int i = 0; i < n; i++) S = S + tau[(size_t)i * T + y0];
    cpx<double> acc = {0.0, 0.0};
    for (int i = 0; i < n; i++) acc = acc + tau[(size_t)i * T + x0] * (S - tau[(size_t)i * T + y0]);
    C[e] = cpx<double>{acc.re * scale, acc.im * scale};
}

}  // namespace

dd_status disconnected_traces(dd_ctx* c, const cpx<double>* U, double kappa, const dd_domain* doms, int ndom,
                              int nsrc, const cpx<double>* eta, int n_hop, const dd_solver_params& p,
                              cpx<double>* tau, dd_solve_stats* stats) {
    const dd_lattice& lat = c->lat;
    const int T = lat.T, L3 = lat.L * lat.L * lat.L;
    const size_t V = (size_t)T * L3;
    const int nd = doms ? ndom : 1;
    size_t maxsite = 0;
    for (int d = 0; d < nd; d++) maxsite = std::max(maxsite, (size_t)(doms ? doms[d].nt : T) * L3);
    const size_t fb = (size_t)DD_MAX_RHS * 12 * maxsite * sizeof(cpx<double>);
    dd_status e = DD_OK;
    cpx<double>* rhs = (cpx<double>*)workspace(c, W_DISC0, fb, &e);
    if (e != DD_OK) return e;
    cpx<double>* x = (cpx<double>*)workspace(c, W_DISC1, fb, &e);
    if (e != DD_OK) return e;
    cpx<double>* y = (cpx<double>*)workspace(c, W_DISC2, fb, &e);
    if (e != DD_OK) return e;
    launch_zero<double>(c, (size_t)nsrc * T, tau);
    dd_status worst = DD_OK;
    for (int d = 0; d < nd; d++) {
        const Geo g = make_geo(lat, doms ? &doms[d] : nullptr);
        const int t0 = g.t0, nt = g.nt, nsite = g.nsite;
        dd_solve_stats tot;
        std::memset(&tot, 0, sizeof(tot));
        tot.nrhs = nsrc;
        for (int a0 = 0; a0 < nsrc; a0 += DD_MAX_RHS) {
            const int nc = std::min(DD_MAX_RHS, nsrc - a0);
            hipLaunchKernelGGL(k_gather_g5, dim3((unsigned)((nsite + kTB - 1) / kTB), (unsigned)(12 * nc)), dim3(kTB),
                               0, c->stream, T, L3, t0, nt, eta + (size_t)a0 * 12 * V, rhs);
            DD_HIP(c, hipGetLastError());
            dd_solve_stats st;
            e = solve(c, U, kappa, g, nc, rhs, x, p, &st, 0);
            if (e != DD_OK && e != DD_ERR_NOCONV) return e;
            if (e == DD_ERR_NOCONV) worst = e;
            tot.iters += st.iters;
            tot.updates += st.updates;
            tot.restarts += st.restarts;
            tot.ms += st.ms;
            for (int j = 0; j < nc; j++)
                tot.true_rel_resid[(a0 + j) % DD_MAX_RHS] =
                    std::max(tot.true_rel_resid[(a0 + j) % DD_MAX_RHS], st.true_rel_resid[j]);
            cpx<double>*src = x, *dst = y;
            for (int k = 0; k < n_hop; k++) {
                launch_dslash<double>(c, g, U, kappa, 0, EPI_HOP, src, dst, nullptr, nc, nullptr, nullptr);
                std::swap(src, dst);
            }
            hipLaunchKernelGGL(k_trace_slices, dim3((unsigned)nt, (unsigned)nc), dim3(kTB), 0, c->stream, T, L3, t0, nt,
                               a0, rhs, src, tau);
            DD_HIP(c, hipGetLastError());
        }
        if (stats) stats[d] = tot;
    }
    DD_HIP(c, hipStreamSynchronize(c->stream));
    if (worst != DD_OK) return fail(c, worst, "a disconnected-trace solve did not converge: " + c->err);
    return DD_OK;
}

dd_status disconnected_correlator(dd_ctx* c, int nsrc, const cpx<double>* tau, double* C_host) {
    const int T = c->lat.T, L3 = c->lat.L * c->lat.L * c->lat.L;
    dd_status e = DD_OK;
    cpx<double>* C = (cpx<double>*)workspace(c, W_DISC3, (size_t)T * T * sizeof(cpx<double>), &e);
    if (e != DD_OK) return e;
    const double scale = 1.0 / ((double)nsrc * (nsrc - 1) * L3);
    hipLaunchKernelGGL(k_disc_corr, dim3((unsigned)((T * T + kTB - 1) / kTB)), dim3(kTB), 0, c->stream, T, nsrc, scale,
                       tau, C);
    DD_HIP(c, hipGetLastError());
    DD_HIP(c, hipMemcpyAsync(C_host, C, (size_t)T * T * sizeof(cpx<double>), hipMemcpyDeviceToHost, c->stream));
    DD_HIP(c, hipStreamSynchronize(c->stream));
    return DD_OK;
}

}  // namespace dd
