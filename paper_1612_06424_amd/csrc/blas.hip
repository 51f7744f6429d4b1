// blas.hip -- vector kernels of the Krylov solvers (fused updates with FP64
// partial reductions), the per-column scalar updates, precision conversions and
// the smaller pieces of the hot path: frontier hop, slab copies, point sources,
// the pion contraction and the link force.
//
// Reductions are deterministic: every workgroup writes its partial sums (FP64)
// to a fixed slot and one workgroup per column adds them in a fixed order, so
// results are bitwise reproducible run to run.
#include <cmath>

#include "dd_internal.h"
#include "dd_wilson.h"

namespace dd {

namespace {

__device__ inline cpx<double> cd(double a, double b) { return {a, b}; }

template <typename R>
__device__ inline cpx<R> scal(const double re, const double im, cpx<R> a) {
    return {R(re) * a.re - R(im) * a.im, R(re) * a.im + R(im) * a.re};
}

inline dim3 egrid(int n, int ncol) { return dim3((unsigned)((n + kBlock - 1) / kBlock), (unsigned)ncol); }

// p = r + beta (p - omega v)
template <typename R>
__global__ __launch_bounds__(kBlock) void k_bicg_p(int n, const cpx<R>* __restrict__ r, cpx<R>* __restrict__ p,
                                                   const cpx<R>* __restrict__ v, const ColState* __restrict__ st) {
    const int col = blockIdx.y;
    if (!st[col].active) return;
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const size_t k = (size_t)col * n + i;
    const ColState& s = st[col];
    const cpx<R> t = p[k] - scal(s.omega_re, s.omega_im, v[k]);
    p[k] = r[k] + scal(s.beta_re, s.beta_im, t);
}

// s = r - alpha v
template <typename R>
__global__ __launch_bounds__(kBlock) void k_bicg_s(int n, const cpx<R>* __restrict__ r, const cpx<R>* __restrict__ v,
                                                   cpx<R>* __restrict__ s_, const ColState* __restrict__ st) {
    const int col = blockIdx.y;
    if (!st[col].active) return;
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const size_t k = (size_t)col * n + i;
    s_[k] = r[k] - scal(st[col].alpha_re, st[col].alpha_im, v[k]);
}

// x += alpha p + omega s; r = s - omega t; partials <r^, r>, |r|^2
template <typename R>
__global__ __launch_bounds__(kBlock) void k_bicg_xr(int n, cpx<R>* __restrict__ x, cpx<R>* __restrict__ r,
                                                    const cpx<R>* __restrict__ p, const cpx<R>* __restrict__ s_,
                                                    const cpx<R>* __restrict__ t, const cpx<R>* __restrict__ rh,
                                                    double* __restrict__ partial, const ColState* __restrict__ st) {
    const int col = blockIdx.y;
    if (!st[col].active) return;
    const int i = blockIdx.x * kBlock + threadIdx.x;
    double d0 = 0, d1 = 0, d2 = 0;
    if (i < n) {
        const size_t k = (size_t)col * n + i;
        const ColState& s = st[col];
        const cpx<R> sv = s_[k];
        x[k] = x[k] + scal(s.alpha_re, s.alpha_im, p[k]) + scal(s.omega_re, s.omega_im, sv);
        const cpx<R> rn = sv - scal(s.omega_re, s.omega_im, t[k]);
        r[k] = rn;
        const cpx<R> q = rh[k];
        d0 = (double)q.re * rn.re + (double)q.im * rn.im;
        d1 = (double)q.re * rn.im - (double)q.im * rn.re;
        d2 = (double)rn.re * rn.re + (double)rn.im * rn.im;
    }
    block_sum3(d0, d1, d2, partial + ((size_t)col * gridDim.x + blockIdx.x) * 3);
}

// CGNR: x += alpha p; r -= alpha w; partial |r|^2 (alpha real)
template <typename R>
__global__ __launch_bounds__(kBlock) void k_cg_xr(int n, cpx<R>* __restrict__ x, cpx<R>* __restrict__ r,
                                                  const cpx<R>* __restrict__ p, const cpx<R>* __restrict__ w,
                                                  double* __restrict__ partial, const ColState* __restrict__ st) {
    const int col = blockIdx.y;
    if (!st[col].active) return;
    const int i = blockIdx.x * kBlock + threadIdx.x;
    double d0 = 0;
    if (i < n) {
        const size_t k = (size_t)col * n + i;
        const R a = R(st[col].alpha_re);
        x[k] = x[k] + a * p[k];
        const cpx<R> rn = r[k] - a * w[k];
        r[k] = rn;
        d0 = (double)rn.re * rn.re + (double)rn.im * rn.im;
    }
    block_sum3(d0, 0.0, 0.0, partial + ((size_t)col * gridDim.x + blockIdx.x) * 3);
}

// CGNR: p = z + beta p (beta real)
template <typename R>
__global__ __launch_bounds__(kBlock) void k_cg_p(int n, cpx<R>* __restrict__ p, const cpx<R>* __restrict__ z,
                                                 const ColState* __restrict__ st) {
    const int col = blockIdx.y;
    if (!st[col].active) return;
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const size_t k = (size_t)col * n + i;
    p[k] = z[k] + R(st[col].beta_re) * p[k];
}

template <typename R>
__global__ __launch_bounds__(kBlock) void k_norm2(int n, const cpx<R>* __restrict__ a, double* __restrict__ partial) {
    const int col = blockIdx.y;
    const int i = blockIdx.x * kBlock + threadIdx.x;
    double d0 = 0;
    if (i < n) {
        const cpx<R> v = a[(size_t)col * n + i];
        d0 = (double)v.re * v.re + (double)v.im * v.im;
    }
    block_sum3(d0, 0.0, 0.0, partial + ((size_t)col * gridDim.x + blockIdx.x) * 3);
}

// One workgroup per column: fixed-order sum of the column's partials, then the
// scalar recurrences of BiCGStab / CG for that column.
__global__ __launch_bounds__(kBlock) void k_finalize(int fin, int nsb, const double* __restrict__ partial,
                                                     ColState* __restrict__ st, double* __restrict__ out) {
    const int col = blockIdx.x;
    if (fin != FIN_STORE && !st[col].active) return;
    double d0 = 0, d1 = 0, d2 = 0;
    const double* p = partial + (size_t)col * nsb * 3;
    for (int k = threadIdx.x; k < nsb; k += kBlock) {
        d0 += p[3 * k];
        d1 += p[3 * k + 1];
        d2 += p[3 * k + 2];
    }
    __shared__ double red[3];
    block_sum3(d0, d1, d2, red);
    __syncthreads();
    if (threadIdx.x != 0) return;
    d0 = red[0];
    d1 = red[1];
    d2 = red[2];
    if (fin == FIN_STORE) {
        out[col * 3 + 0] = d0;
        out[col * 3 + 1] = d1;
        out[col * 3 + 2] = d2;
        return;
    }
    ColState& s = st[col];
    switch (fin) {
        case FIN_ALPHA: {  // alpha = rho / <r^, v>
            const double den = d0 * d0 + d1 * d1;
            if (!(den > 0) || !isfinite(den)) {
                s.breakdown = isfinite(den) ? 1 : 2;
                s.active = 0;
                break;
            }
            s.alpha_re = (s.rho_re * d0 + s.rho_im * d1) / den;
            s.alpha_im = (s.rho_im * d0 - s.rho_re * d1) / den;
            break;
        }
        case FIN_OMEGA: {  // omega = <t, s> / <t, t>
            if (!(d2 > 0) || !isfinite(d2)) {
                s.breakdown = isfinite(d2) ? 1 : 2;
                s.active = 0;
                break;
            }
            s.omega_re = d0 / d2;
            s.omega_im = d1 / d2;
            if (s.omega_re == 0.0 && s.omega_im == 0.0) {
                s.breakdown = 1;
                s.active = 0;
            }
            break;
        }
        case FIN_RHO: {  // beta = (rho_new / rho) (alpha / omega), rho = rho_new
            const double rr = d2;
            s.rr = rr;
            s.iters += 1;
            if (!isfinite(rr) || !isfinite(d0) || !isfinite(d1)) {
                s.breakdown = 2;
                s.active = 0;
                break;
            }
            if (rr <= s.stop2) {
                s.active = 0;
                break;
            }
            const double rden = s.rho_re * s.rho_re + s.rho_im * s.rho_im;
            const double q_re = (d0 * s.rho_re + d1 * s.rho_im) / rden;  // rho_new / rho
            const double q_im = (d1 * s.rho_re - d0 * s.rho_im) / rden;
            const double oden = s.omega_re * s.omega_re + s.omega_im * s.omega_im;
            const double w_re = (s.alpha_re * s.omega_re + s.alpha_im * s.omega_im) / oden;  // alpha / omega
            const double w_im = (s.alpha_im * s.omega_re - s.alpha_re * s.omega_im) / oden;
            s.beta_re = q_re * w_re - q_im * w_im;
            s.beta_im = q_re * w_im + q_im * w_re;
            s.rho_re = d0;
            s.rho_im = d1;
            if (d0 * d0 + d1 * d1 < 1e-24 * rr * s.rh2) {  // r^ numerically orthogonal to r
                s.breakdown = 1;
                s.active = 0;
            }
            break;
        }
        case FIN_CG_ALPHA: {
            if (!(d0 > 0) || !isfinite(d0)) {
                s.breakdown = isfinite(d0) ? 1 : 2;
                s.active = 0;
                break;
            }
            s.alpha_re = s.zz / d0;
            s.alpha_im = 0;
            break;
        }
        case FIN_CG_RR: {
            s.rr = d0;
            s.iters += 1;
            if (!isfinite(d0)) {
                s.breakdown = 2;
                s.active = 0;
            } else if (d0 <= s.stop2) {
                s.active = 0;
            }
            break;
        }
        case FIN_CG_BETA: {
            s.beta_re = d0 / s.zz;
            s.beta_im = 0;
            s.zz = d0;
            break;
        }
        case FIN_INIT: {
            s.rr = d0;
            s.rh2 = d0;
            s.rho_re = d0;
            s.rho_im = 0;
            s.stop2 *= d0;
            s.alpha_re = s.omega_re = 1.0;
            s.alpha_im = s.omega_im = 0.0;
            s.beta_re = s.beta_im = 0.0;
            s.iters = 0;
            s.breakdown = 0;
            if (!isfinite(d0)) {
                s.breakdown = 2;
                s.active = 0;
            } else if (!(d0 > 0)) {
                s.active = 0;
            }
            break;
        }
        case FIN_CG_ZZ: {
            s.zz = d0;
            if (!(d0 > 0) || !isfinite(d0)) {
                s.breakdown = isfinite(d0) ? 1 : 2;
                s.active = 0;
            }
            break;
        }
        default:
            break;
    }
}

template <typename R>
__global__ __launch_bounds__(kBlock) void k_copy_cols(int n, const cpx<R>* __restrict__ a, cpx<R>* __restrict__ b,
                                                      const ColState* __restrict__ st) {
    const int col = blockIdx.y;
    if (st != nullptr && !st[col].active) return;
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    b[(size_t)col * n + i] = a[(size_t)col * n + i];
}


// Reliable update helpers (columns selected by mask[col] != 0):
//   x64 += xk; xk = 0        (xk in the Krylov precision)
//   rk = (Rk) r64            (replace the recursive residual by the true one)
template <typename R>
__global__ __launch_bounds__(kBlock) void k_fold_x(int n, cpx<double>* __restrict__ x, cpx<R>* __restrict__ xk,
                                                   const int* __restrict__ mask) {
    const int col = blockIdx.y;
    if (!mask[col]) return;
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const size_t k = (size_t)col * n + i;
    const cpx<R> e = xk[k];
    const cpx<double> v = x[k];
    x[k] = cd(v.re + (double)e.re, v.im + (double)e.im);
    xk[k] = cpx<R>{R(0), R(0)};
}
template <typename R>
__global__ __launch_bounds__(kBlock) void k_set_resid(int n, const cpx<double>* __restrict__ r64, cpx<R>* __restrict__ rk,
                                                      const int* __restrict__ mask) {
    const int col = blockIdx.y;
    if (!mask[col]) return;
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const size_t k = (size_t)col * n + i;
    const cpx<double> v = r64[k];
    rk[k] = cpx<R>{(R)v.re, (R)v.im};
}
template <typename R>
__global__ __launch_bounds__(kBlock) void k_restart_dirs(int n, const cpx<R>* __restrict__ r, cpx<R>* __restrict__ rh,
                                                         cpx<R>* __restrict__ p, cpx<R>* __restrict__ v,
                                                         const int* __restrict__ mask) {
    const int col = blockIdx.y;
    if (mask[col] != 2) return;
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const size_t k = (size_t)col * n + i;
    rh[k] = r[k];
    p[k] = cpx<R>{R(0), R(0)};
    v[k] = cpx<R>{R(0), R(0)};
}

// CGNR reliable update: p += t - z; z = t (columns with mask != 0)
template <typename R>
__global__ __launch_bounds__(kBlock) void k_cg_shift(int n, cpx<R>* __restrict__ p, cpx<R>* __restrict__ z,
                                                     const cpx<R>* __restrict__ t, const int* __restrict__ mask) {
    const int col = blockIdx.y;
    if (!mask[col]) return;
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const size_t k = (size_t)col * n + i;
    const cpx<R> tv = t[k];
    p[k] = p[k] + tv - z[k];
    z[k] = tv;
}

__global__ __launch_bounds__(kBlock) void k_links_to_f32(size_t n, const cpx<double>* __restrict__ a,
                                                         cpx<float>* __restrict__ b) {
    const size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const cpx<double> v = a[i];
    b[i] = cpx<float>{(float)v.re, (float)v.im};
}

// gamma_5 = diag(1,1,-1,-1): negate spin components 2, 3 (c >= 6)
template <typename R>
__global__ __launch_bounds__(kBlock) void k_gamma5(int nsite, const cpx<R>* __restrict__ a, cpx<R>* __restrict__ b) {
    const int col = blockIdx.y;
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= 12 * nsite) return;
    const size_t k = (size_t)col * 12 * nsite + i;
    const cpx<R> v = a[k];
    b[k] = (i >= 6 * nsite) ? cpx<R>{-v.re, -v.im} : v;
}

template <typename R>
__global__ __launch_bounds__(kBlock) void k_zero(size_t n, cpx<R>* __restrict__ a) {
    const size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) a[i] = cpx<R>{R(0), R(0)};
}

// Frontier block: for each site of dst's first / last time slice, the time hop
// from the neighbouring slice if that slice belongs to src.
__global__ __launch_bounds__(kBlock) void k_frontier(int T, int L3, int bc, int vlink, const cpx<double>* __restrict__ U,
                                                     int dt0, int dnt, int st0, int snt,
                                                     const cpx<double>* __restrict__ in, cpx<double>* __restrict__ out,
                                                     double alpha) {
    const int col = blockIdx.y;
    const int sp = blockIdx.x * kBlock + threadIdx.x;
    if (sp >= L3) return;
    const int nin = snt * L3, nout = dnt * L3;
    const cpx<double>* f = in + (size_t)col * 12 * nin;
    cpx<double>* o = out + (size_t)col * 12 * nout;
    cpx<double> a0[12], a1[12];
#pragma unroll
    for (int c = 0; c < 12; c++) a0[c] = a1[c] = cd(0, 0);
    bool w0 = false, w1 = false;
    // backward hop into dst's first slice
    {
        const int tg = dt0;
        const int tn = (tg == 0) ? T - 1 : tg - 1;
        const int pos = ((tn - st0) % T + T) % T;
        const double ph = (tg == 0) ? (double)bc : 1.0;
        if (pos < snt && ph != 0.0) {
            hop<double, 0, +1, true>(a0, f, nin, pos * L3 + sp, U, vlink, tn * L3 + sp, ph);
            w0 = true;
        }
    }
    // forward hop into dst's last slice
    {
        const int tg = (dt0 + dnt - 1) % T;
        const int tn = (tg == T - 1) ? 0 : tg + 1;
        const int pos = ((tn - st0) % T + T) % T;
        const double ph = (tg == T - 1) ? (double)bc : 1.0;
        if (pos < snt && ph != 0.0) {
            hop<double, 0, -1, false>(a1, f, nin, pos * L3 + sp, U, vlink, tg * L3 + sp, ph);
            w1 = true;
        }
    }
    if (dnt == 1 && w1) {  // a one-slice dst: both hops land on the same site
#pragma unroll
        for (int c = 0; c < 12; c++) a0[c] = a0[c] + a1[c];
        w0 = true;
        w1 = false;
    }
    const double s = -0.5 * alpha;
    if (w0) {
#pragma unroll
        for (int c = 0; c < 12; c++) {
            cpx<double>& y = o[c * nout + sp];
            y = cd(y.re + s * a0[c].re, y.im + s * a0[c].im);
        }
    }
    if (w1) {
        const int sl = (dnt - 1) * L3 + sp;
#pragma unroll
        for (int c = 0; c < 12; c++) {
            cpx<double>& y = o[c * nout + sl];
            y = cd(y.re + s * a1[c].re, y.im + s * a1[c].im);
        }
    }
}

// compact slab field <-> whole-lattice field; dir 0: scatter (slab -> whole), 1: gather
__global__ __launch_bounds__(kBlock) void k_slab_copy(int T, int L3, int t0, int nt, int dir,
                                                      cpx<double>* __restrict__ whole, cpx<double>* __restrict__ part) {
    const int row = blockIdx.y;  // col * 12 + c
    const int i = blockIdx.x * kBlock + threadIdx.x;
    const int nsite = nt * L3;
    if (i >= nsite) return;
    const int tl = i / L3, sp = i - tl * L3;
    int tg = t0 + tl;
    if (tg >= T) tg -= T;
    const size_t w = (size_t)row * T * L3 + (size_t)tg * L3 + sp;
    const size_t p = (size_t)row * nsite + i;
    if (dir == 0)
        whole[w] = part[p];
    else
        part[p] = whole[w];
}

__global__ void k_point_source(int nsite, int site, cpx<double>* __restrict__ eta) {
    const int j = threadIdx.x;
    if (j < 12) eta[(size_t)(j * 12 + j) * nsite + site] = cd(1.0, 0.0);
}

// pion: partial[t][row] = sum over the slice's spatial sites of |S_row|^2
__global__ __launch_bounds__(kBlock) void k_pion_partial(int T, int L3, int nrow, int t_src,
                                                         const cpx<double>* __restrict__ S,
                                                         double* __restrict__ partial) {
    const int row = blockIdx.x, t = blockIdx.y;
    const int ts = (t_src + t) % T;
    const cpx<double>* p = S + (size_t)row * T * L3 + (size_t)ts * L3;
    double acc = 0;
    for (int k = threadIdx.x; k < L3; k += kBlock) {
        const cpx<double> v = p[k];
        acc += v.re * v.re + v.im * v.im;
    }
    block_sum3(acc, 0.0, 0.0, partial + ((size_t)t * nrow + row) * 3);
}

__global__ __launch_bounds__(kBlock) void k_pion_final(int nrow, const double* __restrict__ partial,
                                                       double* __restrict__ C) {
    const int t = blockIdx.x;
    double acc = 0;
    for (int k = threadIdx.x; k < nrow; k += kBlock) acc += partial[((size_t)t * nrow + k) * 3];
    __shared__ double red[3];
    block_sum3(acc, 0.0, 0.0, red);
    __syncthreads();
    if (threadIdx.x == 0) C[t] = red[0];
}

// Link force on slab geometry g: for each slab site and direction whose
// forward hop stays in the slab,
//   grad_mu(x) += coeff ph sum_col sum_spin [ a_s X_s(x+mu)^+ + X_s(x) b_s^+ ],
// a = (1 - gamma_mu) Y(x), b = (1 + gamma_mu) Y(x+mu).
template <int MU>
__device__ inline void full_proj(const cpx<double> (&y)[12], int sgn, cpx<double> (&out)[12]) {
    cpx<double> h[6];
#pragma unroll
    for (int c = 0; c < 12; c++) out[c] = cd(0, 0);
    if (sgn < 0) {
        project<double, MU, -1>(y, h);
        accum<double, MU, -1>(out, h);
    } else {
        project<double, MU, +1>(y, h);
        accum<double, MU, +1>(out, h);
    }
}

template <int MU>
__device__ inline void force_dir(const Geo& g, int s, int nb, int sl, double ph, int ncol,
                                 const cpx<double>* __restrict__ X, const cpx<double>* __restrict__ Y,
                                 double coeff, cpx<double>* __restrict__ grad) {
    cpx<double> G[9];
#pragma unroll
    for (int k = 0; k < 9; k++) G[k] = cd(0, 0);
    const int ns = g.nsite;
    for (int col = 0; col < ncol; col++) {
        const cpx<double>* Xc = X + (size_t)col * 12 * ns;
        const cpx<double>* Yc = Y + (size_t)col * 12 * ns;
        cpx<double> yx[12], yn[12], a[12], b[12], xx[12], xn[12];
        load_spinor(Yc, ns, s, yx);
        load_spinor(Yc, ns, nb, yn);
        load_spinor(Xc, ns, s, xx);
        load_spinor(Xc, ns, nb, xn);
        full_proj<MU>(yx, -1, a);
        full_proj<MU>(yn, +1, b);
#pragma unroll
        for (int sp = 0; sp < 4; sp++)
#pragma unroll
            for (int r = 0; r < 3; r++)
#pragma unroll
                for (int k = 0; k < 3; k++) {
                    // a_r conj(xn_k) + xx_r conj(b_k)
                    const cpx<double> t1 = cmulc(xn[3 * sp + k], a[3 * sp + r]);
                    const cpx<double> t2 = cmulc(b[3 * sp + k], xx[3 * sp + r]);
                    G[3 * r + k] = G[3 * r + k] + t1 + t2;
                }
    }
    const double f = coeff * ph;
#pragma unroll
    for (int k = 0; k < 9; k++) {
        cpx<double>& o = grad[(size_t)(MU * 9 + k) * g.vlink + sl];
        o = cd(o.re + f * G[k].re, o.im + f * G[k].im);
    }
}

__global__ __launch_bounds__(kBlock) void k_link_force(Geo g, int ncol, const cpx<double>* __restrict__ X,
                                                       const cpx<double>* __restrict__ Y, double coeff,
                                                       cpx<double>* __restrict__ grad) {
    const int s = blockIdx.x * kBlock + threadIdx.x;
    if (s >= g.nsite) return;
    const int L = g.L, L2 = g.L2, L3 = g.L3;
    const int tl = s / L3, sp = s - tl * L3;
    const int x = sp % L, yz = sp / L, y = yz % L, z = yz / L;
    int tg = g.t0 + tl;
    if (tg >= g.T) tg -= g.T;
    const int sl = tg * L3 + sp;
    // time: the forward neighbour must be in the field and the hop present
    {
        const bool end = (tl == g.nt - 1);
        const double ph = (tg == g.T - 1) ? (double)g.bc : 1.0;
        if ((!end || g.whole) && ph != 0.0) {
            const int nb = end ? s - (g.nt - 1) * L3 : s + L3;
            force_dir<0>(g, s, nb, sl, ph, ncol, X, Y, coeff, grad);
        }
    }
    force_dir<1>(g, s, s + ((x == L - 1) ? -(L - 1) : 1), sl, 1.0, ncol, X, Y, coeff, grad);
    force_dir<2>(g, s, s + ((y == L - 1) ? -(L - 1) * L : L), sl, 1.0, ncol, X, Y, coeff, grad);
    force_dir<3>(g, s, s + ((z == L - 1) ? -(L - 1) * L2 : L2), sl, 1.0, ncol, X, Y, coeff, grad);
}

}  // namespace

// ------------------------------------------------------------------ launchers

template <typename R>
void launch_bicg_p(dd_ctx* c, int n, int ncol, const cpx<R>* r, cpx<R>* p, const cpx<R>* v, const ColState* st) {
    hipLaunchKernelGGL(k_bicg_p<R>, egrid(n, ncol), dim3(kBlock), 0, c->stream, n, r, p, v, st);
}
template <typename R>
void launch_bicg_s(dd_ctx* c, int n, int ncol, const cpx<R>* r, const cpx<R>* v, cpx<R>* s, const ColState* st) {
    hipLaunchKernelGGL(k_bicg_s<R>, egrid(n, ncol), dim3(kBlock), 0, c->stream, n, r, v, s, st);
}
template <typename R>
void launch_bicg_xr(dd_ctx* c, int n, int ncol, cpx<R>* x, cpx<R>* r, const cpx<R>* p, const cpx<R>* s,
                    const cpx<R>* t, const cpx<R>* rh, double* partial, const ColState* st) {
    hipLaunchKernelGGL(k_bicg_xr<R>, egrid(n, ncol), dim3(kBlock), 0, c->stream, n, x, r, p, s, t, rh, partial, st);
}
template <typename R>
void launch_cg_xr(dd_ctx* c, int n, int ncol, cpx<R>* x, cpx<R>* r, const cpx<R>* p, const cpx<R>* w,
                  double* partial, const ColState* st) {
    hipLaunchKernelGGL(k_cg_xr<R>, egrid(n, ncol), dim3(kBlock), 0, c->stream, n, x, r, p, w, partial, st);
}
template <typename R>
void launch_cg_p(dd_ctx* c, int n, int ncol, cpx<R>* p, const cpx<R>* z, const ColState* st) {
    hipLaunchKernelGGL(k_cg_p<R>, egrid(n, ncol), dim3(kBlock), 0, c->stream, n, p, z, st);
}
template <typename R>
void launch_norm2(dd_ctx* c, int n, int ncol, const cpx<R>* a, double* partial) {
    hipLaunchKernelGGL(k_norm2<R>, egrid(n, ncol), dim3(kBlock), 0, c->stream, n, a, partial);
}
void launch_finalize(dd_ctx* c, int fin, int ncol, int nsb, const double* partial, ColState* st, double* out) {
    hipLaunchKernelGGL(k_finalize, dim3(ncol), dim3(kBlock), 0, c->stream, fin, nsb, partial, st, out);
}
template <typename R>
void launch_copy_cols(dd_ctx* c, int n, int ncol, const cpx<R>* src, cpx<R>* dst, const ColState* st) {
    hipLaunchKernelGGL(k_copy_cols<R>, egrid(n, ncol), dim3(kBlock), 0, c->stream, n, src, dst, st);
}
void launch_links_to_f32(dd_ctx* c, size_t n, const cpx<double>* src, cpx<float>* dst) {
    hipLaunchKernelGGL(k_links_to_f32, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, c->stream,
                       n, src, dst);
}
template <typename R>
void launch_gamma5(dd_ctx* c, int nsite, int ncol, const cpx<R>* in, cpx<R>* out) {
    hipLaunchKernelGGL(k_gamma5<R>, egrid(12 * nsite, ncol), dim3(kBlock), 0, c->stream, nsite, in, out);
}
template <typename R>
void launch_zero(dd_ctx* c, size_t n, cpx<R>* a) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_zero<R>, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, c->stream, n, a);
}

void launch_frontier(dd_ctx* c, const dd_lattice& lat, const cpx<double>* U, const dd_domain& dst,
                     const dd_domain& src, int ncol, const cpx<double>* in, cpx<double>* out, double alpha) {
    const int L3 = lat.L * lat.L * lat.L;
    hipLaunchKernelGGL(k_frontier, dim3((unsigned)((L3 + kBlock - 1) / kBlock), (unsigned)ncol), dim3(kBlock), 0,
                       c->stream, lat.T, L3, lat.time_bc, lat.T * L3, U, dst.t0, dst.nt, src.t0, src.nt, in, out,
                       alpha);
}

void launch_slab_scatter(dd_ctx* c, const dd_lattice& lat, const dd_domain& dom, int ncol,
                         const cpx<double>* part, cpx<double>* whole) {
    const int L3 = lat.L * lat.L * lat.L;
    const int n = dom.nt * L3;
    hipLaunchKernelGGL(k_slab_copy, dim3((unsigned)((n + kBlock - 1) / kBlock), (unsigned)(12 * ncol)), dim3(kBlock),
                       0, c->stream, lat.T, L3, dom.t0, dom.nt, 0, whole, const_cast<cpx<double>*>(part));
}

void launch_slab_gather(dd_ctx* c, const dd_lattice& lat, const dd_domain& dom, int ncol,
                        const cpx<double>* whole, cpx<double>* part) {
    const int L3 = lat.L * lat.L * lat.L;
    const int n = dom.nt * L3;
    hipLaunchKernelGGL(k_slab_copy, dim3((unsigned)((n + kBlock - 1) / kBlock), (unsigned)(12 * ncol)), dim3(kBlock),
                       0, c->stream, lat.T, L3, dom.t0, dom.nt, 1, const_cast<cpx<double>*>(whole), part);
}

void launch_point_source(dd_ctx* c, int nsite, int site, cpx<double>* eta) {
    launch_zero<double>(c, (size_t)144 * nsite, eta);
    hipLaunchKernelGGL(k_point_source, dim3(1), dim3(64), 0, c->stream, nsite, site, eta);
}

void launch_pion(dd_ctx* c, const dd_lattice& lat, int ncol, const cpx<double>* S, int t_src, double* partial,
                 double* C) {
    const int L3 = lat.L * lat.L * lat.L;
    const int nrow = 12 * ncol;
    hipLaunchKernelGGL(k_pion_partial, dim3((unsigned)nrow, (unsigned)lat.T), dim3(kBlock), 0, c->stream, lat.T, L3,
                       nrow, t_src, S, partial);
    hipLaunchKernelGGL(k_pion_final, dim3((unsigned)lat.T), dim3(kBlock), 0, c->stream, nrow, partial, C);
}

void launch_link_force(dd_ctx* c, const Geo& g, int ncol, const cpx<double>* X, const cpx<double>* Y, double coeff,
                       cpx<double>* grad) {
    hipLaunchKernelGGL(k_link_force, dim3((unsigned)site_blocks(g.nsite)), dim3(kBlock), 0, c->stream, g, ncol, X, Y,
                       coeff, grad);
}


template <typename R>
void launch_fold_x(dd_ctx* c, int n, int ncol, cpx<double>* x, cpx<R>* xk, const int* mask) {
    hipLaunchKernelGGL(k_fold_x<R>, egrid(n, ncol), dim3(kBlock), 0, c->stream, n, x, xk, mask);
}
template <typename R>
void launch_set_resid(dd_ctx* c, int n, int ncol, const cpx<double>* r64, cpx<R>* rk, const int* mask) {
    hipLaunchKernelGGL(k_set_resid<R>, egrid(n, ncol), dim3(kBlock), 0, c->stream, n, r64, rk, mask);
}
template <typename R>
void launch_restart_dirs(dd_ctx* c, int n, int ncol, const cpx<R>* r, cpx<R>* rh, cpx<R>* p, cpx<R>* v,
                         const int* mask) {
    hipLaunchKernelGGL(k_restart_dirs<R>, egrid(n, ncol), dim3(kBlock), 0, c->stream, n, r, rh, p, v, mask);
}
template void launch_fold_x<float>(dd_ctx*, int, int, cpx<double>*, cpx<float>*, const int*);
template void launch_set_resid<float>(dd_ctx*, int, int, const cpx<double>*, cpx<float>*, const int*);
template void launch_set_resid<double>(dd_ctx*, int, int, const cpx<double>*, cpx<double>*, const int*);
template void launch_restart_dirs<float>(dd_ctx*, int, int, const cpx<float>*, cpx<float>*, cpx<float>*, cpx<float>*,
                                         const int*);
template void launch_restart_dirs<double>(dd_ctx*, int, int, const cpx<double>*, cpx<double>*, cpx<double>*,
                                          cpx<double>*, const int*);

template <typename R>
void launch_cg_shift(dd_ctx* c, int n, int ncol, cpx<R>* p, cpx<R>* z, const cpx<R>* t, const int* mask) {
    hipLaunchKernelGGL(k_cg_shift<R>, egrid(n, ncol), dim3(kBlock), 0, c->stream, n, p, z, t, mask);
}
template void launch_cg_shift<float>(dd_ctx*, int, int, cpx<float>*, cpx<float>*, const cpx<float>*, const int*);
template void launch_cg_shift<double>(dd_ctx*, int, int, cpx<double>*, cpx<double>*, const cpx<double>*, const int*);

#define DD_INST(R)                                                                                           \
    template void launch_bicg_p<R>(dd_ctx*, int, int, const cpx<R>*, cpx<R>*, const cpx<R>*, const ColState*); \
    template void launch_bicg_s<R>(dd_ctx*, int, int, const cpx<R>*, const cpx<R>*, cpx<R>*, const ColState*); \
    template void launch_bicg_xr<R>(dd_ctx*, int, int, cpx<R>*, cpx<R>*, const cpx<R>*, const cpx<R>*,          \
                                    const cpx<R>*, const cpx<R>*, double*, const ColState*);                   \
    template void launch_cg_xr<R>(dd_ctx*, int, int, cpx<R>*, cpx<R>*, const cpx<R>*, const cpx<R>*, double*,   \
                                  const ColState*);                                                            \
    template void launch_cg_p<R>(dd_ctx*, int, int, cpx<R>*, const cpx<R>*, const ColState*);                  \
    template void launch_norm2<R>(dd_ctx*, int, int, const cpx<R>*, double*);                                   \
    template void launch_copy_cols<R>(dd_ctx*, int, int, const cpx<R>*, cpx<R>*, const ColState*);             \
    template void launch_gamma5<R>(dd_ctx*, int, int, const cpx<R>*, cpx<R>*);                                  \
    template void launch_zero<R>(dd_ctx*, size_t, cpx<R>*);

DD_INST(double)
DD_INST(float)

}  // namespace dd
