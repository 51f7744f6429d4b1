// blas.hip -- the smaller kernels of the hot path: precision conversion of the
// links, gamma_5, the frontier hop, slab copies, point sources, the pion
// contraction and the link force.
//
// Reductions are deterministic: every workgroup writes its partial sums (FP64)
// to a fixed slot and one workgroup adds them in a fixed order, so results are
// bitwise reproducible run to run.
#include <cmath>

#include "dd_internal.h"
#include "dd_wilson.h"

namespace dd {

namespace {

__device__ inline cpx<double> cd(double a, double b) { return {a, b}; }

inline dim3 egrid(int n, int ncol) { return dim3((unsigned)((n + kBlock - 1) / kBlock), (unsigned)ncol); }


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

// b = s a (complex128, real s)
__global__ __launch_bounds__(kBlock) void k_scale(size_t n, double s, const cpx<double>* __restrict__ a,
                                                  cpx<double>* __restrict__ b) {
    const size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) b[i] = s * a[i];
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

void launch_scale(dd_ctx* c, size_t n, double s, const cpx<double>* a, cpx<double>* b) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_scale, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, c->stream, n, s, a, b);
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

void launch_slab_embed(dd_ctx* c, int L3, int nt_big, int off, int nt, int ncol, cpx<double>* part,
                       cpx<double>* big, int dir) {
    // the big slab plays the whole lattice of k_slab_copy: nt_big slices, part at slices [off, off + nt)
    const int n = nt * L3;
    hipLaunchKernelGGL(k_slab_copy, dim3((unsigned)((n + kBlock - 1) / kBlock), (unsigned)(12 * ncol)), dim3(kBlock),
                       0, c->stream, nt_big, L3, off, nt, dir, big, part);
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


#define DD_INST(R)                                                           \
    template void launch_gamma5<R>(dd_ctx*, int, int, const cpx<R>*, cpx<R>*); \
    template void launch_zero<R>(dd_ctx*, size_t, cpx<R>*);

DD_INST(double)
DD_INST(float)

}  // namespace dd
