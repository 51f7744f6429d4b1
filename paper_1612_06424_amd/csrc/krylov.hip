// krylov.hip -- vector kernels of the Krylov solvers.
//
// A solve advances many columns ("segments") together: the columns of one
// lattice, or every column of every domain of a batch.  Segments are laid out
// back to back in each work vector and may differ in length; every elementwise
// workgroup covers kBlock * kElems consecutive elements of one segment (each
// thread kElems of them, kBlock apart, so every load is coalesced), found
// through a workgroup -> segment table (Segs).  Columns whose ColState is inactive skip
// their work; the reliable-update helpers are selected by a per-segment mask.
//
// Reductions are deterministic: every workgroup writes its FP64 partial sums
// to a fixed slot and k_finalize adds a segment's slots in a fixed order, so
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

// This workgroup's segment, and the first of this thread's kElems elements
// (element j of the thread is k + j * kBlock).
struct SegPos {
    int seg;
    int i0;     // offset of the first element inside the segment
    int len;    // segment length
    size_t k;   // index of the first element in the work vectors
    __device__ bool live(int j) const { return i0 + j * kBlock < len; }
    __device__ bool full() const { return i0 + (kElems - 1) * kBlock < len; }
    __device__ size_t at(int j) const { return k + (size_t)j * kBlock; }
};
__device__ inline SegPos seg_pos(const Segs& S) {
    SegPos q;
    q.seg = S.eseg[blockIdx.x];
    q.i0 = ((int)blockIdx.x - S.eb0[q.seg]) * (kBlock * kElems) + (int)threadIdx.x;
    q.len = S.len[q.seg];
    q.k = (size_t)S.off[q.seg] + (size_t)q.i0;
    return q;
}

// Elementwise kernels read all their inputs for the kElems elements first
// (LD), then compute and store (OP), so that every load of a thread is in
// flight at once; a workgroup at the end of a segment takes the checked path.
#define SEG_LOOP(LD, OP)                                          \
    if (q.full()) {                                               \
        _Pragma("unroll") for (int j = 0; j < kElems; j++) LD;    \
        _Pragma("unroll") for (int j = 0; j < kElems; j++) OP;    \
    } else {                                                      \
        for (int j = 0; j < kElems; j++)                          \
            if (q.live(j)) {                                      \
                LD;                                               \
                OP;                                               \
            }                                                     \
    }

// p = r + beta (p - omega v)
template <typename R>
__global__ __launch_bounds__(kBlock) void k_bicg_p(Segs S, const cpx<R>* __restrict__ r, cpx<R>* __restrict__ p,
                                                   const cpx<R>* __restrict__ v, const ColState* __restrict__ st) {
    const SegPos q = seg_pos(S);
    if (!st[q.seg].active) return;
    const ColState& s = st[q.seg];
    cpx<R> rv[kElems], pv[kElems], vv[kElems];
    SEG_LOOP((rv[j] = r[q.at(j)], pv[j] = p[q.at(j)], vv[j] = v[q.at(j)]),
             (p[q.at(j)] = rv[j] + scal(s.beta_re, s.beta_im, pv[j] - scal(s.omega_re, s.omega_im, vv[j]))))
}

// s = r - alpha v
template <typename R>
__global__ __launch_bounds__(kBlock) void k_bicg_s(Segs S, const cpx<R>* __restrict__ r, const cpx<R>* __restrict__ v,
                                                   cpx<R>* __restrict__ s_, const ColState* __restrict__ st) {
    const SegPos q = seg_pos(S);
    if (!st[q.seg].active) return;
    const ColState& s = st[q.seg];
    cpx<R> rv[kElems], vv[kElems];
    SEG_LOOP((rv[j] = r[q.at(j)], vv[j] = v[q.at(j)]), (s_[q.at(j)] = rv[j] - scal(s.alpha_re, s.alpha_im, vv[j])))
}

// x += alpha p + omega s; r = s - omega t; partials <r^, r>, |r|^2
template <typename R>
__global__ __launch_bounds__(kBlock) void k_bicg_xr(Segs S, cpx<R>* __restrict__ x, cpx<R>* __restrict__ r,
                                                    const cpx<R>* __restrict__ p, const cpx<R>* __restrict__ s_,
                                                    const cpx<R>* __restrict__ t, const cpx<R>* __restrict__ rh,
                                                    double* __restrict__ partial, const ColState* __restrict__ st) {
    const SegPos q = seg_pos(S);
    if (!st[q.seg].active) return;  // uniform over the workgroup
    double d0 = 0, d1 = 0, d2 = 0;
    const ColState& s = st[q.seg];
    cpx<R> xv[kElems], pv[kElems], sv[kElems], tv[kElems], hv[kElems];
    SEG_LOOP((xv[j] = x[q.at(j)], pv[j] = p[q.at(j)], sv[j] = s_[q.at(j)], tv[j] = t[q.at(j)], hv[j] = rh[q.at(j)]),
             ({
                 x[q.at(j)] = xv[j] + scal(s.alpha_re, s.alpha_im, pv[j]) + scal(s.omega_re, s.omega_im, sv[j]);
                 const cpx<R> rn = sv[j] - scal(s.omega_re, s.omega_im, tv[j]);
                 r[q.at(j)] = rn;
                 d0 += (double)hv[j].re * rn.re + (double)hv[j].im * rn.im;
                 d1 += (double)hv[j].re * rn.im - (double)hv[j].im * rn.re;
                 d2 += (double)rn.re * rn.re + (double)rn.im * rn.im;
             }))
    block_sum3(d0, d1, d2, partial + (size_t)blockIdx.x * 3);
}

// CGNR: x += alpha p; r -= alpha w; partial |r|^2 (alpha real)
template <typename R>
__global__ __launch_bounds__(kBlock) void k_cg_xr(Segs S, cpx<R>* __restrict__ x, cpx<R>* __restrict__ r,
                                                  const cpx<R>* __restrict__ p, const cpx<R>* __restrict__ w,
                                                  double* __restrict__ partial, const ColState* __restrict__ st) {
    const SegPos q = seg_pos(S);
    if (!st[q.seg].active) return;
    double d0 = 0;
    const R a = R(st[q.seg].alpha_re);
    cpx<R> xv[kElems], pv[kElems], rv[kElems], wv[kElems];
    SEG_LOOP((xv[j] = x[q.at(j)], pv[j] = p[q.at(j)], rv[j] = r[q.at(j)], wv[j] = w[q.at(j)]),
             ({
                 x[q.at(j)] = xv[j] + a * pv[j];
                 const cpx<R> rn = rv[j] - a * wv[j];
                 r[q.at(j)] = rn;
                 d0 += (double)rn.re * rn.re + (double)rn.im * rn.im;
             }))
    block_sum3(d0, 0.0, 0.0, partial + (size_t)blockIdx.x * 3);
}

// CGNR: p = z + beta p (beta real)
template <typename R>
__global__ __launch_bounds__(kBlock) void k_cg_p(Segs S, cpx<R>* __restrict__ p, const cpx<R>* __restrict__ z,
                                                 const ColState* __restrict__ st) {
    const SegPos q = seg_pos(S);
    if (!st[q.seg].active) return;
    const R b = R(st[q.seg].beta_re);
    cpx<R> zv[kElems], pv[kElems];
    SEG_LOOP((zv[j] = z[q.at(j)], pv[j] = p[q.at(j)]), (p[q.at(j)] = zv[j] + b * pv[j]))
}

// partial |a|^2 of every segment
template <typename R>
__global__ __launch_bounds__(kBlock) void k_norm2(Segs S, const cpx<R>* __restrict__ a, double* __restrict__ partial) {
    const SegPos q = seg_pos(S);
    double d0 = 0;
    cpx<R> v[kElems];
    SEG_LOOP((v[j] = a[q.at(j)]), (d0 += (double)v[j].re * v[j].re + (double)v[j].im * v[j].im))
    block_sum3(d0, 0.0, 0.0, partial + (size_t)blockIdx.x * 3);
}

// b = a on the active segments
template <typename R>
__global__ __launch_bounds__(kBlock) void k_copy_segs(Segs S, const cpx<R>* __restrict__ a, cpx<R>* __restrict__ b,
                                                      const ColState* __restrict__ st) {
    const SegPos q = seg_pos(S);
    if (!st[q.seg].active) return;
    cpx<R> v[kElems];
    SEG_LOOP((v[j] = a[q.at(j)]), (b[q.at(j)] = v[j]))
}

// Reliable-update helpers (segments selected by mask[seg] != 0):
//   x64 += xk; xk = 0        (xk in the Krylov precision)
//   rk = (Rk) r64            (replace the recursive residual by the true one)
template <typename R>
__global__ __launch_bounds__(kBlock) void k_fold_x(Segs S, cpx<double>* __restrict__ x, cpx<R>* __restrict__ xk,
                                                   const int* __restrict__ mask) {
    const SegPos q = seg_pos(S);
    if (!mask[q.seg]) return;
    cpx<R> e[kElems];
    cpx<double> v[kElems];
    SEG_LOOP((e[j] = xk[q.at(j)], v[j] = x[q.at(j)]),
             (x[q.at(j)] = cd(v[j].re + (double)e[j].re, v[j].im + (double)e[j].im), xk[q.at(j)] = cpx<R>{R(0), R(0)}))
}
template <typename R>
__global__ __launch_bounds__(kBlock) void k_set_resid(Segs S, const cpx<double>* __restrict__ r64,
                                                      cpx<R>* __restrict__ rk, const int* __restrict__ mask) {
    const SegPos q = seg_pos(S);
    if (!mask[q.seg]) return;
    cpx<double> v[kElems];
    SEG_LOOP((v[j] = r64[q.at(j)]), (rk[q.at(j)] = cpx<R>{(R)v[j].re, (R)v[j].im}))
}
// BiCGStab restart (mask == 2): fresh shadow residual r^ = r, directions cleared
template <typename R>
__global__ __launch_bounds__(kBlock) void k_restart_dirs(Segs S, const cpx<R>* __restrict__ r, cpx<R>* __restrict__ rh,
                                                         cpx<R>* __restrict__ p, cpx<R>* __restrict__ v,
                                                         const int* __restrict__ mask) {
    const SegPos q = seg_pos(S);
    if (mask[q.seg] != 2) return;
    cpx<R> v_[kElems];
    SEG_LOOP((v_[j] = r[q.at(j)]),
             (rh[q.at(j)] = v_[j], p[q.at(j)] = cpx<R>{R(0), R(0)}, v[q.at(j)] = cpx<R>{R(0), R(0)}))
}
// CGNR reliable update: p += t - z; z = t
template <typename R>
__global__ __launch_bounds__(kBlock) void k_cg_shift(Segs S, cpx<R>* __restrict__ p, cpx<R>* __restrict__ z,
                                                     const cpx<R>* __restrict__ t, const int* __restrict__ mask) {
    const SegPos q = seg_pos(S);
    if (!mask[q.seg]) return;
    cpx<R> tv[kElems], pv[kElems], zv[kElems];
    SEG_LOOP((tv[j] = t[q.at(j)], pv[j] = p[q.at(j)], zv[j] = z[q.at(j)]),
             (p[q.at(j)] = pv[j] + tv[j] - zv[j], z[q.at(j)] = tv[j]))
}

// a = 0 on the masked segments (a solve started from a guess whose source column is zero)
__global__ __launch_bounds__(kBlock) void k_zero_segs(Segs S, cpx<double>* __restrict__ a, const int* __restrict__ mask) {
    const SegPos q = seg_pos(S);
    if (!mask[q.seg]) return;
    SEG_LOOP((void)0, (a[q.at(j)] = cd(0.0, 0.0)))
}

// One workgroup per segment: fixed-order sum of the segment's partial slots
// [p0[seg], p0[seg+1]), then the scalar recurrences of BiCGStab / CG for it.
__global__ __launch_bounds__(kBlock) void k_finalize(int fin, const int* __restrict__ p0,
                                                     const double* __restrict__ partial, ColState* __restrict__ st,
                                                     double* __restrict__ out) {
    const int seg = blockIdx.x;
    if (fin != FIN_STORE && !st[seg].active) return;
    double d0 = 0, d1 = 0, d2 = 0;
    const int k0 = p0[seg], k1 = p0[seg + 1];
    for (int k = k0 + (int)threadIdx.x; k < k1; k += kBlock) {
        d0 += partial[3 * (size_t)k];
        d1 += partial[3 * (size_t)k + 1];
        d2 += partial[3 * (size_t)k + 2];
    }
    __shared__ double red[3];
    block_sum3(d0, d1, d2, red);
    __syncthreads();
    if (threadIdx.x != 0) return;
    d0 = red[0];
    d1 = red[1];
    d2 = red[2];
    if (fin == FIN_STORE) {
        out[seg * 3 + 0] = d0;
        out[seg * 3 + 1] = d1;
        out[seg * 3 + 2] = d2;
        return;
    }
    ColState& s = st[seg];
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


#undef SEG_LOOP

}  // namespace

inline dim3 sgrid(const Segs& S) { return dim3((unsigned)S.neb); }

template <typename R>
void launch_bicg_p(dd_ctx* c, const Segs& S, const cpx<R>* r, cpx<R>* p, const cpx<R>* v, const ColState* st) {
    hipLaunchKernelGGL(k_bicg_p<R>, sgrid(S), dim3(kBlock), 0, c->stream, S, r, p, v, st);
}
template <typename R>
void launch_bicg_s(dd_ctx* c, const Segs& S, const cpx<R>* r, const cpx<R>* v, cpx<R>* s, const ColState* st) {
    hipLaunchKernelGGL(k_bicg_s<R>, sgrid(S), dim3(kBlock), 0, c->stream, S, r, v, s, st);
}
template <typename R>
void launch_bicg_xr(dd_ctx* c, const Segs& S, cpx<R>* x, cpx<R>* r, const cpx<R>* p, const cpx<R>* s,
                    const cpx<R>* t, const cpx<R>* rh, double* partial, const ColState* st) {
    hipLaunchKernelGGL(k_bicg_xr<R>, sgrid(S), dim3(kBlock), 0, c->stream, S, x, r, p, s, t, rh, partial, st);
}
template <typename R>
void launch_cg_xr(dd_ctx* c, const Segs& S, cpx<R>* x, cpx<R>* r, const cpx<R>* p, const cpx<R>* w,
                  double* partial, const ColState* st) {
    hipLaunchKernelGGL(k_cg_xr<R>, sgrid(S), dim3(kBlock), 0, c->stream, S, x, r, p, w, partial, st);
}
template <typename R>
void launch_cg_p(dd_ctx* c, const Segs& S, cpx<R>* p, const cpx<R>* z, const ColState* st) {
    hipLaunchKernelGGL(k_cg_p<R>, sgrid(S), dim3(kBlock), 0, c->stream, S, p, z, st);
}
template <typename R>
void launch_norm2(dd_ctx* c, const Segs& S, const cpx<R>* a, double* partial) {
    hipLaunchKernelGGL(k_norm2<R>, sgrid(S), dim3(kBlock), 0, c->stream, S, a, partial);
}
template <typename R>
void launch_copy_segs(dd_ctx* c, const Segs& S, const cpx<R>* a, cpx<R>* b, const ColState* st) {
    hipLaunchKernelGGL(k_copy_segs<R>, sgrid(S), dim3(kBlock), 0, c->stream, S, a, b, st);
}
template <typename R>
void launch_fold_x(dd_ctx* c, const Segs& S, cpx<double>* x, cpx<R>* xk, const int* mask) {
    hipLaunchKernelGGL(k_fold_x<R>, sgrid(S), dim3(kBlock), 0, c->stream, S, x, xk, mask);
}
template <typename R>
void launch_set_resid(dd_ctx* c, const Segs& S, const cpx<double>* r64, cpx<R>* rk, const int* mask) {
    hipLaunchKernelGGL(k_set_resid<R>, sgrid(S), dim3(kBlock), 0, c->stream, S, r64, rk, mask);
}
template <typename R>
void launch_restart_dirs(dd_ctx* c, const Segs& S, const cpx<R>* r, cpx<R>* rh, cpx<R>* p, cpx<R>* v,
                         const int* mask) {
    hipLaunchKernelGGL(k_restart_dirs<R>, sgrid(S), dim3(kBlock), 0, c->stream, S, r, rh, p, v, mask);
}
template <typename R>
void launch_cg_shift(dd_ctx* c, const Segs& S, cpx<R>* p, cpx<R>* z, const cpx<R>* t, const int* mask) {
    hipLaunchKernelGGL(k_cg_shift<R>, sgrid(S), dim3(kBlock), 0, c->stream, S, p, z, t, mask);
}
void launch_zero_segs(dd_ctx* c, const Segs& S, cpx<double>* a, const int* mask) {
    hipLaunchKernelGGL(k_zero_segs, dim3((unsigned)S.neb), dim3(kBlock), 0, c->stream, S, a, mask);
}

void launch_finalize(dd_ctx* c, int fin, int nseg, const int* p0, const double* partial, ColState* st,
                     double* out) {
    hipLaunchKernelGGL(k_finalize, dim3((unsigned)nseg), dim3(kBlock), 0, c->stream, fin, p0, partial, st, out);
}

#define DD_INST(R)                                                                                              \
    template void launch_bicg_p<R>(dd_ctx*, const Segs&, const cpx<R>*, cpx<R>*, const cpx<R>*, const ColState*); \
    template void launch_bicg_s<R>(dd_ctx*, const Segs&, const cpx<R>*, const cpx<R>*, cpx<R>*, const ColState*); \
    template void launch_bicg_xr<R>(dd_ctx*, const Segs&, cpx<R>*, cpx<R>*, const cpx<R>*, const cpx<R>*,       \
                                    const cpx<R>*, const cpx<R>*, double*, const ColState*);                   \
    template void launch_cg_xr<R>(dd_ctx*, const Segs&, cpx<R>*, cpx<R>*, const cpx<R>*, const cpx<R>*, double*, \
                                  const ColState*);                                                            \
    template void launch_cg_p<R>(dd_ctx*, const Segs&, cpx<R>*, const cpx<R>*, const ColState*);               \
    template void launch_norm2<R>(dd_ctx*, const Segs&, const cpx<R>*, double*);                               \
    template void launch_copy_segs<R>(dd_ctx*, const Segs&, const cpx<R>*, cpx<R>*, const ColState*);          \
    template void launch_fold_x<R>(dd_ctx*, const Segs&, cpx<double>*, cpx<R>*, const int*);                   \
    template void launch_set_resid<R>(dd_ctx*, const Segs&, const cpx<double>*, cpx<R>*, const int*);          \
    template void launch_restart_dirs<R>(dd_ctx*, const Segs&, const cpx<R>*, cpx<R>*, cpx<R>*, cpx<R>*,        \
                                         const int*);                                                          \
    template void launch_cg_shift<R>(dd_ctx*, const Segs&, cpx<R>*, cpx<R>*, const cpx<R>*, const int*);
DD_INST(double)
DD_INST(float)
#undef DD_INST

}  // namespace dd
