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

// The unit a lane moves per access: one complex number (16 bytes in FP64, 8 in FP32).
// (Two FP32 complex numbers per 16-byte access halve the address requests, but a 16-byte
// FP32 store whose data registers the next arithmetic overwrites at once was seen to
// store the next value for some lanes on this hardware, so FP32 keeps 8-byte units.)
template <typename R>
struct Lane {
    using T = cpx<R>;
    static constexpr int P = 1;
};
template <typename R>
__device__ inline cpx<R> zero_of(cpx<R>) { return {R(0), R(0)}; }
// sums of conj(h) r (re, im) and |r|^2
template <typename R>
__device__ inline void dot_acc(double& d0, double& d1, cpx<R> h, cpx<R> r) {
    d0 += (double)h.re * r.re + (double)h.im * r.im;
    d1 += (double)h.re * r.im - (double)h.im * r.re;
}
template <typename R>
__device__ inline void norm_acc(double& d, cpx<R> r) {
    d += (double)r.re * r.re + (double)r.im * r.im;
}
// FP64 <-> Krylov precision
template <typename R>
__device__ inline cpx<R> narrow(cpx<double> v) { return {(R)v.re, (R)v.im}; }
__device__ inline cpx<double> widen_add(cpx<double> x, cpx<double> e) { return {x.re + e.re, x.im + e.im}; }
__device__ inline cpx<double> widen_add(cpx<double> x, cpx<float> e) {
    return {x.re + (double)e.re, x.im + (double)e.im};
}

// This workgroup's segment, and the first of this thread's units (unit j of the
// thread is k + j * kBlock); P complex numbers per unit.
template <int P>
struct SegPos {
    static constexpr int NE = kElems / P;  // units per thread
    int seg;
    int i0;     // offset of the first unit inside the segment
    int len;    // segment length in units
    size_t k;   // index of the first unit in the work vectors
    __device__ bool live(int j) const { return i0 + j * kBlock < len; }
    __device__ bool full() const { return i0 + (NE - 1) * kBlock < len; }
    __device__ size_t at(int j) const { return k + (size_t)j * kBlock; }
};
template <int P = 1>
__device__ inline SegPos<P> seg_pos(const Segs& S) {
    SegPos<P> q;
    q.seg = S.eseg[blockIdx.x];
    q.i0 = ((int)blockIdx.x - S.eb0[q.seg]) * (kBlock * kElems / P) + (int)threadIdx.x;
    q.len = S.len[q.seg] / P;
    q.k = (size_t)(S.off[q.seg] / P) + (size_t)q.i0;
    return q;
}

// Elementwise kernels read all their inputs for the NE units first (LD), then
// compute and store (OP), so that every load of a thread is in flight at once;
// a workgroup at the end of a segment takes the checked path.
#define SEG_LOOP(LD, OP)                                          \
    if (q.full()) {                                               \
        _Pragma("unroll") for (int j = 0; j < NE; j++) LD;      \
        _Pragma("unroll") for (int j = 0; j < NE; j++) OP;      \
    } else {                                                      \
        for (int j = 0; j < NE; j++)                            \
            if (q.live(j)) {                                      \
                LD;                                               \
                OP;                                               \
            }                                                     \
    }

#define LANE_SETUP(R)                               \
    using T = typename Lane<R>::T;                  \
    constexpr int NE = kElems / Lane<R>::P;         \
    const SegPos<Lane<R>::P> q = seg_pos<Lane<R>::P>(S)
#define AS(T, ptr) reinterpret_cast<T*>(ptr)
#define AS_C(T, ptr) reinterpret_cast<const T*>(ptr)

// p = r + beta (p - omega v)
template <typename R>
__global__ __launch_bounds__(kBlock) void k_bicg_p(Segs S, const cpx<R>* __restrict__ r_, cpx<R>* __restrict__ p_,
                                                   const cpx<R>* __restrict__ v_, const ColState* __restrict__ st) {
    LANE_SETUP(R);
    if (!st[q.seg].active) return;
    const ColState& s = st[q.seg];
    const T* r = AS_C(T, r_);
    T* p = AS(T, p_);
    const T* v = AS_C(T, v_);
    T rv[NE], pv[NE], vv[NE];
    SEG_LOOP((rv[j] = r[q.at(j)], pv[j] = p[q.at(j)], vv[j] = v[q.at(j)]),
             (p[q.at(j)] = rv[j] + scal(s.beta_re, s.beta_im, pv[j] - scal(s.omega_re, s.omega_im, vv[j]))))
}

// s = r - alpha v
template <typename R>
__global__ __launch_bounds__(kBlock) void k_bicg_s(Segs S, const cpx<R>* __restrict__ r_, const cpx<R>* __restrict__ v_,
                                                   cpx<R>* __restrict__ s_, const ColState* __restrict__ st) {
    LANE_SETUP(R);
    if (!st[q.seg].active) return;
    const ColState& s = st[q.seg];
    const T* r = AS_C(T, r_);
    const T* v = AS_C(T, v_);
    T* so = AS(T, s_);
    T rv[NE], vv[NE];
    SEG_LOOP((rv[j] = r[q.at(j)], vv[j] = v[q.at(j)]), (so[q.at(j)] = rv[j] - scal(s.alpha_re, s.alpha_im, vv[j])))
}

// x += alpha p + omega s; r = s - omega t; partials <r^, r>, |r|^2
template <typename R>
__global__ __launch_bounds__(kBlock) void k_bicg_xr(Segs S, cpx<R>* __restrict__ x_, cpx<R>* __restrict__ r_,
                                                    const cpx<R>* __restrict__ p_, const cpx<R>* __restrict__ s_,
                                                    const cpx<R>* __restrict__ t_, const cpx<R>* __restrict__ rh_,
                                                    double* __restrict__ partial, const ColState* __restrict__ st) {
    LANE_SETUP(R);
    if (!st[q.seg].active) return;  // uniform over the workgroup
    double d0 = 0, d1 = 0, d2 = 0;
    const ColState& s = st[q.seg];
    T* x = AS(T, x_);
    T* r = AS(T, r_);
    const T* p = AS_C(T, p_);
    const T* sv_ = AS_C(T, s_);
    const T* t = AS_C(T, t_);
    const T* rh = AS_C(T, rh_);
    T xv[NE], pv[NE], sv[NE], tv[NE], hv[NE];
    SEG_LOOP((xv[j] = x[q.at(j)], pv[j] = p[q.at(j)], sv[j] = sv_[q.at(j)], tv[j] = t[q.at(j)], hv[j] = rh[q.at(j)]),
             ({
                 x[q.at(j)] = xv[j] + scal(s.alpha_re, s.alpha_im, pv[j]) + scal(s.omega_re, s.omega_im, sv[j]);
                 const T rn = sv[j] - scal(s.omega_re, s.omega_im, tv[j]);
                 r[q.at(j)] = rn;
                 dot_acc(d0, d1, hv[j], rn);
                 norm_acc(d2, rn);
             }))
    block_sum3(d0, d1, d2, partial + (size_t)blockIdx.x * 3);
}

// CGNR: r -= alpha w; partial |r|^2 (alpha real)
template <typename R>
__global__ __launch_bounds__(kBlock) void k_cg_r(Segs S, cpx<R>* __restrict__ r_, const cpx<R>* __restrict__ w_,
                                                 double* __restrict__ partial, const ColState* __restrict__ st) {
    LANE_SETUP(R);
    if (!st[q.seg].active) return;
    double d0 = 0;
    const R a = R(st[q.seg].alpha_re);
    T* r = AS(T, r_);
    const T* w = AS_C(T, w_);
    T rv[NE], wv[NE];
    SEG_LOOP((rv[j] = r[q.at(j)], wv[j] = w[q.at(j)]),
             ({
                 const T rn = rv[j] - a * wv[j];
                 r[q.at(j)] = rn;
                 norm_acc(d0, rn);
             }))
    block_sum3(d0, 0.0, 0.0, partial + (size_t)blockIdx.x * 3);
}

// CGNR, the end of an iteration: x += alpha p while that update is due (also for a
// column that stopped in this iteration), then p = z + beta p for running columns
// (alpha, beta real).  The x update waits until here so that p is read once.
template <typename R>
__global__ __launch_bounds__(kBlock) void k_cg_px(Segs S, cpx<R>* __restrict__ x_, cpx<R>* __restrict__ p_,
                                                  const cpx<R>* __restrict__ z_, const ColState* __restrict__ st) {
    LANE_SETUP(R);
    const ColState& s = st[q.seg];
    const bool run = s.active != 0, due = s.xdue != 0;  // uniform over the workgroup
    if (!run && !due) return;
    const R a = R(s.alpha_re), b = R(s.beta_re);
    T* x = AS(T, x_);
    T* p = AS(T, p_);
    const T* z = AS_C(T, z_);
    T xv[NE], pv[NE], zv[NE];
    if (run) {
        SEG_LOOP((xv[j] = x[q.at(j)], pv[j] = p[q.at(j)], zv[j] = z[q.at(j)]),
                 (x[q.at(j)] = xv[j] + a * pv[j], p[q.at(j)] = zv[j] + b * pv[j]))
    } else {
        SEG_LOOP((xv[j] = x[q.at(j)], pv[j] = p[q.at(j)]), (x[q.at(j)] = xv[j] + a * pv[j]))
    }
}

// partial |a|^2 of every segment
template <typename R>
__global__ __launch_bounds__(kBlock) void k_norm2(Segs S, const cpx<R>* __restrict__ a_, double* __restrict__ partial) {
    LANE_SETUP(R);
    double d0 = 0;
    const T* a = AS_C(T, a_);
    T v[NE];
    SEG_LOOP((v[j] = a[q.at(j)]), norm_acc(d0, v[j]))
    block_sum3(d0, 0.0, 0.0, partial + (size_t)blockIdx.x * 3);
}

// b = a on the active segments
template <typename R>
__global__ __launch_bounds__(kBlock) void k_copy_segs(Segs S, const cpx<R>* __restrict__ a_, cpx<R>* __restrict__ b_,
                                                      const ColState* __restrict__ st) {
    LANE_SETUP(R);
    if (!st[q.seg].active) return;
    const T* a = AS_C(T, a_);
    T* b = AS(T, b_);
    T v[NE];
    SEG_LOOP((v[j] = a[q.at(j)]), (b[q.at(j)] = v[j]))
}

// Reliable-update helpers (segments selected by mask[seg] != 0):
//   x64 += xk; xk = 0        (xk in the Krylov precision)
//   rk = (Rk) r64            (replace the recursive residual by the true one)
// FP64 fields are [12][n] per segment; FP32 ones the same, or (S.paired) even-odd half
// fields with paired components, whose element 2 (q n + h) + e is component 2q + e of
// site h (n = len / 12 sites).
template <typename R>
__device__ inline size_t wide_index(const Segs& S, const SegPos<1>& q, int j) {
    const int u = q.i0 + j * kBlock;  // element within the segment
    if (sizeof(R) == 8 || !S.paired) return q.at(j);  // FP64 half fields are not paired
    const int n = S.len[q.seg] / 12;
    const int pu = u >> 1, e = u & 1;
    const int qq = pu / n, h = pu - qq * n;
    return (size_t)S.off[q.seg] + (size_t)(2 * qq + e) * n + h;
}
template <typename R>
__global__ __launch_bounds__(kBlock) void k_fold_x(Segs S, cpx<double>* __restrict__ x, cpx<R>* __restrict__ xk,
                                                   const int* __restrict__ mask) {
    LANE_SETUP(R);
    if (!mask[q.seg]) return;
    T e[NE];
    cpx<double> v[NE];
    size_t w[NE];
    SEG_LOOP((e[j] = xk[q.at(j)], w[j] = wide_index<R>(S, q, j), v[j] = x[w[j]]),
             (x[w[j]] = widen_add(v[j], e[j]), xk[q.at(j)] = zero_of(e[j])))
}
template <typename R>
__global__ __launch_bounds__(kBlock) void k_set_resid(Segs S, const cpx<double>* __restrict__ r64,
                                                      cpx<R>* __restrict__ rk, const int* __restrict__ mask) {
    LANE_SETUP(R);
    if (!mask[q.seg]) return;
    cpx<double> v[NE];
    SEG_LOOP((v[j] = r64[wide_index<R>(S, q, j)]), (rk[q.at(j)] = narrow<R>(v[j])))
}
// BiCGStab restart (mask == 2): fresh shadow residual r^ = r, directions cleared
template <typename R>
__global__ __launch_bounds__(kBlock) void k_restart_dirs(Segs S, const cpx<R>* __restrict__ r_, cpx<R>* __restrict__ rh_,
                                                         cpx<R>* __restrict__ p_, cpx<R>* __restrict__ v_,
                                                         const int* __restrict__ mask) {
    LANE_SETUP(R);
    if (mask[q.seg] != 2) return;
    const T* r = AS_C(T, r_);
    T* rh = AS(T, rh_);
    T* p = AS(T, p_);
    T* v = AS(T, v_);
    T w[NE];
    SEG_LOOP((w[j] = r[q.at(j)]), (rh[q.at(j)] = w[j], p[q.at(j)] = zero_of(w[j]), v[q.at(j)] = zero_of(w[j])))
}
// CGNR reliable update: p += t - z; z = t
template <typename R>
__global__ __launch_bounds__(kBlock) void k_cg_shift(Segs S, cpx<R>* __restrict__ p_, cpx<R>* __restrict__ z_,
                                                     const cpx<R>* __restrict__ t_, const int* __restrict__ mask) {
    LANE_SETUP(R);
    if (!mask[q.seg]) return;
    T* p = AS(T, p_);
    T* z = AS(T, z_);
    const T* t = AS_C(T, t_);
    T tv[NE], pv[NE], zv[NE];
    SEG_LOOP((tv[j] = t[q.at(j)], pv[j] = p[q.at(j)], zv[j] = z[q.at(j)]),
             (p[q.at(j)] = pv[j] + tv[j] - zv[j], z[q.at(j)] = tv[j]))
}

// a = 0 on the masked segments (a solve started from a guess whose source column is zero)
__global__ __launch_bounds__(kBlock) void k_zero_segs(Segs S, cpx<double>* __restrict__ a, const int* __restrict__ mask) {
    constexpr int NE = kElems;
    const SegPos<1> q = seg_pos<1>(S);
    if (!mask[q.seg]) return;
    SEG_LOOP((void)0, (a[q.at(j)] = cd(0.0, 0.0)))
}

// One workgroup per segment: fixed-order sum of the segment's partial slots
// [p0[seg], p0[seg+1]), then the scalar recurrences of BiCGStab / CG for it.
__global__ __launch_bounds__(kBlock) void k_finalize(int fin, const int* __restrict__ p0,
                                                     const double* __restrict__ partial, ColState* __restrict__ st,
                                                     double* __restrict__ out) {
    const int seg = blockIdx.x;
    if (fin != FIN_STORE && !st[seg].active) {
        // a stopped column: its last x update (if any) was applied by k_cg_px
        if (fin == FIN_CG_ALPHA && threadIdx.x == 0) st[seg].xdue = 0;
        return;
    }
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
            s.xdue = 0;  // the previous iteration's update was applied; due again once alpha is known
            if (!(d0 > 0) || !isfinite(d0)) {
                s.breakdown = isfinite(d0) ? 1 : 2;
                s.active = 0;
                break;
            }
            s.alpha_re = s.zz / d0;
            s.alpha_im = 0;
            s.xdue = 1;
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
#undef LANE_SETUP
#undef AS
#undef AS_C

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
void launch_cg_r(dd_ctx* c, const Segs& S, cpx<R>* r, const cpx<R>* w, double* partial, const ColState* st) {
    hipLaunchKernelGGL(k_cg_r<R>, sgrid(S), dim3(kBlock), 0, c->stream, S, r, w, partial, st);
}
template <typename R>
void launch_cg_px(dd_ctx* c, const Segs& S, cpx<R>* x, cpx<R>* p, const cpx<R>* z, const ColState* st) {
    hipLaunchKernelGGL(k_cg_px<R>, sgrid(S), dim3(kBlock), 0, c->stream, S, x, p, z, st);
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
    template void launch_cg_r<R>(dd_ctx*, const Segs&, cpx<R>*, const cpx<R>*, double*, const ColState*);       \
    template void launch_cg_px<R>(dd_ctx*, const Segs&, cpx<R>*, cpx<R>*, const cpx<R>*, const ColState*);     \
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
