// dd_wilson.h -- device helpers shared by the stencil, frontier and force kernels:
// spin projection / reconstruction in the chiral basis, one hop of the Wilson
// operator, and fixed-order wavefront / workgroup reductions.
#pragma once

#include "dd_internal.h"

namespace dd {


// h = upper two spin components of (1 + SGN gamma_MU) psi (chiral basis); the
// lower two are a fixed linear function of h, applied in accum().
template <typename R, int MU, int SGN>
__device__ __forceinline__ void project(const cpx<R> (&p)[12], cpx<R> (&h)[6]) {
#pragma unroll
    for (int c = 0; c < 3; c++) {
        const cpx<R> p0 = p[c], p1 = p[3 + c], p2 = p[6 + c], p3 = p[9 + c];
        if (MU == 0) {        // gamma_0 = [[0,-1],[-1,0]]
            h[c] = SGN > 0 ? p0 - p2 : p0 + p2;
            h[3 + c] = SGN > 0 ? p1 - p3 : p1 + p3;
        } else if (MU == 1) { // gamma_1 = [[0,-i s1],[i s1,0]]
            h[c] = SGN > 0 ? p0 - imul(p3) : p0 + imul(p3);
            h[3 + c] = SGN > 0 ? p1 - imul(p2) : p1 + imul(p2);
        } else if (MU == 2) { // gamma_2 = [[0,-i s2],[i s2,0]]
            h[c] = SGN > 0 ? p0 - p3 : p0 + p3;
            h[3 + c] = SGN > 0 ? p1 + p2 : p1 - p2;
        } else {              // gamma_3 = [[0,-i s3],[i s3,0]]
            h[c] = SGN > 0 ? p0 - imul(p2) : p0 + imul(p2);
            h[3 + c] = SGN > 0 ? p1 + imul(p3) : p1 - imul(p3);
        }
    }
}

// a += (1 + SGN gamma_MU)-reconstructed spinor from the transported half spinor u.
template <typename R, int MU, int SGN>
__device__ __forceinline__ void accum(cpx<R> (&a)[12], const cpx<R> (&u)[6]) {
#pragma unroll
    for (int c = 0; c < 3; c++) {
        const cpx<R> u0 = u[c], u1 = u[3 + c];
        a[c] = a[c] + u0;
        a[3 + c] = a[3 + c] + u1;
        if (MU == 0) {
            a[6 + c] = SGN > 0 ? a[6 + c] - u0 : a[6 + c] + u0;
            a[9 + c] = SGN > 0 ? a[9 + c] - u1 : a[9 + c] + u1;
        } else if (MU == 1) {
            a[6 + c] = SGN > 0 ? a[6 + c] + imul(u1) : a[6 + c] - imul(u1);
            a[9 + c] = SGN > 0 ? a[9 + c] + imul(u0) : a[9 + c] - imul(u0);
        } else if (MU == 2) {
            a[6 + c] = SGN > 0 ? a[6 + c] + u1 : a[6 + c] - u1;
            a[9 + c] = SGN > 0 ? a[9 + c] - u0 : a[9 + c] + u0;
        } else {
            a[6 + c] = SGN > 0 ? a[6 + c] + imul(u0) : a[6 + c] - imul(u0);
            a[9 + c] = SGN > 0 ? a[9 + c] - imul(u1) : a[9 + c] + imul(u1);
        }
    }
}

template <typename R>
__device__ __forceinline__ void load_spinor(const cpx<R>* __restrict__ f, int nsite, int s,
                                            cpx<R> (&p)[12]) {
#pragma unroll
    for (int c = 0; c < 12; c++) p[c] = f[c * nsite + s];
}

// One hop: a += (1 + SGN gamma_MU) W psi(nb) * ph, W = U (fwd) or U^+ (bwd).
template <typename R, int MU, int SGN, bool BWD>
__device__ __forceinline__ void hop(cpx<R> (&a)[12], const cpx<R>* __restrict__ f, int nsite, int nb,
                                    const cpx<R>* __restrict__ U, int vlink, int sl, R ph) {
    cpx<R> p[12];
    load_spinor(f, nsite, nb, p);
    cpx<R> h[6];
    project<R, MU, SGN>(p, h);
    cpx<R> w[9];
    const cpx<R>* u = U + (size_t)(MU * 9) * vlink + sl;
#pragma unroll
    for (int k = 0; k < 9; k++) w[k] = u[(size_t)k * vlink];
    cpx<R> t[6];
#pragma unroll
    for (int hs = 0; hs < 2; hs++)
#pragma unroll
        for (int i = 0; i < 3; i++) {
            cpx<R> acc;
            if (!BWD) {
                acc = w[3 * i + 0] * h[3 * hs + 0];
                acc = acc + w[3 * i + 1] * h[3 * hs + 1];
                acc = acc + w[3 * i + 2] * h[3 * hs + 2];
            } else {
                acc = cmulc(w[0 * 3 + i], h[3 * hs + 0]);
                acc = acc + cmulc(w[1 * 3 + i], h[3 * hs + 1]);
                acc = acc + cmulc(w[2 * 3 + i], h[3 * hs + 2]);
            }
            t[3 * hs + i] = ph * acc;
        }
    accum<R, MU, SGN>(a, t);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// Fixed-order block reduction of three doubles; thread k < 3 writes out[k].
__device__ __forceinline__ void block_sum3(double d0, double d1, double d2, double* __restrict__ out) {
    __shared__ double sh[kBlock / kWave][3];
    d0 = wave_sum(d0);
    d1 = wave_sum(d1);
    d2 = wave_sum(d2);
    const int w = threadIdx.x / kWave, l = threadIdx.x % kWave;
    if (l == 0) {
        sh[w][0] = d0;
        sh[w][1] = d1;
        sh[w][2] = d2;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        double s = 0;
#pragma unroll
        for (int k = 0; k < kBlock / kWave; k++) s += sh[k][threadIdx.x];
        out[threadIdx.x] = s;
    }
}

}  // namespace dd
