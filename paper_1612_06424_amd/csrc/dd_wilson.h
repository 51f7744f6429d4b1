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

// Element `idx` of an array whose base is wave-uniform: the byte offset is a
// 32-bit unsigned value, so the compiler addresses with an SGPR base plus one
// VGPR offset (global_load ... saddr) instead of a 64-bit VGPR address per load.
// Valid while idx * sizeof(T) < 2^32 (a field component or link row is < 4 GiB).
// Plain element access (kernels off the hot path).
template <typename R>
__device__ __forceinline__ void load_spinor(const cpx<R>* __restrict__ f, int nsite, int s,
                                            cpx<R> (&p)[12]) {
#pragma unroll
    for (int c = 0; c < 12; c++) p[c] = f[(size_t)c * nsite + s];
}

// ---------------------------------------------------------------- buffer access
// The stencil addresses memory through raw buffer resources: the resource
// (base, size) and the component / link-row stride sit in scalar registers, so
// all loads of one site share a single 32-bit VGPR offset, and any offset past
// the resource reads 0 / drops the store instead of touching other memory.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef __amdgpu_buffer_rsrc_t rsrc_t;

// dword3 of a raw (untyped, stride 0) buffer resource on gfx9-family GPUs
constexpr int kRsrcWord3 = 0x00020000;

__device__ __forceinline__ rsrc_t make_rsrc(const void* base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, kRsrcWord3);
}

template <typename R>
__device__ __forceinline__ cpx<R> bload(rsrc_t r, uint32_t voff, uint32_t soff);
template <>
__device__ __forceinline__ cpx<double> bload<double>(rsrc_t r, uint32_t voff, uint32_t soff) {
    return __builtin_bit_cast(cpx<double>, __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, (int)soff, 0));
}
template <>
__device__ __forceinline__ cpx<float> bload<float>(rsrc_t r, uint32_t voff, uint32_t soff) {
    return __builtin_bit_cast(cpx<float>, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0));
}
template <typename R>
__device__ __forceinline__ void bstore(rsrc_t r, uint32_t voff, uint32_t soff, cpx<R> v);
template <>
__device__ __forceinline__ void bstore<double>(rsrc_t r, uint32_t voff, uint32_t soff, cpx<double> v) {
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, v), r, (int)voff, (int)soff, 0);
}
template <>
__device__ __forceinline__ void bstore<float>(rsrc_t r, uint32_t voff, uint32_t soff, cpx<float> v) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, (int)voff, (int)soff, 0);
}
// The same stores marked non-temporal (cache-policy bit nt), for outputs the launch
// does not read again.
template <typename R>
__device__ __forceinline__ void bstore_nt(rsrc_t r, uint32_t voff, uint32_t soff, cpx<R> v);
template <>
__device__ __forceinline__ void bstore_nt<double>(rsrc_t r, uint32_t voff, uint32_t soff, cpx<double> v) {
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, v), r, (int)voff, (int)soff, 2);
}
template <>
__device__ __forceinline__ void bstore_nt<float>(rsrc_t r, uint32_t voff, uint32_t soff, cpx<float> v) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, (int)voff, (int)soff, 2);
}

// spinor of local site s from a field resource with component stride cs (bytes)
template <typename R>
__device__ __forceinline__ void bload_spinor(rsrc_t f, uint32_t cs, int s, cpx<R> (&p)[12]) {
    const uint32_t vo = (uint32_t)s * (uint32_t)sizeof(cpx<R>);
#pragma unroll
    for (int c = 0; c < 12; c++) p[c] = bload<R>(f, vo, (uint32_t)c * cs);
}

// t = ph * W h for the two colour vectors of a half spinor, W = U or U^+.
template <typename R, bool BWD>
__device__ __forceinline__ void transport(const cpx<R> (&w)[9], const cpx<R> (&h)[6], R ph, cpx<R> (&t)[6]) {
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
}

// One hop through buffer resources: a += ph (1 + SGN gamma_MU) W psi(nb),
// W = U_MU(sl) (fwd) or its adjoint (bwd); u is the resource of direction MU's
// nine link rows (row stride ls bytes).
template <typename R, int MU, int SGN, bool BWD>
__device__ __forceinline__ void bhop(cpx<R> (&a)[12], rsrc_t f, uint32_t cs, int nb, rsrc_t u, uint32_t ls,
                                     int sl, R ph) {
    cpx<R> p[12];
    bload_spinor<R>(f, cs, nb, p);
    cpx<R> h[6];
    project<R, MU, SGN>(p, h);
    cpx<R> w[9];
    const uint32_t vo = (uint32_t)sl * (uint32_t)sizeof(cpx<R>);
#pragma unroll
    for (int k = 0; k < 9; k++) w[k] = bload<R>(u, vo, (uint32_t)k * ls);
    cpx<R> t[6];
    transport<R, BWD>(w, h, ph, t);
    accum<R, MU, SGN>(a, t);
}

// The same hop with plain pointers (frontier kernel).
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
    transport<R, BWD>(w, h, ph, t);
    accum<R, MU, SGN>(a, t);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// Fixed-order block reduction of three doubles over NT threads; thread k < 3
// writes out[k].
template <int NT = kBlock>
__device__ __forceinline__ void block_sum3(double d0, double d1, double d2, double* __restrict__ out) {
    __shared__ double sh[NT / kWave][3];
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
        for (int k = 0; k < NT / kWave; k++) s += sh[k][threadIdx.x];
        out[threadIdx.x] = s;
    }
}

}  // namespace dd
