// dd_eo.h -- even-odd (checkerboard) pieces of the Wilson-Dirac operator.
//
// With D = m - 1/2 H (m = 1/(2 kappa), H the hopping term of Sec. 5) and H
// connecting only sites of opposite parity (t + x + y + z mod 2, local time),
// D x = b is equivalent to the even-site Schur complement system
//     Dhat x_e = b_e + (1/(2m)) H_eo b_o,   Dhat = m - (1/(4m)) H_eo H_oe,
// followed by x_o = (b_o + 1/2 H_oe x_e) / m; the residual of the full system
// is the Schur residual on the even sites and zero on the odd ones.  This
// needs a bipartite lattice: L even, and T even unless the field is a slab.
//
// Half fields: [col][12][nsite / 2]; the site with local index s lives at
// s >> 1 of the half field of its parity (L even makes s and s ^ 1 a pair of
// opposite parity).  Links are reordered the same way, local to the field:
// Ueo[mu][k][parity][nsite / 2] holds U_mu(x)_k of the field site x, so every
// link load of a wavefront reads consecutive elements.  A hop leaving a slab
// is dropped, so no link outside the field is needed.  The kernels compute
//     out = a_self * self + c_hop * (H in)_site      (in: the other parity)
// (SELF = false: no self term, the pure hop) with the fused epilogues of the
// full stencil (dd_dslash.h).
#pragma once

#include "dd_internal.h"
#include "dd_wilson.h"

namespace dd {

// Spinor of site nb in column k of a group of columns stored back to back
// (column stride fs bytes, component stride cs bytes).
template <typename R>
__device__ __forceinline__ void bload_spinor_col(rsrc_t f, uint32_t cs, uint32_t col_off, int nb,
                                                 cpx<R> (&p)[12]) {
    const uint32_t vo = (uint32_t)nb * (uint32_t)sizeof(cpx<R>);
#pragma unroll
    for (int c = 0; c < 12; c++) p[c] = bload<R>(f, vo, col_off + (uint32_t)c * cs);
}

// FP32 half fields of the even-odd solves keep their spin-colour components in pairs:
// the 16-byte unit (c / 2) nh + h of a column holds components c & ~1 and c | 1 of half
// site h.  FP64 half fields keep [12][nh] (one component is 16 bytes already).  Either
// way every lane access is 16 bytes; a column is 12 cs bytes (cs = nh sizeof(cpx<R>)).
typedef float f32x4v __attribute__((ext_vector_type(4)));
template <typename R>
__device__ __forceinline__ void hload_spinor(rsrc_t f, uint32_t cs, uint32_t col_off, int h, cpx<R> (&p)[12]) {
    if constexpr (sizeof(R) == 8) {
        bload_spinor_col<R>(f, cs, col_off, h, p);
    } else {
        const uint32_t vo = (uint32_t)h * 16u;
#pragma unroll
        for (int q = 0; q < 6; q++) {
            // the whole vector is bit-cast at once (element by element it was lowered to one 4-byte load)
            const f32x4v v =
                __builtin_bit_cast(f32x4v, __builtin_amdgcn_raw_buffer_load_b128(f, (int)vo, (int)(col_off + q * 2u * cs), 0));
            p[2 * q] = cpx<R>{v.x, v.y};
            p[2 * q + 1] = cpx<R>{v.z, v.w};
        }
    }
}
// components 2q and 2q + 1 of half site h
template <typename R>
__device__ __forceinline__ void hload_pair(rsrc_t f, uint32_t cs, uint32_t col_off, int h, int q, cpx<R>& a,
                                           cpx<R>& b) {
    if constexpr (sizeof(R) == 8) {
        const uint32_t vo = (uint32_t)h * (uint32_t)sizeof(cpx<R>);
        a = bload<R>(f, vo, col_off + (uint32_t)(2 * q) * cs);
        b = bload<R>(f, vo, col_off + (uint32_t)(2 * q + 1) * cs);
    } else {
        const f32x4v v = __builtin_bit_cast(
            f32x4v, __builtin_amdgcn_raw_buffer_load_b128(f, (int)((uint32_t)h * 16u), (int)(col_off + (uint32_t)q * 2u * cs), 0));
        a = cpx<R>{v.x, v.y};
        b = cpx<R>{v.z, v.w};
    }
}
template <typename R, bool NTS>
__device__ __forceinline__ void hstore_pair(rsrc_t f, uint32_t cs, uint32_t col_off, int h, int q, cpx<R> a,
                                            cpx<R> b) {
    if constexpr (sizeof(R) == 8) {
        const uint32_t vo = (uint32_t)h * (uint32_t)sizeof(cpx<R>);
        if constexpr (NTS) {
            bstore_nt<R>(f, vo, col_off + (uint32_t)(2 * q) * cs, a);
            bstore_nt<R>(f, vo, col_off + (uint32_t)(2 * q + 1) * cs, b);
        } else {
            bstore<R>(f, vo, col_off + (uint32_t)(2 * q) * cs, a);
            bstore<R>(f, vo, col_off + (uint32_t)(2 * q + 1) * cs, b);
        }
    } else {
        // two 8-byte stores per unit: with one 16-byte store, whose data registers the next
        // unit's arithmetic overwrites at once, groups of four lanes stored the next unit's
        // low half on this hardware (found on the 64x32^3 fields; the 8-byte form is exact)
        // the second half's 8 bytes go into the scalar offset, so the two stores are not fused
        const uint32_t vo = (uint32_t)h * 16u, so = col_off + (uint32_t)q * 2u * cs;
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, a), f, (int)vo, (int)so, NTS ? 2 : 0);
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, b), f, (int)vo, (int)(so + 8u), NTS ? 2 : 0);
    }
}

// The nine entries of the link at half-site index sl of one (mu, parity) block.
template <typename R>
__device__ __forceinline__ void bload_link(rsrc_t u, uint32_t ls, int sl, cpx<R> (&w)[9]) {
    const uint32_t vo = (uint32_t)sl * (uint32_t)sizeof(cpx<R>);
#pragma unroll
    for (int k = 0; k < 9; k++) w[k] = bload<R>(u, vo, (uint32_t)k * ls);
}

// The same link from its first two rows (REC: links stored as 12 reals).  An
// SU(3) matrix is unitary with unit determinant, so its third row is the
// complex conjugate of the cross product of the first two.
// FP32 two-row links pair their entries as the FP32 half fields do: Ueo12[mu][k / 2]
// [parity][nsite / 2][k & 1], so that the 16-byte unit (mu, kp, parity, h) holds entries
// 2 kp and 2 kp + 1; the resource of one (mu, parity) block starts at unit (6 mu + parity)
// nh (rec_link_base) and a row of units is 2 ls bytes apart (ls = 2 nh sizeof(cpx<float>)).
__device__ __forceinline__ size_t rec_link_base(int mu, int parity, int nh) {
    return ((size_t)(6 * mu + parity) * (size_t)nh) * 2;  // in cpx<float>
}
template <typename R, bool REC>
__device__ __forceinline__ void bload_link_r(rsrc_t u, uint32_t ls, int sl, cpx<R> (&w)[9]) {
    if constexpr (!REC) {
        bload_link<R>(u, ls, sl, w);
    } else {
        if constexpr (sizeof(R) == 4) {
            const uint32_t vo = (uint32_t)sl * 16u;
#pragma unroll
            for (int kp = 0; kp < 3; kp++) {
                const f32x4v v = __builtin_bit_cast(
                    f32x4v, __builtin_amdgcn_raw_buffer_load_b128(u, (int)vo, (int)((uint32_t)kp * 2u * ls), 0));
                w[2 * kp] = cpx<R>{v.x, v.y};
                w[2 * kp + 1] = cpx<R>{v.z, v.w};
            }
        } else {
            const uint32_t vo = (uint32_t)sl * (uint32_t)sizeof(cpx<R>);
#pragma unroll
            for (int k = 0; k < 6; k++) w[k] = bload<R>(u, vo, (uint32_t)k * ls);
        }
        const cpx<R> c6 = w[1] * w[5] - w[2] * w[4];
        const cpx<R> c7 = w[2] * w[3] - w[0] * w[5];
        const cpx<R> c8 = w[0] * w[4] - w[1] * w[3];
        w[6] = mk<R>(c6.re, -c6.im);
        w[7] = mk<R>(c7.re, -c7.im);
        w[8] = mk<R>(c8.re, -c8.im);
    }
}

// One spatial hop for KC columns: the link is loaded once and transports the
// projected neighbour of every column.
// HALF: f is an even-odd half field (paired components in FP32), else a full field.
template <typename R, int MU, int SGN, bool BWD, int KC, bool REC, bool HALF = false>
__device__ __forceinline__ void bhop_cols(cpx<R> (&a)[KC][12], rsrc_t f, uint32_t cs, uint32_t fs, int nb, rsrc_t u,
                                          uint32_t ls, int sl) {
    cpx<R> w[9];
    bload_link_r<R, REC>(u, ls, sl, w);
#pragma unroll
    for (int k = 0; k < KC; k++) {
        cpx<R> p[12];
        if constexpr (HALF) hload_spinor<R>(f, cs, (uint32_t)k * fs, nb, p);
        else bload_spinor_col<R>(f, cs, (uint32_t)k * fs, nb, p);
        cpx<R> h[6];
        project<R, MU, SGN>(p, h);
        cpx<R> t[6];
        transport<R, BWD>(w, h, R(1), t);
        accum<R, MU, SGN>(a[k], t);
    }
}

// One hop of a half field (one column): a += (1 + SGN gamma_MU) W psi(nb).
template <typename R, int MU, int SGN, bool BWD>
__device__ __forceinline__ void bhop_half(cpx<R> (&a)[12], rsrc_t f, uint32_t cs, int nb, rsrc_t u, uint32_t ls,
                                          int sl) {
    cpx<R> p[12];
    hload_spinor<R>(f, cs, 0u, nb, p);
    cpx<R> h[6];
    project<R, MU, SGN>(p, h);
    cpx<R> w[9];
    const uint32_t vo = (uint32_t)sl * (uint32_t)sizeof(cpx<R>);
#pragma unroll
    for (int k = 0; k < 9; k++) w[k] = bload<R>(u, vo, (uint32_t)k * ls);
    cpx<R> t[6];
    transport<R, BWD>(w, h, R(1), t);
    accum<R, MU, SGN>(a, t);
}

// Workgroup sums of three partial values per column; column k's sums go to
// slot + 3 k col_stride.
template <int NT, int KC>
__device__ __forceinline__ void block_sum_cols(double (&d)[KC][3], double* __restrict__ slot, size_t col_stride) {
    __shared__ double sh[NT / kWave][KC * 3];
    const int w = threadIdx.x / kWave, l = threadIdx.x % kWave;
#pragma unroll
    for (int k = 0; k < KC; k++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            const double v = wave_sum(d[k][j]);
            if (l == 0) sh[w][k * 3 + j] = v;
        }
    __syncthreads();
    if (threadIdx.x < KC * 3) {
        double s = 0;
#pragma unroll
        for (int q = 0; q < NT / kWave; q++) s += sh[q][threadIdx.x];
        const int k = threadIdx.x / 3, j = threadIdx.x % 3;
        slot[(size_t)k * col_stride * 3 + j] = s;
    }
}

// Pair index pr of a slice -> (xh, y, z).  Rows: NT consecutive pairs fill
// whole x rows of one z plane after another.  Blocked (L a multiple of 4): the
// (y, z) plane is cut into 4 x 4 blocks of full x rows, so a tile of NT pairs is
// a compact brick and its y and z neighbours mostly lie inside it; a wavefront
// still reads 4 consecutive rows (contiguous memory).
__device__ __forceinline__ void pair_site(int pr, int Lh, int L, int blocked, int& xh, int& y, int& z) {
    if (blocked) {
        const int per = Lh * 16;
        const int b = pr / per, r = pr - b * per;
        const int q = r / Lh, nby = L >> 2;
        xh = r - q * Lh;
        y = (b % nby) * 4 + (q & 3);
        z = (b / nby) * 4 + (q >> 2);
    } else {
        const int yz = pr / Lh;
        xh = pr - yz * Lh;
        y = yz % L;
        z = yz / L;
    }
}

// Time-sweep form of the half hop.  A thread owns one pair (xh, y, z) of
// every slice and walks a chunk of tc_len slices; at slice t its output site is
// x = 2 xh + b(t), with b alternating from slice to slice.  The forward time
// neighbour loaded at slice t, (x(t), t + 1), is the backward time neighbour of
// the output at slice t + 2 (same x), so its projected half spinor is carried
// two steps and every input site of the chunk is loaded once in time
// direction.  tile: NT consecutive pair indices of a slice (pair_site).
template <typename R, int DAG, int EPI, int NT, bool SELF>
__device__ __forceinline__ void eo_sweep_tile(const Geo& g, const cpx<R>* __restrict__ Ueo, R a_self, R c_hop,
                                              int p_out, const cpx<R>* __restrict__ in,
                                              const cpx<R>* __restrict__ self, cpx<R>* __restrict__ out,
                                              const cpx<R>* __restrict__ aux, int tile, int chunk, int tc_len,
                                              int blocked, double* __restrict__ slot) {
    const int L = g.L, L2 = g.L2, L3 = g.L3;
    const int nh = g.nsite >> 1;
    const int Lh = L >> 1, L3h = L3 >> 1;
    constexpr uint32_t CB = sizeof(cpx<R>);
    const uint32_t cs = (uint32_t)nh * CB;
    const uint32_t ls = 2u * (uint32_t)nh * CB;
    const uint32_t ubytes = 17u * (uint32_t)nh * CB;
    constexpr int FW = DAG ? +1 : -1;
    constexpr int BW = -FW;
    constexpr bool has_self = SELF || EPI == EPI_TS;
    double d0 = 0, d1 = 0, d2 = 0;
    const int pr = tile * NT + (int)threadIdx.x;  // pair index within a slice
    if (pr < L3h) {
        int xh, y, z;
        pair_site(pr, Lh, L, blocked, xh, y, z);
        const int yz = z * L + y;
        const int nt = g.nt;
        const int tb = chunk * tc_len;
        const int te = min(nt, tb + tc_len);
        auto tglob = [&](int tl) {
            const int t = g.t0 + tl;
            return t >= g.T ? t - g.T : t;
        };
        auto xof = [&](int tl) { return 2 * xh + ((p_out + tl + y + z) & 1); };
        const rsrc_t rf = make_rsrc(in, 12u * cs);
        const rsrc_t ro = make_rsrc(out, 12u * cs);
        const rsrc_t rs = make_rsrc(self != nullptr ? self : in, 12u * cs);
        const rsrc_t rx = make_rsrc(aux != nullptr ? aux : in, 12u * cs);
        rsrc_t uf[4], ub[4];
#pragma unroll
        for (int mu = 0; mu < 4; mu++) {
            uf[mu] = make_rsrc(Ueo + (size_t)(mu * 18 + p_out) * nh, ubytes);
            ub[mu] = make_rsrc(Ueo + (size_t)(mu * 18 + 1 - p_out) * nh, ubytes);
        }
        const int dyp = (y == L - 1) ? -(L - 1) * L : L, dym = (y == 0) ? (L - 1) * L : -L;
        const int dzp = (z == L - 1) ? -(L - 1) * L2 : L2, dzm = (z == 0) ? (L - 1) * L2 : -L2;
        // projected backward neighbours for the first two slices of the chunk:
        // slot cA serves slice tl, cB slice tl + 1
        cpx<R> cA[6], cB[6];
#pragma unroll
        for (int k = 0; k < 6; k++) cA[k] = cB[k] = mk<R>(0, 0);
        auto load_bw = [&](int tl, cpx<R> (&h)[6]) {
            // P psi_in(x(tl), tl - 1), or 0 where there is no backward time hop
            if (tl < nt && (tl > 0 || g.whole)) {
                const int tm = tl > 0 ? tl - 1 : nt - 1;
                cpx<R> p[12];
                hload_spinor<R>(rf, cs, 0u, (tm * L3 + yz * L + xof(tl)) >> 1, p);
                project<R, 0, BW>(p, h);
            }
        };
        if (tb < te) load_bw(tb, cA);
        if (tb + 1 < te) load_bw(tb + 1, cB);
#pragma unroll 1
        for (int tl = tb; tl < te; tl++) {
            const int x = xof(tl);
            const int sp = yz * L + x;
            const int s = tl * L3 + sp;
            const int h = s >> 1;
            const int tg = tglob(tl);
            cpx<R> a[12];
#pragma unroll
            for (int c = 0; c < 12; c++) a[c] = mk<R>(0, 0);
            // backward time hop from the carried half spinor, link U_0(x, tl - 1) on the input parity
            if (tl > 0 || g.whole) {
                const R ph = (tg == 0) ? R(g.bc) : R(1);
                if (ph != R(0)) {
                    const int hm = ((tl > 0 ? tl - 1 : nt - 1) * L3 + sp) >> 1;
                    cpx<R> w[9];
                    const uint32_t vo = (uint32_t)hm * CB;
#pragma unroll
                    for (int k = 0; k < 9; k++) w[k] = bload<R>(ub[0], vo, (uint32_t)k * ls);
                    cpx<R> t[6];
                    transport<R, true>(w, cA, ph, t);
                    accum<R, 0, BW>(a, t);
                }
            }
            // forward time hop; the loaded spinor is also the backward neighbour of slice tl + 2
            cpx<R> nb2[6];
#pragma unroll
            for (int k = 0; k < 6; k++) nb2[k] = mk<R>(0, 0);
            const bool endt = (tl == nt - 1);
            if (!endt || g.whole) {
                cpx<R> p[12];
                hload_spinor<R>(rf, cs, 0u, (endt ? sp : s + L3) >> 1, p);
                const R ph = (tg == g.T - 1) ? R(g.bc) : R(1);
                if (ph != R(0)) {
                    cpx<R> hf[6];
                    project<R, 0, FW>(p, hf);
                    cpx<R> w[9];
                    const uint32_t vo = (uint32_t)h * CB;
#pragma unroll
                    for (int k = 0; k < 9; k++) w[k] = bload<R>(uf[0], vo, (uint32_t)k * ls);
                    cpx<R> t[6];
                    transport<R, false>(w, hf, ph, t);
                    accum<R, 0, FW>(a, t);
                }
                if (!endt) project<R, 0, BW>(p, nb2);
            }
            const int dxp = (x == L - 1) ? -(L - 1) : 1, dxm = (x == 0) ? (L - 1) : -1;
            bhop_half<R, 1, FW, false>(a, rf, cs, (s + dxp) >> 1, uf[1], ls, h);
            bhop_half<R, 1, BW, true>(a, rf, cs, (s + dxm) >> 1, ub[1], ls, (s + dxm) >> 1);
            bhop_half<R, 2, FW, false>(a, rf, cs, (s + dyp) >> 1, uf[2], ls, h);
            bhop_half<R, 2, BW, true>(a, rf, cs, (s + dym) >> 1, ub[2], ls, (s + dym) >> 1);
            bhop_half<R, 3, FW, false>(a, rf, cs, (s + dzp) >> 1, uf[3], ls, h);
            bhop_half<R, 3, BW, true>(a, rf, cs, (s + dzm) >> 1, ub[3], ls, (s + dzm) >> 1);

#pragma unroll
            for (int qq = 0; qq < 6; qq++) {
                cpx<R> pc2[2] = {mk<R>(0, 0), mk<R>(0, 0)}, q2[2] = {mk<R>(0, 0), mk<R>(0, 0)}, r2[2];
                if (has_self) hload_pair<R>(rs, cs, 0u, h, qq, pc2[0], pc2[1]);
                if (EPI == EPI_RESID || EPI == EPI_DOT_AUX) hload_pair<R>(rx, cs, 0u, h, qq, q2[0], q2[1]);
#pragma unroll
                for (int e = 0; e < 2; e++) {
                    const int c = 2 * qq + e;
                    const cpx<R> pc = pc2[e], q = q2[e];
                    cpx<R> r = mk<R>(a_self * pc.re + c_hop * a[c].re, a_self * pc.im + c_hop * a[c].im);
                    if (EPI == EPI_RESID) r = q - r;
                    r2[e] = r;
                    if (EPI == EPI_DOT_AUX) {
                        d0 += (double)q.re * r.re + (double)q.im * r.im;
                        d1 += (double)q.re * r.im - (double)q.im * r.re;
                    } else if (EPI == EPI_TS) {
                        d0 += (double)r.re * pc.re + (double)r.im * pc.im;
                        d1 += (double)r.re * pc.im - (double)r.im * pc.re;
                        d2 += (double)r.re * r.re + (double)r.im * r.im;
                    } else if (EPI == EPI_RESID || EPI == EPI_NORM) {
                        d0 += (double)r.re * r.re + (double)r.im * r.im;
                    }
                }
                hstore_pair<R, false>(ro, cs, 0u, h, qq, r2[0], r2[1]);
            }
            // slice tl + 1 uses cB; slice tl + 2 the half spinor just loaded
#pragma unroll
            for (int k = 0; k < 6; k++) {
                cA[k] = cB[k];
                cB[k] = nb2[k];
            }
        }
    }
    if (EPI != EPI_STORE) block_sum3<NT>(d0, d1, d2, slot);
}


// The same sweep for KC > 1 columns stored back to back from in / self / out
// / aux (12 nsite/2 entries each): every link is loaded once for all of them;
// the sums of column k go to slot + 3 k slot_col.  Column k's output is
// written only if bit k of live is set (a stopped column keeps its vectors):
// its stores go through a buffer resource of size 0 otherwise, which drops
// them without a branch.  REC: Ueo holds only the first two rows of every link
// (Ueo12, in FP32 with its entries paired, see rec_link_base) and the third is
// rebuilt (bload_link_r).
// NTS: the output stores are non-temporal.
template <typename R, int DAG, int EPI, int NT, bool SELF, int KC, bool REC, bool NTS = false>
__device__ __forceinline__ void eo_sweep_cols(const Geo& g, const cpx<R>* __restrict__ Ueo, R a_self, R c_hop,
                                              int p_out, const cpx<R>* __restrict__ in,
                                              const cpx<R>* __restrict__ self, cpx<R>* __restrict__ out,
                                              const cpx<R>* __restrict__ aux, unsigned live, int tile, int chunk,
                                              int tc_len, int blocked, double* __restrict__ slot, size_t slot_col) {
    const int L = g.L, L2 = g.L2, L3 = g.L3;
    const int nh = g.nsite >> 1;
    const int Lh = L >> 1, L3h = L3 >> 1;
    constexpr uint32_t CB = sizeof(cpx<R>);
    const uint32_t cs = (uint32_t)nh * CB;
    const uint32_t fs = 12u * cs;  // column stride (bytes)
    const uint32_t ls = 2u * (uint32_t)nh * CB;
    constexpr int NROW = REC ? 6 : 9;  // stored rows of a link
    constexpr bool PAIRED_LINKS = REC && sizeof(R) == 4;  // two-row FP32 links in 16-byte units
    const uint32_t ubytes = PAIRED_LINKS ? 5u * (uint32_t)nh * 16u : (uint32_t)(2 * NROW - 1) * (uint32_t)nh * CB;
    constexpr int FW = DAG ? +1 : -1;
    constexpr int BW = -FW;
    constexpr bool has_self = SELF || EPI == EPI_TS;
    double d[KC][3];
#pragma unroll
    for (int k = 0; k < KC; k++) d[k][0] = d[k][1] = d[k][2] = 0;
    const int pr = tile * NT + (int)threadIdx.x;  // pair index within a slice
    if (pr < L3h) {
        int xh, y, z;
        pair_site(pr, Lh, L, blocked, xh, y, z);
        const int yz = z * L + y;
        const int nt = g.nt;
        const int tb = chunk * tc_len;
        const int te = min(nt, tb + tc_len);
        auto tglob = [&](int tl) {
            const int t = g.t0 + tl;
            return t >= g.T ? t - g.T : t;
        };
        auto xof = [&](int tl) { return 2 * xh + ((p_out + tl + y + z) & 1); };
        const rsrc_t rf = make_rsrc(in, (uint32_t)KC * fs);
        rsrc_t ro[KC];
#pragma unroll
        for (int k = 0; k < KC; k++) ro[k] = make_rsrc(out + (size_t)k * 12 * nh, ((live >> k) & 1u) ? fs : 0u);
        const rsrc_t rs = make_rsrc(self != nullptr ? self : in, (uint32_t)KC * fs);
        const rsrc_t rx = make_rsrc(aux != nullptr ? aux : in, (uint32_t)KC * fs);
        rsrc_t uf[4], ub[4];
#pragma unroll
        for (int mu = 0; mu < 4; mu++) {
            uf[mu] = make_rsrc(Ueo + (PAIRED_LINKS ? rec_link_base(mu, p_out, nh) : (size_t)(mu * 2 * NROW + p_out) * nh),
                               ubytes);
            ub[mu] = make_rsrc(
                Ueo + (PAIRED_LINKS ? rec_link_base(mu, 1 - p_out, nh) : (size_t)(mu * 2 * NROW + 1 - p_out) * nh), ubytes);
        }
        const int dyp = (y == L - 1) ? -(L - 1) * L : L, dym = (y == 0) ? (L - 1) * L : -L;
        const int dzp = (z == L - 1) ? -(L - 1) * L2 : L2, dzm = (z == 0) ? (L - 1) * L2 : -L2;
        // projected backward neighbours for the first two slices of the chunk:
        // slot cA serves slice tl, cB slice tl + 1
        cpx<R> cA[KC][6], cB[KC][6];
#pragma unroll
        for (int k = 0; k < KC; k++)
#pragma unroll
            for (int j = 0; j < 6; j++) cA[k][j] = cB[k][j] = mk<R>(0, 0);
        auto load_bw = [&](int tl, cpx<R> (&h)[KC][6]) {
            // P psi_in(x(tl), tl - 1), or 0 where there is no backward time hop
            if (tl < nt && (tl > 0 || g.whole)) {
                const int tm = tl > 0 ? tl - 1 : nt - 1;
#pragma unroll
                for (int k = 0; k < KC; k++) {
                    cpx<R> p[12];
                    hload_spinor<R>(rf, cs, (uint32_t)k * fs, (tm * L3 + yz * L + xof(tl)) >> 1, p);
                    project<R, 0, BW>(p, h[k]);
                }
            }
        };
        if (tb < te) load_bw(tb, cA);
        if (tb + 1 < te) load_bw(tb + 1, cB);
#pragma unroll 1
        for (int tl = tb; tl < te; tl++) {
            const int x = xof(tl);
            const int sp = yz * L + x;
            const int s = tl * L3 + sp;
            const int h = s >> 1;
            const int tg = tglob(tl);
            cpx<R> a[KC][12];
#pragma unroll
            for (int k = 0; k < KC; k++)
#pragma unroll
                for (int c = 0; c < 12; c++) a[k][c] = mk<R>(0, 0);
            // backward time hop from the carried half spinors, link U_0(x, tl - 1) on the input parity
            if (tl > 0 || g.whole) {
                const R ph = (tg == 0) ? R(g.bc) : R(1);
                if (ph != R(0)) {
                    cpx<R> w[9];
                    bload_link_r<R, REC>(ub[0], ls, ((tl > 0 ? tl - 1 : nt - 1) * L3 + sp) >> 1, w);
#pragma unroll
                    for (int k = 0; k < KC; k++) {
                        cpx<R> t[6];
                        transport<R, true>(w, cA[k], ph, t);
                        accum<R, 0, BW>(a[k], t);
                    }
                }
            }
            // forward time hop; the loaded spinors are also the backward neighbours of slice tl + 2
            cpx<R> nb2[KC][6];
#pragma unroll
            for (int k = 0; k < KC; k++)
#pragma unroll
                for (int j = 0; j < 6; j++) nb2[k][j] = mk<R>(0, 0);
            const bool endt = (tl == nt - 1);
            if (!endt || g.whole) {
                const R ph = (tg == g.T - 1) ? R(g.bc) : R(1);
                cpx<R> w[9];
#pragma unroll
                for (int k = 0; k < KC; k++) {
                    cpx<R> p[12];
                    hload_spinor<R>(rf, cs, (uint32_t)k * fs, (endt ? sp : s + L3) >> 1, p);
                    if (k == 0 && ph != R(0)) bload_link_r<R, REC>(uf[0], ls, h, w);
                    if (ph != R(0)) {
                        cpx<R> hf[6];
                        project<R, 0, FW>(p, hf);
                        cpx<R> t[6];
                        transport<R, false>(w, hf, ph, t);
                        accum<R, 0, FW>(a[k], t);
                    }
                    if (!endt) project<R, 0, BW>(p, nb2[k]);
                }
            }
            const int dxp = (x == L - 1) ? -(L - 1) : 1, dxm = (x == 0) ? (L - 1) : -1;
            bhop_cols<R, 1, FW, false, KC, REC, true>(a, rf, cs, fs, (s + dxp) >> 1, uf[1], ls, h);
            bhop_cols<R, 1, BW, true, KC, REC, true>(a, rf, cs, fs, (s + dxm) >> 1, ub[1], ls, (s + dxm) >> 1);
            bhop_cols<R, 2, FW, false, KC, REC, true>(a, rf, cs, fs, (s + dyp) >> 1, uf[2], ls, h);
            bhop_cols<R, 2, BW, true, KC, REC, true>(a, rf, cs, fs, (s + dym) >> 1, ub[2], ls, (s + dym) >> 1);
            bhop_cols<R, 3, FW, false, KC, REC, true>(a, rf, cs, fs, (s + dzp) >> 1, uf[3], ls, h);
            bhop_cols<R, 3, BW, true, KC, REC, true>(a, rf, cs, fs, (s + dzm) >> 1, ub[3], ls, (s + dzm) >> 1);

#pragma unroll
            for (int k = 0; k < KC; k++) {
#pragma unroll
                for (int qq = 0; qq < 6; qq++) {
                    cpx<R> pc2[2] = {mk<R>(0, 0), mk<R>(0, 0)}, q2[2] = {mk<R>(0, 0), mk<R>(0, 0)}, r2[2];
                    if (has_self) hload_pair<R>(rs, cs, (uint32_t)k * fs, h, qq, pc2[0], pc2[1]);
                    if (EPI == EPI_RESID || EPI == EPI_DOT_AUX) hload_pair<R>(rx, cs, (uint32_t)k * fs, h, qq, q2[0], q2[1]);
#pragma unroll
                    for (int e = 0; e < 2; e++) {
                        const int c = 2 * qq + e;
                        const cpx<R> pc = pc2[e], q = q2[e];
                        cpx<R> r = mk<R>(a_self * pc.re + c_hop * a[k][c].re, a_self * pc.im + c_hop * a[k][c].im);
                        if (EPI == EPI_RESID) r = q - r;
                        r2[e] = r;
                        if (EPI == EPI_DOT_AUX) {
                            d[k][0] += (double)q.re * r.re + (double)q.im * r.im;
                            d[k][1] += (double)q.re * r.im - (double)q.im * r.re;
                        } else if (EPI == EPI_TS) {
                            d[k][0] += (double)r.re * pc.re + (double)r.im * pc.im;
                            d[k][1] += (double)r.re * pc.im - (double)r.im * pc.re;
                            d[k][2] += (double)r.re * r.re + (double)r.im * r.im;
                        } else if (EPI == EPI_RESID || EPI == EPI_NORM) {
                            d[k][0] += (double)r.re * r.re + (double)r.im * r.im;
                        }
                    }
                    hstore_pair<R, NTS>(ro[k], cs, 0u, h, qq, r2[0], r2[1]);
                }
            }
            // slice tl + 1 uses cB; slice tl + 2 the half spinors just loaded
#pragma unroll
            for (int k = 0; k < KC; k++)
#pragma unroll
                for (int j = 0; j < 6; j++) {
                    cA[k][j] = cB[k][j];
                    cB[k][j] = nb2[k][j];
                }
        }
    }
    if (EPI != EPI_STORE) block_sum_cols<NT, KC>(d, slot, slot_col);
}

}  // namespace dd
