// dd_dslash.h -- the Wilson-Dirac stencil on one tile, shared by the
// single-lattice kernel (dirac.hip) and the multi-domain kernel (batched.hip).
//
// D psi(x) = psi(x)/(2 kappa) - 1/2 sum_mu [ (1-gamma_mu) U_mu(x) psi(x+mu)
//                                          + (1+gamma_mu) U_mu(x-mu)^+ psi(x-mu) ]
// (normalisation 2 kappa D = 1 - kappa D_hop, paper Sec. 5), on a whole lattice
// or on a Dirichlet time slab (paper Sec. 3 Eq. 10: the diagonal block of D; hops
// leaving the slab are dropped).  D^+ = gamma_5 D gamma_5 swaps the projectors.
//
// A tile is NT consecutive spatial sites of KC columns over a chunk of tc_len
// time slices.  A thread owns one spatial site and sweeps the chunk: psi(t) and
// the transported backward half spinor U_0(t)^+ P_+ psi(t) are carried in
// registers from one slice to the next, so the time neighbours and the
// backward time link are fetched exactly once; the spatial neighbours of slice
// t are fetched by the threads that own them at about the same moment and are
// served from L1 / L2.  Each neighbour spinor is projected to a half spinor
// (2 spins x 3 colours) before the SU(3) multiply.  All loads and stores go
// through raw buffer resources (32-bit offsets within one column).
//
// XS (L dividing 64, at least 4): a wavefront holds whole x rows, one site per
// lane, so the two x hops need no loads: each lane projects its own psi(x),
// hands P psi(x) to the lane of x - 1 (its forward neighbour's hop) and
// U_1(x)^+ P psi(x) (with the link it loads for its own forward hop) to the lane
// of x + 1, through cross-lane permutes.  The products and the order of the hop
// sums are those of the loading form; the compiler's multiply-add contraction
// differs between the two forms, so they agree to rounding, not bitwise.
//
// Fused epilogues (EPI): the result is stored and, per workgroup, FP64 partial
// sums are written to slot[0..2]:
//   EPI_STORE    nothing
//   EPI_DOT_AUX  <aux, D in>            (BiCGStab alpha denominator)
//   EPI_TS       <D in, in>, |D in|^2   (BiCGStab omega)
//   EPI_RESID    stores aux - D in and its norm^2 (true residual)
//   EPI_NORM     |D in|^2               (CGNR)
//   EPI_HOP      nothing; stores kappa D_hop in (the hopping term alone, Sec. 5:
//                2 kappa D = 1 - kappa D_hop), with `mass` carrying kappa
#pragma once

#include "dd_eo.h"
#include "dd_internal.h"
#include "dd_wilson.h"

namespace dd {

// in / out / aux point at the first component of the tile's first column
// (layout [col][12][nsite], KC columns back to back); U points at the links of
// the tile's lattice ([4][9][vlink]).  Every link is loaded once for the KC
// columns, whose arithmetic is that of one column each, in the same order, so
// the result does not depend on KC.  Column k's output is written only if bit
// k of live is set (its stores go through a buffer resource of size 0
// otherwise, which drops them); its sums go to slot + 3 k slot_col.
// Site of thread tid of spatial tile sb: NT consecutive sites (whole x rows of z
// planes), or (bricks = true, NT a multiple of L, see brick_rows) a brick of RY x RZ
// whole x rows in (y, z), so that most y and z neighbours lie inside the tile; a
// wavefront still reads whole consecutive rows.  Returns L3 for a thread past the end.
__device__ __forceinline__ int tile_site(int sb, int tid, int NT, int L, int L3, bool bricks, int ry) {
    if (!bricks) return min(sb * NT + tid, L3);
    const int rows = NT / L, rz = rows / ry;
    const int nby = L / ry;
    const int by = sb % nby, bz = sb / nby;
    const int r = tid / L, x = tid - r * L;
    const int y = by * ry + r % ry, z = bz * rz + r / ry;
    return (z * L + y) * L + x;
}

// Value v of the lane whose index is src_lane (all 64 lanes of the wavefront active).
__device__ __forceinline__ float lane_read(float v, int src_lane) {
    return __int_as_float(__builtin_amdgcn_ds_bpermute(src_lane << 2, __float_as_int(v)));
}
__device__ __forceinline__ double lane_read(double v, int src_lane) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_ds_bpermute(src_lane << 2, (int)(b & 0xffffffffll));
    const int hi = __builtin_amdgcn_ds_bpermute(src_lane << 2, (int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// The x hops of a site from the lanes of its x neighbours (XS form): a[k] += the
// forward hop (1 + FW gamma_1) U_1(x) psi(x + 1), then the backward hop
// (1 - FW gamma_1) U_1(x - 1)^+ psi(x - 1), as bhop_cols adds them.
template <typename R, int FW, int KC>
__device__ __forceinline__ void xhops_lanes(cpx<R> (&a)[KC][12], const cpx<R> (&cur)[KC][12], rsrc_t u, uint32_t ls,
                                            int sl, int x, int L) {
    constexpr int BW = -FW;
    cpx<R> w[9];
    bload_link<R>(u, ls, sl, w);  // U_1(x)
    const int lane = (int)(threadIdx.x & (kWave - 1));
    const int up = x == L - 1 ? lane - (L - 1) : lane + 1;  // the lane of x + 1
    const int dn = x == 0 ? lane + (L - 1) : lane - 1;      // the lane of x - 1
#pragma unroll
    for (int k = 0; k < KC; k++) {
        cpx<R> h[6], t[6];
        project<R, 1, FW>(cur[k], h);
#pragma unroll
        for (int j = 0; j < 6; j++) h[j] = mk<R>(lane_read(h[j].re, up), lane_read(h[j].im, up));
        transport<R, false>(w, h, R(1), t);
        accum<R, 1, FW>(a[k], t);
        project<R, 1, BW>(cur[k], h);
        transport<R, true>(w, h, R(1), t);
#pragma unroll
        for (int j = 0; j < 6; j++) t[j] = mk<R>(lane_read(t[j].re, dn), lane_read(t[j].im, dn));
        accum<R, 1, BW>(a[k], t);
    }
}

template <typename R, int DAG, int EPI, int NT, int KC, bool XS = false>
__device__ __forceinline__ void dslash_tile_cols(const Geo& g, const cpx<R>* __restrict__ U, R mass,
                                                 const cpx<R>* __restrict__ in, cpx<R>* __restrict__ out,
                                                 const cpx<R>* __restrict__ aux, unsigned live, int sb, int tc,
                                                 int tc_len, double* __restrict__ slot, size_t slot_col,
                                                 bool bricks = false, int ry = 1) {
    const int L = g.L, L2 = g.L2, L3 = g.L3;
    const int sp = tile_site(sb, (int)threadIdx.x, NT, L, L3, bricks, ry);
    const int nsite = g.nsite, nt = g.nt;
    constexpr uint32_t CB = sizeof(cpx<R>);
    const uint32_t cs = (uint32_t)nsite * CB;    // component stride (bytes)
    const uint32_t fs = 12u * cs;                // column stride (bytes)
    const uint32_t ls = (uint32_t)g.vlink * CB;  // link-row stride (bytes)
    constexpr int FW = DAG ? +1 : -1;            // forward hop projector (1 + FW gamma)
    constexpr int BW = -FW;
    double d[KC][3];
#pragma unroll
    for (int k = 0; k < KC; k++) d[k][0] = d[k][1] = d[k][2] = 0;

    if (sp < L3) {
        const rsrc_t rf = make_rsrc(in, (uint32_t)KC * fs);
        rsrc_t ro[KC];
#pragma unroll
        for (int k = 0; k < KC; k++) ro[k] = make_rsrc(out + (size_t)k * 12 * nsite, ((live >> k) & 1u) ? fs : 0u);
        const rsrc_t ru0 = make_rsrc(U, 9u * ls);
        const rsrc_t ru1 = make_rsrc(U + (size_t)9 * g.vlink, 9u * ls);
        const rsrc_t ru2 = make_rsrc(U + (size_t)18 * g.vlink, 9u * ls);
        const rsrc_t ru3 = make_rsrc(U + (size_t)27 * g.vlink, 9u * ls);
        const int x = sp % L, yz = sp / L;
        const int y = yz % L, z = yz / L;
        const int dxp = (x == L - 1) ? -(L - 1) : 1, dxm = (x == 0) ? (L - 1) : -1;
        const int dyp = (y == L - 1) ? -(L - 1) * L : L, dym = (y == 0) ? (L - 1) * L : -L;
        const int dzp = (z == L - 1) ? -(L - 1) * L2 : L2, dzm = (z == 0) ? (L - 1) * L2 : -L2;
        const int tb = tc * tc_len;
        const int te = min(nt, tb + tc_len);
        auto tglob = [&](int tl) {
            const int t = g.t0 + tl;
            return t >= g.T ? t - g.T : t;
        };
        // backward half spinors entering slice tb: ph U_0(tb-1)^+ P psi(tb-1)
        cpx<R> hb[KC][6];
#pragma unroll
        for (int k = 0; k < KC; k++)
#pragma unroll
            for (int j = 0; j < 6; j++) hb[k][j] = mk<R>(0, 0);
        if (tb > 0 || g.whole) {
            const int tlm = tb > 0 ? tb - 1 : nt - 1;
            const R ph = (tglob(tb) == 0) ? R(g.bc) : R(1);
            if (ph != R(0)) {
                cpx<R> w[9];
                const uint32_t vo = (uint32_t)(tglob(tlm) * L3 + sp) * CB;
#pragma unroll
                for (int j = 0; j < 9; j++) w[j] = bload<R>(ru0, vo, (uint32_t)j * ls);
#pragma unroll
                for (int k = 0; k < KC; k++) {
                    cpx<R> p[12];
                    bload_spinor_col<R>(rf, cs, (uint32_t)k * fs, tlm * L3 + sp, p);
                    cpx<R> h[6];
                    project<R, 0, BW>(p, h);
                    transport<R, true>(w, h, ph, hb[k]);
                }
            }
        }
        cpx<R> cur[KC][12];
        if (tb < te) {
#pragma unroll
            for (int k = 0; k < KC; k++) bload_spinor_col<R>(rf, cs, (uint32_t)k * fs, tb * L3 + sp, cur[k]);
        }
        const rsrc_t rx = (EPI == EPI_RESID || EPI == EPI_DOT_AUX) ? make_rsrc(aux, (uint32_t)KC * fs) : rf;
        const R half = R(0.5);
#pragma unroll 1
        for (int tl = tb; tl < te; tl++) {
            const int s = tl * L3 + sp;
            const int tg = tglob(tl);
            const int sl = tg * L3 + sp;
            cpx<R> a[KC][12];
#pragma unroll
            for (int k = 0; k < KC; k++) {
#pragma unroll
                for (int c = 0; c < 12; c++) a[k][c] = mk<R>(0, 0);
                accum<R, 0, BW>(a[k], hb[k]);
            }
            // forward time hop; the same link transports psi(t) into the next slice
            cpx<R> nxt[KC][12];
            const bool endt = (tl == nt - 1);
            const R phf = (tg == g.T - 1) ? R(g.bc) : R(1);
            const bool hasf = (!endt || g.whole) && phf != R(0);
            if (hasf) {
                cpx<R> w[9];
                const uint32_t vo = (uint32_t)sl * CB;
#pragma unroll
                for (int j = 0; j < 9; j++) w[j] = bload<R>(ru0, vo, (uint32_t)j * ls);
#pragma unroll
                for (int k = 0; k < KC; k++) {
                    bload_spinor_col<R>(rf, cs, (uint32_t)k * fs, endt ? sp : s + L3, nxt[k]);
                    cpx<R> h[6];
                    project<R, 0, FW>(nxt[k], h);
                    cpx<R> t[6];
                    transport<R, false>(w, h, phf, t);
                    accum<R, 0, FW>(a[k], t);
                    cpx<R> h2[6];
                    project<R, 0, BW>(cur[k], h2);
                    transport<R, true>(w, h2, phf, hb[k]);
                }
            } else {
#pragma unroll
                for (int k = 0; k < KC; k++)
#pragma unroll
                    for (int j = 0; j < 6; j++) hb[k][j] = mk<R>(0, 0);
            }
            if constexpr (XS) {
                xhops_lanes<R, FW, KC>(a, cur, ru1, ls, sl, x, L);
            } else {
                bhop_cols<R, 1, FW, false, KC, false>(a, rf, cs, fs, s + dxp, ru1, ls, sl);
                bhop_cols<R, 1, BW, true, KC, false>(a, rf, cs, fs, s + dxm, ru1, ls, sl + dxm);
            }
            bhop_cols<R, 2, FW, false, KC, false>(a, rf, cs, fs, s + dyp, ru2, ls, sl);
            bhop_cols<R, 2, BW, true, KC, false>(a, rf, cs, fs, s + dym, ru2, ls, sl + dym);
            bhop_cols<R, 3, FW, false, KC, false>(a, rf, cs, fs, s + dzp, ru3, ls, sl);
            bhop_cols<R, 3, BW, true, KC, false>(a, rf, cs, fs, s + dzm, ru3, ls, sl + dzm);

            const uint32_t vo = (uint32_t)s * CB;
#pragma unroll
            for (int k = 0; k < KC; k++) {
#pragma unroll
                for (int c = 0; c < 12; c++) {
                    const uint32_t so = (uint32_t)c * cs;
                    const cpx<R> pc = cur[k][c];
                    cpx<R> r = EPI == EPI_HOP
                                   ? mk<R>(mass * a[k][c].re, mass * a[k][c].im)
                                   : mk<R>(mass * pc.re - half * a[k][c].re, mass * pc.im - half * a[k][c].im);
                    cpx<R> q = mk<R>(0, 0);
                    if (EPI == EPI_RESID || EPI == EPI_DOT_AUX) q = bload<R>(rx, vo, (uint32_t)k * fs + so);
                    if (EPI == EPI_RESID) r = q - r;
                    bstore<R>(ro[k], vo, so, r);
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
            }
            if (tl + 1 < te) {
                if (hasf && !endt) {
#pragma unroll
                    for (int k = 0; k < KC; k++)
#pragma unroll
                        for (int c = 0; c < 12; c++) cur[k][c] = nxt[k][c];
                } else {
#pragma unroll
                    for (int k = 0; k < KC; k++)
                        bload_spinor_col<R>(rf, cs, (uint32_t)k * fs, (tl + 1) * L3 + sp, cur[k]);
                }
            }
        }
    }
    if (EPI != EPI_STORE && EPI != EPI_HOP) block_sum_cols<NT, KC>(d, slot, slot_col);
}

// One column (the multi-domain kernel's tile).
template <typename R, int DAG, int EPI, int NT>
__device__ __forceinline__ void dslash_tile(const Geo& g, const cpx<R>* __restrict__ U, R mass,
                                            const cpx<R>* __restrict__ in, cpx<R>* __restrict__ out,
                                            const cpx<R>* __restrict__ aux, int sb, int tc, int tc_len,
                                            double* __restrict__ slot) {
    dslash_tile_cols<R, DAG, EPI, NT, 1>(g, U, mass, in, out, aux, 1u, sb, tc, tc_len, slot, 0);
}

}  // namespace dd
