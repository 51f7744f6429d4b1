// dd_dslash.h -- the Wilson-Dirac stencil on one tile, shared by the
// single-lattice kernel (dirac.hip) and the multi-domain kernel (batched.hip).
//
// D psi(x) = psi(x)/(2 kappa) - 1/2 sum_mu [ (1-gamma_mu) U_mu(x) psi(x+mu)
//                                          + (1+gamma_mu) U_mu(x-mu)^+ psi(x-mu) ]
// (normalisation 2 kappa D = 1 - kappa D_hop, paper Sec. 5), on a whole lattice
// or on a Dirichlet time slab (paper Sec. 3 Eq. 10: the diagonal block of D; hops
// leaving the slab are dropped).  D^+ = gamma_5 D gamma_5 swaps the projectors.
//
// A tile is NT consecutive spatial sites of one column over a chunk of tc_len
// time slices.  A thread owns one spatial site and sweeps the chunk: psi(t) and
// the transported backward half spinor U_0(t)^+ P_+ psi(t) are carried in
// registers from one slice to the next, so the time neighbours and the
// backward time link are fetched exactly once; the spatial neighbours of slice
// t are fetched by the threads that own them at about the same moment and are
// served from L1 / L2.  Each neighbour spinor is projected to a half spinor
// (2 spins x 3 colours) before the SU(3) multiply.  All loads and stores go
// through raw buffer resources (32-bit offsets within one column).
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

#include "dd_internal.h"
#include "dd_wilson.h"

namespace dd {

// in / out / aux point at the first component of this tile's column (layout
// [12][nsite]); U points at the links of the tile's lattice ([4][9][vlink]).
template <typename R, int DAG, int EPI, int NT>
__device__ __forceinline__ void dslash_tile(const Geo& g, const cpx<R>* __restrict__ U, R mass,
                                            const cpx<R>* __restrict__ in, cpx<R>* __restrict__ out,
                                            const cpx<R>* __restrict__ aux, int sb, int tc, int tc_len,
                                            double* __restrict__ slot) {
    const int L = g.L, L2 = g.L2, L3 = g.L3;
    const int sp = sb * NT + threadIdx.x;
    const int nsite = g.nsite, nt = g.nt;
    constexpr uint32_t CB = sizeof(cpx<R>);
    const uint32_t cs = (uint32_t)nsite * CB;    // component stride (bytes)
    const uint32_t ls = (uint32_t)g.vlink * CB;  // link-row stride (bytes)
    constexpr int FW = DAG ? +1 : -1;            // forward hop projector (1 + FW gamma)
    constexpr int BW = -FW;
    double d0 = 0, d1 = 0, d2 = 0;

    if (sp < L3) {
        const rsrc_t rf = make_rsrc(in, 12u * cs);
        const rsrc_t ro = make_rsrc(out, 12u * cs);
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
        // backward half spinor entering slice tb: ph U_0(tb-1)^+ P psi(tb-1)
        cpx<R> hb[6];
#pragma unroll
        for (int k = 0; k < 6; k++) hb[k] = mk<R>(0, 0);
        if (tb > 0 || g.whole) {
            const int tlm = tb > 0 ? tb - 1 : nt - 1;
            const R ph = (tglob(tb) == 0) ? R(g.bc) : R(1);
            if (ph != R(0)) {
                cpx<R> p[12];
                bload_spinor<R>(rf, cs, tlm * L3 + sp, p);
                cpx<R> h[6];
                project<R, 0, BW>(p, h);
                cpx<R> w[9];
                const uint32_t vo = (uint32_t)(tglob(tlm) * L3 + sp) * CB;
#pragma unroll
                for (int k = 0; k < 9; k++) w[k] = bload<R>(ru0, vo, (uint32_t)k * ls);
                transport<R, true>(w, h, ph, hb);
            }
        }
        cpx<R> cur[12];
        if (tb < te) bload_spinor<R>(rf, cs, tb * L3 + sp, cur);
        const rsrc_t rx = (EPI == EPI_RESID || EPI == EPI_DOT_AUX) ? make_rsrc(aux, 12u * cs) : rf;
        const R half = R(0.5);
#pragma unroll 1
        for (int tl = tb; tl < te; tl++) {
            const int s = tl * L3 + sp;
            const int tg = tglob(tl);
            const int sl = tg * L3 + sp;
            cpx<R> a[12];
#pragma unroll
            for (int c = 0; c < 12; c++) a[c] = mk<R>(0, 0);
            accum<R, 0, BW>(a, hb);
            // forward time hop; the same link transports psi(t) into the next slice
            cpx<R> nxt[12];
            const bool endt = (tl == nt - 1);
            const R phf = (tg == g.T - 1) ? R(g.bc) : R(1);
            const bool hasf = (!endt || g.whole) && phf != R(0);
            if (hasf) {
                cpx<R> w[9];
                const uint32_t vo = (uint32_t)sl * CB;
#pragma unroll
                for (int k = 0; k < 9; k++) w[k] = bload<R>(ru0, vo, (uint32_t)k * ls);
                bload_spinor<R>(rf, cs, endt ? sp : s + L3, nxt);
                cpx<R> h[6];
                project<R, 0, FW>(nxt, h);
                cpx<R> t[6];
                transport<R, false>(w, h, phf, t);
                accum<R, 0, FW>(a, t);
                cpx<R> h2[6];
                project<R, 0, BW>(cur, h2);
                transport<R, true>(w, h2, phf, hb);
            } else {
#pragma unroll
                for (int k = 0; k < 6; k++) hb[k] = mk<R>(0, 0);
            }
            bhop<R, 1, FW, false>(a, rf, cs, s + dxp, ru1, ls, sl, R(1));
            bhop<R, 1, BW, true>(a, rf, cs, s + dxm, ru1, ls, sl + dxm, R(1));
            bhop<R, 2, FW, false>(a, rf, cs, s + dyp, ru2, ls, sl, R(1));
            bhop<R, 2, BW, true>(a, rf, cs, s + dym, ru2, ls, sl + dym, R(1));
            bhop<R, 3, FW, false>(a, rf, cs, s + dzp, ru3, ls, sl, R(1));
            bhop<R, 3, BW, true>(a, rf, cs, s + dzm, ru3, ls, sl + dzm, R(1));

            const uint32_t vo = (uint32_t)s * CB;
#pragma unroll
            for (int c = 0; c < 12; c++) {
                const uint32_t so = (uint32_t)c * cs;
                const cpx<R> pc = cur[c];
                cpx<R> r = EPI == EPI_HOP ? mk<R>(mass * a[c].re, mass * a[c].im)
                                          : mk<R>(mass * pc.re - half * a[c].re, mass * pc.im - half * a[c].im);
                cpx<R> q = mk<R>(0, 0);
                if (EPI == EPI_RESID || EPI == EPI_DOT_AUX) q = bload<R>(rx, vo, so);
                if (EPI == EPI_RESID) r = q - r;
                bstore<R>(ro, vo, so, r);
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
            if (tl + 1 < te) {
                if (hasf && !endt) {
#pragma unroll
                    for (int c = 0; c < 12; c++) cur[c] = nxt[c];
                } else {
                    bload_spinor<R>(rf, cs, (tl + 1) * L3 + sp, cur);
                }
            }
        }
    }
    if (EPI != EPI_STORE && EPI != EPI_HOP) block_sum3<NT>(d0, d1, d2, slot);
}

}  // namespace dd
