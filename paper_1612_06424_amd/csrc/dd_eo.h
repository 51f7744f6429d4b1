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
// is dropped, so no link outside the field is needed.  One thread computes
// one output half site:
//     out = a_self * self + c_hop * (H in)_site      (in: the other parity)
// (SELF = false: no self term, the pure hop).
// with the fused epilogues of the full stencil (dd_dslash.h).
#pragma once

#include "dd_internal.h"
#include "dd_wilson.h"

namespace dd {

template <typename R, int DAG, int EPI, int NT, bool SELF>
__device__ __forceinline__ void eo_hop_site(const Geo& g, const cpx<R>* __restrict__ Ueo, R a_self, R c_hop,
                                            int p_out, int h, const cpx<R>* __restrict__ in,
                                            const cpx<R>* __restrict__ self, cpx<R>* __restrict__ out,
                                            const cpx<R>* __restrict__ aux, double* __restrict__ slot) {
    const int L = g.L, L2 = g.L2, L3 = g.L3;
    const int nh = g.nsite >> 1;
    constexpr uint32_t CB = sizeof(cpx<R>);
    const uint32_t cs = (uint32_t)nh * CB;       // component stride of a half field (bytes)
    const uint32_t ls = 2u * (uint32_t)nh * CB;  // link-row stride of Ueo (bytes)
    const uint32_t ubytes = 17u * (uint32_t)nh * CB;  // rows 0..8 of one (mu, parity)
    constexpr int FW = DAG ? +1 : -1;            // forward hop projector (1 + FW gamma)
    constexpr int BW = -FW;
    double d0 = 0, d1 = 0, d2 = 0;
    if (h < nh) {
        const int Lh = L >> 1, L3h = L3 >> 1;
        const int tl = h / L3h;
        const int rem = h - tl * L3h;
        const int xh = rem % Lh, yz = rem / Lh;
        const int y = yz % L, z = yz / L;
        const int x = 2 * xh + ((p_out + tl + y + z) & 1);
        const int sp = yz * L + x;
        const int s = tl * L3 + sp;
        const int t = g.t0 + tl;
        const int tg = t >= g.T ? t - g.T : t;
        const rsrc_t rf = make_rsrc(in, 12u * cs);
        // forward links at this site (parity p_out), backward ones at the neighbour (1 - p_out)
        rsrc_t uf[4], ub[4];
#pragma unroll
        for (int mu = 0; mu < 4; mu++) {
            uf[mu] = make_rsrc(Ueo + (size_t)(mu * 18 + p_out) * nh, ubytes);
            ub[mu] = make_rsrc(Ueo + (size_t)(mu * 18 + 1 - p_out) * nh, ubytes);
        }
        const int dxp = (x == L - 1) ? -(L - 1) : 1, dxm = (x == 0) ? (L - 1) : -1;
        const int dyp = (y == L - 1) ? -(L - 1) * L : L, dym = (y == 0) ? (L - 1) * L : -L;
        const int dzp = (z == L - 1) ? -(L - 1) * L2 : L2, dzm = (z == 0) ? (L - 1) * L2 : -L2;
        cpx<R> a[12];
#pragma unroll
        for (int c = 0; c < 12; c++) a[c] = mk<R>(0, 0);
        // time: forward to tl + 1 (link at this site), backward from tl - 1 (link there)
        const bool endt = (tl == g.nt - 1), begt = (tl == 0);
        if (!endt || g.whole) {
            const R ph = (tg == g.T - 1) ? R(g.bc) : R(1);
            if (ph != R(0)) bhop<R, 0, FW, false>(a, rf, cs, (endt ? sp : s + L3) >> 1, uf[0], ls, h, ph);
        }
        if (!begt || g.whole) {
            const R ph = (tg == 0) ? R(g.bc) : R(1);
            const int nb = (begt ? (g.nt - 1) * L3 + sp : s - L3) >> 1;
            if (ph != R(0)) bhop<R, 0, BW, true>(a, rf, cs, nb, ub[0], ls, nb, ph);
        }
        bhop<R, 1, FW, false>(a, rf, cs, (s + dxp) >> 1, uf[1], ls, h, R(1));
        bhop<R, 1, BW, true>(a, rf, cs, (s + dxm) >> 1, ub[1], ls, (s + dxm) >> 1, R(1));
        bhop<R, 2, FW, false>(a, rf, cs, (s + dyp) >> 1, uf[2], ls, h, R(1));
        bhop<R, 2, BW, true>(a, rf, cs, (s + dym) >> 1, ub[2], ls, (s + dym) >> 1, R(1));
        bhop<R, 3, FW, false>(a, rf, cs, (s + dzp) >> 1, uf[3], ls, h, R(1));
        bhop<R, 3, BW, true>(a, rf, cs, (s + dzm) >> 1, ub[3], ls, (s + dzm) >> 1, R(1));

        const rsrc_t ro = make_rsrc(out, 12u * cs);
        constexpr bool has_self = SELF || EPI == EPI_TS;
        const rsrc_t rs = make_rsrc(self != nullptr ? self : in, 12u * cs);
        const rsrc_t rx = make_rsrc(aux != nullptr ? aux : in, 12u * cs);
        const uint32_t vo = (uint32_t)h * CB;
#pragma unroll
        for (int c = 0; c < 12; c++) {
            const uint32_t so = (uint32_t)c * cs;
            const cpx<R> pc = has_self ? bload<R>(rs, vo, so) : mk<R>(0, 0);
            cpx<R> r = mk<R>(a_self * pc.re + c_hop * a[c].re, a_self * pc.im + c_hop * a[c].im);
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
    }
    if (EPI != EPI_STORE) block_sum3<NT>(d0, d1, d2, slot);
}

// Time-sweep form of the half hop.  A thread owns one pair (xh, y, z) of
// every slice and walks a chunk of tc_len slices; at slice t its output site is
// x = 2 xh + b(t), with b alternating from slice to slice.  The forward time
// neighbour loaded at slice t, (x(t), t + 1), is the backward time neighbour of
// the output at slice t + 2 (same x), so its projected half spinor is carried
// two steps and every input site of the chunk is loaded once in time
// direction.  tile: NT consecutive pair indices of a slice.
template <typename R, int DAG, int EPI, int NT, bool SELF>
__device__ __forceinline__ void eo_sweep_tile(const Geo& g, const cpx<R>* __restrict__ Ueo, R a_self, R c_hop,
                                              int p_out, const cpx<R>* __restrict__ in,
                                              const cpx<R>* __restrict__ self, cpx<R>* __restrict__ out,
                                              const cpx<R>* __restrict__ aux, int tile, int chunk, int tc_len,
                                              double* __restrict__ slot) {
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
        const int xh = pr % Lh, yz = pr / Lh;
        const int y = yz % L, z = yz / L;
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
                bload_spinor<R>(rf, cs, (tm * L3 + yz * L + xof(tl)) >> 1, p);
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
                bload_spinor<R>(rf, cs, (endt ? sp : s + L3) >> 1, p);
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
            bhop<R, 1, FW, false>(a, rf, cs, (s + dxp) >> 1, uf[1], ls, h, R(1));
            bhop<R, 1, BW, true>(a, rf, cs, (s + dxm) >> 1, ub[1], ls, (s + dxm) >> 1, R(1));
            bhop<R, 2, FW, false>(a, rf, cs, (s + dyp) >> 1, uf[2], ls, h, R(1));
            bhop<R, 2, BW, true>(a, rf, cs, (s + dym) >> 1, ub[2], ls, (s + dym) >> 1, R(1));
            bhop<R, 3, FW, false>(a, rf, cs, (s + dzp) >> 1, uf[3], ls, h, R(1));
            bhop<R, 3, BW, true>(a, rf, cs, (s + dzm) >> 1, ub[3], ls, (s + dzm) >> 1, R(1));

            const uint32_t vo = (uint32_t)h * CB;
#pragma unroll
            for (int c = 0; c < 12; c++) {
                const uint32_t so = (uint32_t)c * cs;
                const cpx<R> pc = has_self ? bload<R>(rs, vo, so) : mk<R>(0, 0);
                cpx<R> r = mk<R>(a_self * pc.re + c_hop * a[c].re, a_self * pc.im + c_hop * a[c].im);
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

}  // namespace dd
