// dd_eo_lds.h -- the even-odd half hop with its input tile staged in LDS.
//
// The same operator as the time-sweep kernels of dd_eo.h,
//     out = a_self * self + c_hop * (H in)_site     (in: the other parity),
// organised for reuse instead of for a register carry:
//   * a workgroup owns one time slice of a brick of RY x RZ rows (y, z) of full
//     x rows (LH pairs each, RY RZ LH = 256 output sites, one per thread) and
//     loops over a group of columns;
//   * the links of its 256 output sites (8 per site, two rows each, the third
//     rebuilt from the unitarity of SU(3)) are loaded once into registers and
//     serve every column of the group;
//   * per column the input half field of the brick's rows and of the one-row
//     halo around it in y and z is staged in LDS (each thread two neighbouring
//     sites, 16-byte loads of component pairs); halo sites are stored already
//     spin-projected (the one
//     hop that reads each needs one projection), so each input site is fetched
//     from memory about twice per launch instead of once per neighbour;
//   * the spatial hops read LDS, the two time hops read the thread's own site
//     on the slices either side directly (a coalesced, per-thread access).
// The output parity alternates with the row's y + z, so a thread's output site
// is x = 2 xh + b(row); its x neighbours are pair xh or xh +- 1 of the same row
// and its y and z neighbours sit in pair xh of the adjacent rows.
#pragma once

#include "dd_eo.h"

namespace dd {

// Brick of RY x RZ rows for L = 2 LH (RY RZ LH = 256 threads, one output site each).
template <int LH>
struct LdsTile;
template <>
struct LdsTile<16> {
    static constexpr int RY = 4, RZ = 4;
};
template <>
struct LdsTile<8> {
    static constexpr int RY = 8, RZ = 4;
};

constexpr int kLdsNT = 256;

// The first two rows of a link (six entries); the third is rebuilt where the link is used.
// (FP32: the paired layout of dd_eo.h, rows of units 2 ls bytes apart.)
template <typename R>
__device__ __forceinline__ void bload_link6(rsrc_t u, uint32_t ls, int sl, cpx<R> (&w)[6]) {
    cpx<R> w9[9];
    bload_link_r<R, true>(u, ls, sl, w9);
#pragma unroll
    for (int k = 0; k < 6; k++) w[k] = w9[k];
}
template <typename R>
__device__ __forceinline__ void link_full(const cpx<R> (&w6)[6], cpx<R> (&w)[9]) {
#pragma unroll
    for (int k = 0; k < 6; k++) w[k] = w6[k];
    const cpx<R> c6 = w6[1] * w6[5] - w6[2] * w6[4];
    const cpx<R> c7 = w6[2] * w6[3] - w6[0] * w6[5];
    const cpx<R> c8 = w6[0] * w6[4] - w6[1] * w6[3];
    w[6] = mk<R>(c6.re, -c6.im);
    w[7] = mk<R>(c7.re, -c7.im);
    w[8] = mk<R>(c8.re, -c8.im);
}

// a += (1 + SGN gamma_MU) W h with W = U (fwd) or U^+ (bwd), h already projected.
template <typename R, int MU, int SGN, bool BWD>
__device__ __forceinline__ void hop_half(cpx<R> (&a)[12], const cpx<R> (&w6)[6], const cpx<R> (&h)[6], R ph) {
    cpx<R> w[9];
    link_full<R>(w6, w);
    cpx<R> t[6];
    transport<R, BWD>(w, h, ph, t);
    accum<R, MU, SGN>(a, t);
}

// One workgroup: slice tl of brick `tile`, columns [col_lo, col_hi).  Partial
// slot of (col, block) = col * nblk + block, block = tile + ntile * tl.
template <typename R, int DAG, int EPI, bool SELF, int LH, bool NTS>
__device__ __forceinline__ void eo_lds_body(const Geo& g, const cpx<R>* __restrict__ U12, R a_self, R c_hop, int p_out,
                                            const cpx<R>* __restrict__ in, const cpx<R>* __restrict__ self,
                                            cpx<R>* __restrict__ out, const cpx<R>* __restrict__ aux, int ncol,
                                            int cpw, int remap, double* __restrict__ partial,
                                            const ColState* __restrict__ st) {
    constexpr int RY = LdsTile<LH>::RY, RZ = LdsTile<LH>::RZ;
    constexpr int L = 2 * LH, L2 = L * L, L3 = L2 * L;
    constexpr int NR = RY * RZ;                  // rows of the brick
    constexpr int NHR = 2 * RZ + 2 * RY;         // halo rows: y-, y+ (per z), z-, z+ (per y)
    constexpr int NPAIR = (NR + NHR) * (LH / 2); // staging units: two sites of a row, 12 components
    static_assert(NR * LH == kLdsNT, "one output site per thread");
    static_assert(NPAIR <= kLdsNT, "one staging unit per thread at most");
    __shared__ cpx<R> s_in[12][NR][LH];  // brick rows, full spinors
    __shared__ cpx<R> s_h[6][NHR][LH];   // halo rows, projected for the hop that reads them

    constexpr uint32_t CB = sizeof(cpx<R>);
    const int nt = g.nt;
    const int nh = g.nsite >> 1;
    const uint32_t cs = (uint32_t)nh * CB;         // component stride
    const uint32_t fs = 12u * cs;                  // column stride
    const uint32_t ls = 2u * (uint32_t)nh * CB;    // link-row stride (both parities)
    const uint32_t ubytes = sizeof(R) == 4 ? 5u * (uint32_t)nh * 16u : 11u * (uint32_t)nh * CB;
    constexpr int FW = DAG ? +1 : -1;  // forward hop projector (1 + FW gamma)
    constexpr int BW = -FW;
    constexpr bool has_self = SELF || EPI == EPI_TS;

    constexpr int NBY = L / RY;
    const int ntile = NBY * (L / RZ);
    const int nblk = ntile * nt;
    const int lb = remap ? xcd_remap(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    const int tile = lb % ntile;
    const int rest = lb / ntile;
    const int tl = rest % nt;
    const int col_lo = (rest / nt) * cpw;
    const int col_hi = min(ncol, col_lo + cpw);
    const int blk = tile + ntile * tl;
    const int y0 = (tile % NBY) * RY, z0 = (tile / NBY) * RZ;

    const int tid = (int)threadIdx.x;
    const int r = tid / LH, xh = tid - r * LH;
    const int ry = r % RY, rz = r / RY;
    const int y = y0 + ry, z = z0 + rz;
    const int bo = (p_out + tl + y + z) & 1;  // output site x = 2 xh + bo
    const int x = 2 * xh + bo;
    const int sp = (z * L + y) * L + x;
    const int s = tl * L3 + sp;
    const int h = s >> 1;
    const int tgl = g.t0 + tl;
    const int tg = tgl >= g.T ? tgl - g.T : tgl;
    // time hops: dropped at a slab's ends, across the time edge of a whole lattice with time_bc
    const R phb = (tl > 0 || g.whole) ? (tg == 0 ? R(g.bc) : R(1)) : R(0);
    const R phf = (tl < nt - 1 || g.whole) ? (tg == g.T - 1 ? R(g.bc) : R(1)) : R(0);
    const int hb = ((tl > 0 ? tl - 1 : nt - 1) * L3 + sp) >> 1;
    const int hf = ((tl < nt - 1 ? tl + 1 : 0) * L3 + sp) >> 1;

    // the eight links of this output site, two rows each
    cpx<R> wf[4][6], wb[4][6];
    {
        const int dxm = (x == 0) ? (L - 1) : -1;
        const int dym = (y == 0) ? (L - 1) * L : -L;
        const int dzm = (z == 0) ? (L - 1) * L2 : -L2;
        const int hbk[4] = {hb, (s + dxm) >> 1, (s + dym) >> 1, (s + dzm) >> 1};
#pragma unroll
        for (int mu = 0; mu < 4; mu++) {
            const size_t bf = sizeof(R) == 4 ? rec_link_base(mu, p_out, nh) : (size_t)(mu * 12 + p_out) * nh;
            const size_t bb = sizeof(R) == 4 ? rec_link_base(mu, 1 - p_out, nh) : (size_t)(mu * 12 + 1 - p_out) * nh;
            bload_link6<R>(make_rsrc(U12 + bf, ubytes), ls, h, wf[mu]);
            bload_link6<R>(make_rsrc(U12 + bb, ubytes), ls, hbk[mu], wb[mu]);
        }
    }

    // this thread's staging unit of every slice-tl tile: a brick row or a halo row
    // (face 0..3: y0 - 1, y0 + RY, z0 - 1, z0 + RZ, stored projected for the hop
    // that reads it), two neighbouring sites of it
    const bool stage = NPAIR == kLdsNT || tid < NPAIR;
    const int row = tid / (LH / 2), j = tid - row * (LH / 2);
    int face = -1, hr = 0;
    int sh0;  // the first of the unit's two half sites
    {
        int yy, zz;
        if (row < NR) {
            yy = y0 + row % RY;
            zz = z0 + row / RY;
        } else {
            hr = row - NR;
            if (hr < RZ) {
                face = 0;
                yy = y0 - 1;
                zz = z0 + hr;
            } else if (hr < 2 * RZ) {
                face = 1;
                yy = y0 + RY;
                zz = z0 + hr - RZ;
            } else if (hr < 2 * RZ + RY) {
                face = 2;
                zz = z0 - 1;
                yy = y0 + hr - 2 * RZ;
            } else {
                face = 3;
                zz = z0 + RZ;
                yy = y0 + hr - 2 * RZ - RY;
            }
            yy = yy < 0 ? yy + L : (yy >= L ? yy - L : yy);
            zz = zz < 0 ? zz + L : (zz >= L ? zz - L : zz);
        }
        const int base = (tl * L3 + (zz * L + yy) * L) >> 1;  // half-site index of the row's pair 0
        sh0 = base + 2 * j;
    }

    // Columns are software-pipelined: the loads of the next live column are issued
    // before the current one is computed, so a column's memory traffic overlaps the
    // previous column's arithmetic (one workgroup per CU holds enough in flight).
    auto next_live = [&](int c0) {
        int c1 = c0;
        while (c1 < col_hi && st != nullptr && !st[c1].active) c1++;  // uniform over the workgroup
        return c1;
    };
    cpx<R> pa[12], pc[12], pb[12], pf[12];  // staging unit (two sites) and the time neighbours
    auto issue = [&](int col) {
        const rsrc_t rf = make_rsrc(in + (size_t)col * 12 * (size_t)nh, fs);
        if (stage) {
            hload_spinor<R>(rf, cs, 0u, sh0, pa);
            hload_spinor<R>(rf, cs, 0u, sh0 + 1, pc);
        }
        // the thread's own site on the slices either side: always in range, unused where the hop is dropped
        hload_spinor<R>(rf, cs, 0u, hb, pb);
        hload_spinor<R>(rf, cs, 0u, hf, pf);
    };
    int col = next_live(col_lo);
    if (col < col_hi) issue(col);
    while (col < col_hi) {
        const size_t coff = (size_t)col * 12 * (size_t)nh;
        if (stage) {
            if (face < 0) {
#pragma unroll
                for (int c = 0; c < 12; c++) {
                    s_in[c][row][2 * j] = pa[c];
                    s_in[c][row][2 * j + 1] = pc[c];
                }
            } else {
                cpx<R> ha[6], hc[6];
                if (face == 0) {
                    project<R, 2, BW>(pa, ha);
                    project<R, 2, BW>(pc, hc);
                } else if (face == 1) {
                    project<R, 2, FW>(pa, ha);
                    project<R, 2, FW>(pc, hc);
                } else if (face == 2) {
                    project<R, 3, BW>(pa, ha);
                    project<R, 3, BW>(pc, hc);
                } else {
                    project<R, 3, FW>(pa, ha);
                    project<R, 3, FW>(pc, hc);
                }
#pragma unroll
                for (int k = 0; k < 6; k++) {
                    s_h[k][hr][2 * j] = ha[k];
                    s_h[k][hr][2 * j + 1] = hc[k];
                }
            }
        }
        cpx<R> hbp[6], hfp[6];  // projected time neighbours of this column
        project<R, 0, BW>(pb, hbp);
        project<R, 0, FW>(pf, hfp);
        __syncthreads();
        // the epilogue's loads go out before the next column's prefetch: loads retire in
        // order, so waiting for them then does not wait for the prefetch
        const rsrc_t rs = make_rsrc(self != nullptr ? self + coff : in + coff, fs);
        const rsrc_t rx = make_rsrc(aux != nullptr ? aux + coff : in + coff, fs);
        cpx<R> sv[12], xv[12];
#pragma unroll
        for (int c = 0; c < 12; c++) sv[c] = xv[c] = mk<R>(0, 0);
        if (has_self) hload_spinor<R>(rs, cs, 0u, h, sv);
        if (EPI == EPI_RESID || EPI == EPI_DOT_AUX) hload_spinor<R>(rx, cs, 0u, h, xv);
        const int nxt = next_live(col + 1);
        if (nxt < col_hi) issue(nxt);

        cpx<R> a[12];
#pragma unroll
        for (int c = 0; c < 12; c++) a[c] = mk<R>(0, 0);
        if (phb != R(0)) hop_half<R, 0, BW, true>(a, wb[0], hbp, phb);
        if (phf != R(0)) hop_half<R, 0, FW, false>(a, wf[0], hfp, phf);
        cpx<R> hh[6];
        cpx<R> p[12];
        {  // x: same row, pair xh or its neighbour
            const int xp = bo ? (xh + 1 == LH ? 0 : xh + 1) : xh;
            const int xm = bo ? xh : (xh == 0 ? LH - 1 : xh - 1);
#pragma unroll
            for (int c = 0; c < 12; c++) p[c] = s_in[c][r][xp];
            project<R, 1, FW>(p, hh);
            hop_half<R, 1, FW, false>(a, wf[1], hh, R(1));
#pragma unroll
            for (int c = 0; c < 12; c++) p[c] = s_in[c][r][xm];
            project<R, 1, BW>(p, hh);
            hop_half<R, 1, BW, true>(a, wb[1], hh, R(1));
        }
        // y: the adjacent rows of the brick, or the y halo rows
        if (ry + 1 < RY) {
#pragma unroll
            for (int c = 0; c < 12; c++) p[c] = s_in[c][r + 1][xh];
            project<R, 2, FW>(p, hh);
        } else {
#pragma unroll
            for (int k = 0; k < 6; k++) hh[k] = s_h[k][RZ + rz][xh];
        }
        hop_half<R, 2, FW, false>(a, wf[2], hh, R(1));
        if (ry > 0) {
#pragma unroll
            for (int c = 0; c < 12; c++) p[c] = s_in[c][r - 1][xh];
            project<R, 2, BW>(p, hh);
        } else {
#pragma unroll
            for (int k = 0; k < 6; k++) hh[k] = s_h[k][rz][xh];
        }
        hop_half<R, 2, BW, true>(a, wb[2], hh, R(1));
        // z: the brick rows RY apart, or the z halo rows
        if (rz + 1 < RZ) {
#pragma unroll
            for (int c = 0; c < 12; c++) p[c] = s_in[c][r + RY][xh];
            project<R, 3, FW>(p, hh);
        } else {
#pragma unroll
            for (int k = 0; k < 6; k++) hh[k] = s_h[k][2 * RZ + RY + ry][xh];
        }
        hop_half<R, 3, FW, false>(a, wf[3], hh, R(1));
        if (rz > 0) {
#pragma unroll
            for (int c = 0; c < 12; c++) p[c] = s_in[c][r - RY][xh];
            project<R, 3, BW>(p, hh);
        } else {
#pragma unroll
            for (int k = 0; k < 6; k++) hh[k] = s_h[k][2 * RZ + ry][xh];
        }
        hop_half<R, 3, BW, true>(a, wb[3], hh, R(1));

        // epilogue: out = a_self self + c_hop a (or aux - that), fused partial sums
        const rsrc_t ro = make_rsrc(out + coff, fs);
        double d0 = 0, d1 = 0, d2 = 0;
        cpx<R> ov[12];
#pragma unroll
        for (int c = 0; c < 12; c++) {
            const cpx<R> sc = sv[c];
            cpx<R> v = mk<R>(a_self * sc.re + c_hop * a[c].re, a_self * sc.im + c_hop * a[c].im);
            const cpx<R> qv = xv[c];
            if (EPI == EPI_RESID) v = qv - v;
            ov[c] = v;
            if (EPI == EPI_DOT_AUX) {
                d0 += (double)qv.re * v.re + (double)qv.im * v.im;
                d1 += (double)qv.re * v.im - (double)qv.im * v.re;
            } else if (EPI == EPI_TS) {
                d0 += (double)v.re * sc.re + (double)v.im * sc.im;
                d1 += (double)v.re * sc.im - (double)v.im * sc.re;
                d2 += (double)v.re * v.re + (double)v.im * v.im;
            } else if (EPI == EPI_RESID || EPI == EPI_NORM) {
                d0 += (double)v.re * v.re + (double)v.im * v.im;
            }
        }
#pragma unroll
        for (int qq = 0; qq < 6; qq++) hstore_pair<R, NTS>(ro, cs, 0u, h, qq, ov[2 * qq], ov[2 * qq + 1]);
        if (EPI != EPI_STORE) block_sum3<kLdsNT>(d0, d1, d2, partial + ((size_t)col * nblk + blk) * 3);
        __syncthreads();  // the next column's staging overwrites the tile (and the sums' scratch)
        col = nxt;
    }
}

}  // namespace dd
