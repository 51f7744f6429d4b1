// dirac.hip -- Wilson-Dirac stencil on gfx950.
//
// D psi(x) = psi(x)/(2 kappa) - 1/2 sum_mu [ (1-gamma_mu) U_mu(x) psi(x+mu)
//                                          + (1+gamma_mu) U_mu(x-mu)^+ psi(x-mu) ]
// (normalisation 2 kappa D = 1 - kappa D_hop, paper Sec. 5), on the whole lattice
// or on a Dirichlet time slab (paper Sec. 3 Eq. 10: the diagonal block of D; hops
// leaving the slab are dropped).  D^+ = gamma_5 D gamma_5 swaps the projectors.
//
// Mapping: one thread per (site, column); a workgroup covers 256 consecutive
// sites of one column.  Logical workgroups are ordered column-fastest and dealt
// to XCDs in contiguous ranges, so the up-to-12 workgroups that share a site
// block (and its 8 links per site) run on the same XCD and hit its L2 for links
// after the first fetch; neighbour spinors along x, y, z come from the same L2.
// Each neighbour spinor is projected to a half spinor (2 spins x 3 colours)
// before the SU(3) multiply, halving the colour arithmetic.  Site-major SoA
// fields make every component load a coalesced 16-byte (FP64) or 8-byte (FP32)
// access per lane.
#include "dd_internal.h"
#include "dd_wilson.h"

namespace dd {

namespace {

template <typename R, int DAG, int EPI>
__global__ __launch_bounds__(kBlock) void k_dslash(Geo g, const cpx<R>* __restrict__ U, R mass,
                                                   const cpx<R>* __restrict__ in,
                                                   cpx<R>* __restrict__ out,
                                                   const cpx<R>* __restrict__ aux, int ncol,
                                                   int nsb, double* __restrict__ partial,
                                                   const ColState* __restrict__ st) {
    const int lb = xcd_remap(blockIdx.x, gridDim.x);
    const int col = lb % ncol, sb = lb / ncol;
    if (st != nullptr && !st[col].active) return;  // uniform over the workgroup
    const int s = sb * kBlock + threadIdx.x;
    const int nsite = g.nsite;
    const size_t off = (size_t)col * 12 * nsite;
    const cpx<R>* __restrict__ f = in + off;
    double d0 = 0, d1 = 0, d2 = 0;

    if (s < nsite) {
        const int L = g.L, L2 = g.L2, L3 = g.L3;
        const int tl = s / L3;
        const int sp = s - tl * L3;
        const int x = sp % L, yz = sp / L;
        const int y = yz % L, z = yz / L;
        int tg = g.t0 + tl;
        if (tg >= g.T) tg -= g.T;
        const int sl = tg * L3 + sp;  // global site (links)
        constexpr int FW = DAG ? +1 : -1;  // forward hop projector (1 + FW gamma)
        constexpr int BW = -FW;

        cpx<R> a[12];
#pragma unroll
        for (int c = 0; c < 12; c++) a[c] = mk<R>(0, 0);

        // time
        {
            const bool end = (tl == g.nt - 1);
            if (!end || g.whole) {
                const R ph = (tg == g.T - 1) ? R(g.bc) : R(1);
                if (ph != R(0)) {
                    const int nb = end ? s - (g.nt - 1) * L3 : s + L3;
                    hop<R, 0, FW, false>(a, f, nsite, nb, U, g.vlink, sl, ph);
                }
            }
            const bool beg = (tl == 0);
            if (!beg || g.whole) {
                const R ph = (tg == 0) ? R(g.bc) : R(1);
                if (ph != R(0)) {
                    const int nb = beg ? s + (g.nt - 1) * L3 : s - L3;
                    const int slm = (tg == 0 ? g.T - 1 : tg - 1) * L3 + sp;
                    hop<R, 0, BW, true>(a, f, nsite, nb, U, g.vlink, slm, ph);
                }
            }
        }
        // x
        {
            const int dp = (x == L - 1) ? -(L - 1) : 1, dm = (x == 0) ? (L - 1) : -1;
            hop<R, 1, FW, false>(a, f, nsite, s + dp, U, g.vlink, sl, R(1));
            hop<R, 1, BW, true>(a, f, nsite, s + dm, U, g.vlink, sl + dm, R(1));
        }
        // y
        {
            const int dp = (y == L - 1) ? -(L - 1) * L : L, dm = (y == 0) ? (L - 1) * L : -L;
            hop<R, 2, FW, false>(a, f, nsite, s + dp, U, g.vlink, sl, R(1));
            hop<R, 2, BW, true>(a, f, nsite, s + dm, U, g.vlink, sl + dm, R(1));
        }
        // z
        {
            const int dp = (z == L - 1) ? -(L - 1) * L2 : L2, dm = (z == 0) ? (L - 1) * L2 : -L2;
            hop<R, 3, FW, false>(a, f, nsite, s + dp, U, g.vlink, sl, R(1));
            hop<R, 3, BW, true>(a, f, nsite, s + dm, U, g.vlink, sl + dm, R(1));
        }

        cpx<R>* __restrict__ o = out + off;
        const R half = R(0.5);
#pragma unroll
        for (int c = 0; c < 12; c++) {
            const cpx<R> pc = f[c * nsite + s];
            cpx<R> r = mk<R>(mass * pc.re - half * a[c].re, mass * pc.im - half * a[c].im);
            if (EPI == EPI_RESID) r = aux[off + c * nsite + s] - r;
            o[c * nsite + s] = r;
            if (EPI == EPI_DOT_AUX) {
                const cpx<R> q = aux[off + c * nsite + s];
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
    if (EPI != EPI_STORE) block_sum3(d0, d1, d2, partial + ((size_t)col * nsb + sb) * 3);
}

template <typename R, int DAG>
void launch_epi(dd_ctx* c, int epi, dim3 grid, const Geo& g, const cpx<R>* U, R mass,
                const cpx<R>* in, cpx<R>* out, const cpx<R>* aux, int ncol, int nsb,
                double* partial, const ColState* st) {
    switch (epi) {
        case EPI_STORE:
            hipLaunchKernelGGL((k_dslash<R, DAG, EPI_STORE>), grid, dim3(kBlock), 0, c->stream, g, U,
                               mass, in, out, aux, ncol, nsb, partial, st);
            break;
        case EPI_DOT_AUX:
            hipLaunchKernelGGL((k_dslash<R, DAG, EPI_DOT_AUX>), grid, dim3(kBlock), 0, c->stream, g,
                               U, mass, in, out, aux, ncol, nsb, partial, st);
            break;
        case EPI_TS:
            hipLaunchKernelGGL((k_dslash<R, DAG, EPI_TS>), grid, dim3(kBlock), 0, c->stream, g, U,
                               mass, in, out, aux, ncol, nsb, partial, st);
            break;
        case EPI_RESID:
            hipLaunchKernelGGL((k_dslash<R, DAG, EPI_RESID>), grid, dim3(kBlock), 0, c->stream, g, U,
                               mass, in, out, aux, ncol, nsb, partial, st);
            break;
        default:
            hipLaunchKernelGGL((k_dslash<R, DAG, EPI_NORM>), grid, dim3(kBlock), 0, c->stream, g, U,
                               mass, in, out, aux, ncol, nsb, partial, st);
            break;
    }
}

}  // namespace

template <typename R>
void launch_dslash(dd_ctx* c, const Geo& g, const cpx<R>* U, double kappa, int dag, int epi,
                   const cpx<R>* in, cpx<R>* out, const cpx<R>* aux, int ncol, double* partial,
                   const ColState* st) {
    const int nsb = site_blocks(g.nsite);
    const dim3 grid((unsigned)nsb * (unsigned)ncol);
    const R mass = R(1.0 / (2.0 * kappa));
    hipEvent_t ev = nullptr;
    if (c->timing) timing_begin(c, &ev);
    if (dag)
        launch_epi<R, 1>(c, epi, grid, g, U, mass, in, out, aux, ncol, nsb, partial, st);
    else
        launch_epi<R, 0>(c, epi, grid, g, U, mass, in, out, aux, ncol, nsb, partial, st);
    if (c->timing) {
        const double extra = (epi == EPI_DOT_AUX || epi == EPI_RESID) ? 24.0 : 0.0;
        const double bytes = (double)g.nsite * ((48.0 + extra) * ncol + 72.0) * sizeof(R);
        timing_end(c, ev, sizeof(R) == 8 ? 0 : 1, bytes);
    }
}

template void launch_dslash<double>(dd_ctx*, const Geo&, const cpx<double>*, double, int, int,
                                    const cpx<double>*, cpx<double>*, const cpx<double>*, int,
                                    double*, const ColState*);
template void launch_dslash<float>(dd_ctx*, const Geo&, const cpx<float>*, double, int, int,
                                   const cpx<float>*, cpx<float>*, const cpx<float>*, int, double*,
                                   const ColState*);

}  // namespace dd
