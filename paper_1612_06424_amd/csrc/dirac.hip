// dirac.hip -- Wilson-Dirac stencil on gfx950.
//
// D psi(x) = psi(x)/(2 kappa) - 1/2 sum_mu [ (1-gamma_mu) U_mu(x) psi(x+mu)
//                                          + (1+gamma_mu) U_mu(x-mu)^+ psi(x-mu) ]
// (normalisation 2 kappa D = 1 - kappa D_hop, paper Sec. 5), on the whole lattice
// or on a Dirichlet time slab (paper Sec. 3 Eq. 10: the diagonal block of D; hops
// leaving the slab are dropped).  D^+ = gamma_5 D gamma_5 swaps the projectors.
//
// Mapping: a thread owns one spatial site of one column and sweeps a chunk of
// time slices (see k_dslash); workgroups of 128 or 256 consecutive spatial
// sites.  The launch shape (workgroup size, chunk length, XCD remap) comes from
// a per-context autotuner keyed by precision, column count and geometry.
// Each neighbour spinor is projected to a half spinor (2 spins x 3 colours)
// before the SU(3) multiply, halving the colour arithmetic.  Site-major SoA
// fields make every component load a coalesced 16-byte (FP64) or 8-byte (FP32)
// access per lane, all through raw buffer resources.
#include "dd_internal.h"
#include "dd_wilson.h"

namespace dd {

namespace {

// Time-sweep stencil.  A thread owns one spatial site of one column and walks
// a chunk of tc time slices.  psi(t) and the transported backward half spinor
// U_0(t)^+ P_+ psi(t) are carried in registers from one slice to the next, so
// the time neighbours and the backward time link are fetched exactly once;
// the spatial neighbours of slice t are fetched by the threads that own them
// at about the same moment and are served from L1 / L2.
//
// Workgroup index -> (column fastest, spatial block, time chunk), optionally
// remapped so that each XCD takes a contiguous range of workgroups.
template <typename R, int DAG, int EPI, int NT>
__global__ __launch_bounds__(NT) void k_dslash(Geo g, const cpx<R>* __restrict__ U, R mass,
                                               const cpx<R>* __restrict__ in, cpx<R>* __restrict__ out,
                                               const cpx<R>* __restrict__ aux, int ncol, int tc_len,
                                               int remap, double* __restrict__ partial,
                                               const ColState* __restrict__ st) {
    const int lb = remap ? xcd_remap(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    const int L = g.L, L2 = g.L2, L3 = g.L3;
    const int nsb = (L3 + NT - 1) / NT;
    const int col = lb % ncol;
    const int rest = lb / ncol;
    const int sb = rest % nsb, tc = rest / nsb;
    if (st != nullptr && !st[col].active) return;  // uniform over the workgroup
    const int nchunk = gridDim.x / (ncol * nsb);
    const int sp = sb * NT + threadIdx.x;
    const int nsite = g.nsite, nt = g.nt;
    const size_t off = (size_t)col * 12 * nsite;
    constexpr uint32_t CB = sizeof(cpx<R>);
    const uint32_t cs = (uint32_t)nsite * CB;    // component stride (bytes)
    const uint32_t ls = (uint32_t)g.vlink * CB;  // link-row stride (bytes)
    constexpr int FW = DAG ? +1 : -1;            // forward hop projector (1 + FW gamma)
    constexpr int BW = -FW;
    double d0 = 0, d1 = 0, d2 = 0;

    if (sp < L3) {
        const rsrc_t rf = make_rsrc(in + off, 12u * cs);
        const rsrc_t ro = make_rsrc(out + off, 12u * cs);
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
        const rsrc_t rx = (EPI == EPI_RESID || EPI == EPI_DOT_AUX) ? make_rsrc(aux + off, 12u * cs) : rf;
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
                cpx<R> r = mk<R>(mass * pc.re - half * a[c].re, mass * pc.im - half * a[c].im);
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
    if (EPI != EPI_STORE)
        block_sum3<NT>(d0, d1, d2, partial + ((size_t)col * nsb * nchunk + (size_t)tc * nsb + sb) * 3);
}

template <typename R, int DAG, int NT>
void launch_epi(dd_ctx* c, int epi, dim3 grid, const Geo& g, const cpx<R>* U, R mass,
                const cpx<R>* in, cpx<R>* out, const cpx<R>* aux, int ncol, int tc, int remap,
                double* partial, const ColState* st) {
    switch (epi) {
        case EPI_STORE:
            hipLaunchKernelGGL((k_dslash<R, DAG, EPI_STORE, NT>), grid, dim3(NT), 0, c->stream, g, U, mass, in,
                               out, aux, ncol, tc, remap, partial, st);
            break;
        case EPI_DOT_AUX:
            hipLaunchKernelGGL((k_dslash<R, DAG, EPI_DOT_AUX, NT>), grid, dim3(NT), 0, c->stream, g, U, mass, in,
                               out, aux, ncol, tc, remap, partial, st);
            break;
        case EPI_TS:
            hipLaunchKernelGGL((k_dslash<R, DAG, EPI_TS, NT>), grid, dim3(NT), 0, c->stream, g, U, mass, in, out,
                               aux, ncol, tc, remap, partial, st);
            break;
        case EPI_RESID:
            hipLaunchKernelGGL((k_dslash<R, DAG, EPI_RESID, NT>), grid, dim3(NT), 0, c->stream, g, U, mass, in,
                               out, aux, ncol, tc, remap, partial, st);
            break;
        default:
            hipLaunchKernelGGL((k_dslash<R, DAG, EPI_NORM, NT>), grid, dim3(NT), 0, c->stream, g, U, mass, in,
                               out, aux, ncol, tc, remap, partial, st);
            break;
    }
}

}  // namespace

StencilSched default_sched(const Geo& g) {
    StencilSched sc;
    sc.nt = 128;
    sc.tc = g.nt < 8 ? g.nt : 8;
    sc.remap = 0;
    return sc;
}

int stencil_blocks(const Geo& g, const StencilSched& sc) {
    const int nsb = (g.L3 + sc.nt - 1) / sc.nt;
    const int nchunk = (g.nt + sc.tc - 1) / sc.tc;
    return nsb * nchunk;
}

template <typename R>
void launch_dslash_sched(dd_ctx* c, const Geo& g, const StencilSched& sc, const cpx<R>* U, double kappa,
                         int dag, int epi, const cpx<R>* in, cpx<R>* out, const cpx<R>* aux, int ncol,
                         double* partial, const ColState* st) {
    const dim3 grid((unsigned)stencil_blocks(g, sc) * (unsigned)ncol);
    const R mass = R(1.0 / (2.0 * kappa));
    hipEvent_t ev = nullptr;
    if (c->timing) timing_begin(c, &ev);
#define DD_NT_CASE(NTV)                                                                                     \
    if (dag)                                                                                                \
        launch_epi<R, 1, NTV>(c, epi, grid, g, U, mass, in, out, aux, ncol, sc.tc, sc.remap, partial, st); \
    else                                                                                                    \
        launch_epi<R, 0, NTV>(c, epi, grid, g, U, mass, in, out, aux, ncol, sc.tc, sc.remap, partial, st);
    if (sc.nt == 256) {
        DD_NT_CASE(256)
    } else {
        DD_NT_CASE(128)
    }
#undef DD_NT_CASE
    if (c->timing) {
        const double extra = (epi == EPI_DOT_AUX || epi == EPI_RESID) ? 24.0 : 0.0;
        const double bytes = (double)g.nsite * ((48.0 + extra) * ncol + 72.0) * sizeof(R);
        const std::string name = std::string("k_dslash<") + (sizeof(R) == 8 ? "double" : "float") + ", " +
                                 std::to_string(dag ? 1 : 0) + ", " + std::to_string(epi) + ", " +
                                 std::to_string(sc.nt) + ">";
        timing_end(c, ev, name, bytes);
    }
}

template <typename R>
void launch_dslash(dd_ctx* c, const Geo& g, const cpx<R>* U, double kappa, int dag, int epi,
                   const cpx<R>* in, cpx<R>* out, const cpx<R>* aux, int ncol, double* partial,
                   const ColState* st) {
    launch_dslash_sched<R>(c, g, stencil_sched(c, g, sizeof(R) == 8 ? 0 : 1, ncol), U, kappa, dag, epi, in, out,
                           aux, ncol, partial, st);
}

template void launch_dslash<double>(dd_ctx*, const Geo&, const cpx<double>*, double, int, int,
                                    const cpx<double>*, cpx<double>*, const cpx<double>*, int,
                                    double*, const ColState*);
template void launch_dslash<float>(dd_ctx*, const Geo&, const cpx<float>*, double, int, int,
                                   const cpx<float>*, cpx<float>*, const cpx<float>*, int, double*,
                                   const ColState*);
template void launch_dslash_sched<double>(dd_ctx*, const Geo&, const StencilSched&, const cpx<double>*, double,
                                          int, int, const cpx<double>*, cpx<double>*, const cpx<double>*, int,
                                          double*, const ColState*);
template void launch_dslash_sched<float>(dd_ctx*, const Geo&, const StencilSched&, const cpx<float>*, double,
                                         int, int, const cpx<float>*, cpx<float>*, const cpx<float>*, int, double*,
                                         const ColState*);

}  // namespace dd
