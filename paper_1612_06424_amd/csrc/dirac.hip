// dirac.hip -- Wilson-Dirac stencil launches on one lattice or slab (the
// arithmetic lives in dd_dslash.h).
//
// Mapping: one workgroup per tile of NT spatial sites x one time chunk x one
// column.  The launch shape (workgroup size, chunk length, XCD remap) comes
// from a per-context autotuner keyed by precision, column count and geometry.
#include "dd_dslash.h"

namespace dd {

namespace {

// Workgroup index -> (column fastest, spatial block, time chunk), optionally
// remapped so that each XCD takes a contiguous range of workgroups.
template <typename R, int DAG, int EPI, int NT>
__global__ __launch_bounds__(NT, sweep_waves<R>()) void k_dslash(Geo g, const cpx<R>* __restrict__ U, R mass,
                                               const cpx<R>* __restrict__ in, cpx<R>* __restrict__ out,
                                               const cpx<R>* __restrict__ aux, int ncol, int tc_len,
                                               int remap, double* __restrict__ partial,
                                               const ColState* __restrict__ st) {
    const int lb = remap ? xcd_remap(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    const int nsb = (g.L3 + NT - 1) / NT;
    const int col = lb % ncol;
    const int rest = lb / ncol;
    const int sb = rest % nsb, tc = rest / nsb;
    if (st != nullptr && !st[col].active) return;  // uniform over the workgroup
    const int nchunk = gridDim.x / (ncol * nsb);
    const size_t off = (size_t)col * 12 * g.nsite;
    double* slot = partial + ((size_t)col * nsb * nchunk + (size_t)tc * nsb + sb) * 3;
    dslash_tile<R, DAG, EPI, NT>(g, U, mass, in + off, out + off, aux != nullptr ? aux + off : nullptr, sb, tc,
                                 tc_len, slot);
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
        case EPI_HOP:
            hipLaunchKernelGGL((k_dslash<R, DAG, EPI_HOP, NT>), grid, dim3(NT), 0, c->stream, g, U, mass, in,
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
    const R mass = R(epi == EPI_HOP ? kappa : 1.0 / (2.0 * kappa));  // EPI_HOP scales the hop by kappa
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
        const double bytes = (double)g.nsite * ((48.0 + extra) * ncol * c->bill_frac + 72.0) * sizeof(R);
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
