// dirac.hip -- Wilson-Dirac stencil launches on one lattice or slab (the
// arithmetic lives in dd_dslash.h).
//
// Mapping: one workgroup per tile of NT spatial sites x one time chunk x one
// column.  The launch shape (workgroup size, chunk length, XCD remap) comes
// from a per-context autotuner keyed by precision, column count and geometry.
#include "dd_dslash.h"

namespace dd {

namespace {

// Workgroup index -> (group of KC columns fastest, spatial block, time chunk),
// optionally remapped so that each XCD takes a contiguous range of workgroups.
// ncol is a multiple of KC; the workgroup runs while one column of its group is
// active (a stopped column keeps its output).  XS: the x hops through lane
// permutes (whole x rows per wavefront, see dd_dslash.h).
// The XS form in FP32 with two columns per thread is held to two waves per SIMD (256
// registers), where the loading form stores through its epilogue without the bound.
template <typename R, int DAG, int EPI, int NT, int KC, bool XS>
__global__ __launch_bounds__(NT, (sizeof(R) == 4 && KC == 2 && XS) ? 2 : sweep_waves<R>()) void k_dslash(Geo g, const cpx<R>* __restrict__ U, R mass,
                                               const cpx<R>* __restrict__ in, cpx<R>* __restrict__ out,
                                               const cpx<R>* __restrict__ aux, int ncol, int tc_len,
                                               int remap, int blocked, double* __restrict__ partial,
                                               const ColState* __restrict__ st) {
    const int lb = remap ? xcd_remap(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    const int nsb = (g.L3 + NT - 1) / NT;
    const int ngrp = ncol / KC;
    const int col = (lb % ngrp) * KC;
    const int rest = lb / ngrp;
    const int nchunk = gridDim.x / (ngrp * nsb);
    // tile flag bit 1: the time chunks of one tile in adjacent workgroups (the slices either side
    // of a chunk, which the neighbouring chunks read too, are still in L2); otherwise the tiles
    // of one chunk are adjacent
    const bool chunk_major = (blocked & 2) != 0;
    const int sb = chunk_major ? rest / nchunk : rest % nsb;
    const int tc = chunk_major ? rest % nchunk : rest / nsb;
    unsigned live = 0;
#pragma unroll
    for (int k = 0; k < KC; k++)
        if (st == nullptr || st[col + k].active) live |= 1u << k;
    if (live == 0) return;  // uniform over the workgroup
    const size_t off = (size_t)col * 12 * g.nsite;
    double* slot = partial + ((size_t)col * nsb * nchunk + (size_t)tc * nsb + sb) * 3;
    dslash_tile_cols<R, DAG, EPI, NT, KC, XS>(g, U, mass, in + off, out + off, aux != nullptr ? aux + off : nullptr,
                                          live, sb, tc, tc_len, slot, (size_t)nsb * nchunk, (blocked & 1) != 0,
                                          blocked >> 8);
}

template <typename R, int DAG, int NT, int KC, bool XS>
void launch_epi(dd_ctx* c, int epi, dim3 grid, const Geo& g, const cpx<R>* U, R mass,
                const cpx<R>* in, cpx<R>* out, const cpx<R>* aux, int ncol, int tc, int remap, int blocked,
                double* partial, const ColState* st) {
#define DD_EPI_CASE(E)                                                                                               \
    hipLaunchKernelGGL((k_dslash<R, DAG, E, NT, KC, XS>), grid, dim3(NT), 0, c->stream, g, U, mass, in, out, aux, ncol, \
                       tc, remap, blocked, partial, st)
    switch (epi) {
        case EPI_STORE: DD_EPI_CASE(EPI_STORE); break;
        case EPI_DOT_AUX: DD_EPI_CASE(EPI_DOT_AUX); break;
        case EPI_TS: DD_EPI_CASE(EPI_TS); break;
        case EPI_RESID: DD_EPI_CASE(EPI_RESID); break;
        case EPI_HOP: DD_EPI_CASE(EPI_HOP); break;
        default: DD_EPI_CASE(EPI_NORM); break;
    }
#undef DD_EPI_CASE
}

template <typename R, int DAG, int NT, bool XS>
void launch_kc(dd_ctx* c, int kc, int epi, dim3 grid, const Geo& g, const cpx<R>* U, R mass, const cpx<R>* in,
               cpx<R>* out, const cpx<R>* aux, int ncol, int tc, int remap, int blocked, double* partial,
               const ColState* st) {
    if (kc == 2) {
        launch_epi<R, DAG, NT, 2, XS>(c, epi, grid, g, U, mass, in, out, aux, ncol, tc, remap, blocked, partial, st);
        return;
    }
    if constexpr (sizeof(R) == 4) {
        if (kc == 3) {
            launch_epi<R, DAG, NT, 3, XS>(c, epi, grid, g, U, mass, in, out, aux, ncol, tc, remap, blocked, partial, st);
            return;
        }
        if (kc == 4) {
            launch_epi<R, DAG, NT, 4, XS>(c, epi, grid, g, U, mass, in, out, aux, ncol, tc, remap, blocked, partial, st);
            return;
        }
    }
    launch_epi<R, DAG, NT, 1, XS>(c, epi, grid, g, U, mass, in, out, aux, ncol, tc, remap, blocked, partial, st);
}

}  // namespace

// Columns per thread of a launch: the tuned count when it is built for the
// precision (FP32 up to 4; FP64 up to 2, where three columns no longer fit the
// register file), divides ncol and the column group fits one 32-bit buffer
// range, else 1.
int sched_kc(const StencilSched& sc, int ncol, size_t real_bytes, size_t col_bytes) {
    const int kc = sc.kc;
    if (kc <= 1 || kc > (real_bytes == 8 ? 2 : 4) || ncol % kc != 0) return 1;
    if ((size_t)kc * col_bytes >= ((size_t)1 << 32)) return 1;
    return kc;
}

// y rows of a brick tile of nt sites (whole x rows, ry x nt / (L ry) rows in (y, z)), or 0
// where bricks do not fit: nt a multiple of L, the rows split as evenly as possible with
// ry <= 4, and both extents dividing L.
int brick_rows(const Geo& g, int nt) {
    const int L = g.L;
    if (nt % L != 0) return 0;
    const int rows = nt / L;
    if (rows < 2) return 0;
    const int ry = rows >= 16 ? 4 : (rows >= 4 ? (rows >= 8 ? 4 : 2) : rows);
    const int rz = rows / ry;
    if (ry * rz != rows || L % ry != 0 || L % rz != 0) return 0;
    return ry;
}

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
    const int kc = sched_kc(sc, ncol, sizeof(R), (size_t)12 * g.nsite * sizeof(cpx<R>));
    const dim3 grid((unsigned)stencil_blocks(g, sc) * (unsigned)(ncol / kc));
    // tile flags as the kernel reads them: bit 0 bricks (with the brick's y rows in bits 8+),
    // bit 1 chunk-adjacent order
    const int ry = brick_rows(g, sc.nt);
    const int blk = ((sc.blocked & 1) && ry > 0 ? 1 | (ry << 8) : 0) | (sc.blocked & 2);
    const R mass = R(epi == EPI_HOP ? kappa : 1.0 / (2.0 * kappa));  // EPI_HOP scales the hop by kappa
    // x hops through lane permutes where every wavefront holds whole x rows (NT is 128 or 256),
    // unless tile flag bit 2 asks for the loading form (never set by the tuner)
    const bool xs = g.L >= 4 && kWave % g.L == 0 && (sc.blocked & 4) == 0;
    hipEvent_t ev = nullptr;
    if (c->timing) timing_begin(c, &ev);
#define DD_KC_CASE(DAGV, NTV, XSV) \
    launch_kc<R, DAGV, NTV, XSV>(c, kc, epi, grid, g, U, mass, in, out, aux, ncol, sc.tc, sc.remap, blk, partial, st)
#define DD_NT_CASE(NTV)                                  \
    if (dag) {                                           \
        if (xs) DD_KC_CASE(1, NTV, true);                \
        else DD_KC_CASE(1, NTV, false);                  \
    } else {                                             \
        if (xs) DD_KC_CASE(0, NTV, true);                \
        else DD_KC_CASE(0, NTV, false);                  \
    }
    if (sc.nt == 256) {
        DD_NT_CASE(256)
    } else {
        DD_NT_CASE(128)
    }
#undef DD_NT_CASE
#undef DD_KC_CASE
    if (c->timing) {
        const double extra = (epi == EPI_DOT_AUX || epi == EPI_RESID) ? 24.0 : 0.0;
        const double bytes = (double)g.nsite * ((48.0 + extra) * ncol * c->bill_frac + 72.0) * sizeof(R);
        const std::string name = std::string("k_dslash<") + (sizeof(R) == 8 ? "double" : "float") + ", " +
                                 std::to_string(dag ? 1 : 0) + ", " + std::to_string(epi) + ", " +
                                 std::to_string(sc.nt) + (kc > 1 ? ", " + std::to_string(kc) : std::string()) + ">";
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
