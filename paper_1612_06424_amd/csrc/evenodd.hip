// evenodd.hip -- even-odd preconditioned solves on one lattice or slab.
//
// D x = b (or D^+ x = b) is solved through the Schur complement on the even
// sites (dd_eo.h): the source is prepared with one half hop, the reliable-
// update Krylov solver of solver.hip runs on the half fields with
// Dhat = m - (1/(4m)) H_eo H_oe applied as two half hops, the odd half is
// reconstructed with one more half hop, and the answer is checked against the
// full operator (true FP64 residual |b - D x| / |b|).  Since the full residual
// equals the Schur residual on the even sites, the Schur solve converges on
// |b_e' - Dhat x_e| <= tol |b| (the norm of the original source).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "dd_eo.h"
#include "dd_eo_lds.h"

namespace dd {

namespace {

// Workgroup -> (group of KC columns fastest, tile of NT pairs of a slice, chunk
// of tc_len slices); partial slot of (col, block) = col * nblk + block.  ncol is
// a multiple of KC.  REC: U holds two rows per link (KC > 1 only).
template <typename R, int DAG, int EPI, int NT, bool SELF, int KC, bool REC, bool NTS>
__device__ __forceinline__ void eo_hop_body(const Geo& g, const cpx<R>* __restrict__ U, R a_self, R c_hop, int p_out,
                                            const cpx<R>* __restrict__ in, const cpx<R>* __restrict__ self,
                                            cpx<R>* __restrict__ out, const cpx<R>* __restrict__ aux, int ncol,
                                            int tc_len, int remap, int blocked, double* __restrict__ partial,
                                            const ColState* __restrict__ st) {
    const int lb = remap ? xcd_remap(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    const int ngrp = ncol / KC;
    const int col0 = (lb % ngrp) * KC, blk = lb / ngrp;
    unsigned live = 0;  // active columns of the group; the workgroup runs while one is
#pragma unroll
    for (int k = 0; k < KC; k++)
        if (st == nullptr || st[col0 + k].active) live |= 1u << k;
    if (live == 0) return;  // uniform over the workgroup
    const int nblk = (int)gridDim.x / ngrp;
    const int ntile = ((g.L3 >> 1) + NT - 1) / NT;
    const int nchunk = nblk / ntile;
    // bit 1 of the tile flags: the time chunks of one tile are adjacent workgroups (the
    // slice either side of a chunk, which its neighbour chunks read too, stays in L2);
    // otherwise the tiles of one chunk are
    const bool chunk_major = (blocked & 2) != 0;
    const int tile = chunk_major ? blk / nchunk : blk % ntile;
    const int chunk = chunk_major ? blk % nchunk : blk / ntile;
    const int bricks = blocked & 1;
    const size_t off = (size_t)col0 * 12 * (size_t)(g.nsite >> 1);
    double* slot = partial + ((size_t)col0 * nblk + blk) * 3;
    if constexpr (KC == 1)
        eo_sweep_tile<R, DAG, EPI, NT, SELF>(g, U, a_self, c_hop, p_out, in + off,
                                             self != nullptr ? self + off : nullptr, out + off,
                                             aux != nullptr ? aux + off : nullptr, tile, chunk, tc_len, bricks, slot);
    else
        eo_sweep_cols<R, DAG, EPI, NT, SELF, KC, REC, NTS>(g, U, a_self, c_hop, p_out, in + off,
                                                      self != nullptr ? self + off : nullptr, out + off,
                                                      aux != nullptr ? aux + off : nullptr, live, tile, chunk, tc_len,
                                                      bricks, slot, (size_t)nblk);
}

template <typename R, int DAG, int EPI, int NT, bool SELF, int KC, bool REC>
__global__ __launch_bounds__(NT, eo_waves<R>()) void k_eo_hop(Geo g, const cpx<R>* __restrict__ U, R a_self,
                                                             R c_hop, int p_out, const cpx<R>* __restrict__ in,
                                                             const cpx<R>* __restrict__ self,
                                                             cpx<R>* __restrict__ out, const cpx<R>* __restrict__ aux,
                                                             int ncol, int tc_len, int remap, int blocked,
                                                             double* __restrict__ partial,
                                                             const ColState* __restrict__ st) {
    eo_hop_body<R, DAG, EPI, NT, SELF, KC, REC, false>(g, U, a_self, c_hop, p_out, in, self, out, aux, ncol, tc_len,
                                                       remap, blocked, partial, st);
}

// The same half hop with non-temporal output stores (KC > 1).
template <typename R, int DAG, int EPI, int NT, bool SELF, int KC, bool REC>
__global__ __launch_bounds__(NT, eo_waves<R>()) void k_eo_hop_nt(Geo g, const cpx<R>* __restrict__ U, R a_self,
                                                                R c_hop, int p_out, const cpx<R>* __restrict__ in,
                                                                const cpx<R>* __restrict__ self,
                                                                cpx<R>* __restrict__ out,
                                                                const cpx<R>* __restrict__ aux, int ncol, int tc_len,
                                                                int remap, int blocked, double* __restrict__ partial,
                                                                const ColState* __restrict__ st) {
    eo_hop_body<R, DAG, EPI, NT, SELF, KC, REC, true>(g, U, a_self, c_hop, p_out, in, self, out, aux, ncol, tc_len,
                                                      remap, blocked, partial, st);
}

// The LDS-tile form of the half hop (dd_eo_lds.h): one slice of a brick of rows per
// workgroup, cpw columns per workgroup, links of two rows each (SU(3)).
template <typename R, int DAG, int EPI, bool SELF, int LH, bool NTS>
__global__ __launch_bounds__(kLdsNT, 1) void k_eo_lds(Geo g, const cpx<R>* __restrict__ U12, R a_self, R c_hop,
                                                     int p_out, const cpx<R>* __restrict__ in,
                                                     const cpx<R>* __restrict__ self, cpx<R>* __restrict__ out,
                                                     const cpx<R>* __restrict__ aux, int ncol, int cpw, int remap,
                                                     double* __restrict__ partial, const ColState* __restrict__ st) {
    eo_lds_body<R, DAG, EPI, SELF, LH, NTS>(g, U12, a_self, c_hop, p_out, in, self, out, aux, ncol, cpw, remap,
                                            partial, st);
}

// full field [ncol][12][nsite] <-> even / odd half fields [ncol][12][nsite / 2]
__global__ __launch_bounds__(kBlock) void k_eo_split(Geo g, int ncol, const cpx<double>* __restrict__ full,
                                                     cpx<double>* __restrict__ ev, cpx<double>* __restrict__ od) {
    const size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
    const size_t n = (size_t)ncol * 12 * g.nsite;
    if (i >= n) return;
    const int s = (int)(i % (size_t)g.nsite);
    const size_t row = i / (size_t)g.nsite;  // col * 12 + component
    const int tl = s / g.L3, sp = s - tl * g.L3;
    const int par = (tl + sp % g.L + (sp / g.L) % g.L + sp / g.L2) & 1;
    const size_t j = row * (size_t)(g.nsite >> 1) + (size_t)(s >> 1);
    (par ? od : ev)[j] = full[i];
}
__global__ __launch_bounds__(kBlock) void k_eo_merge(Geo g, int ncol, const cpx<double>* __restrict__ ev,
                                                     const cpx<double>* __restrict__ od,
                                                     cpx<double>* __restrict__ full) {
    const size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
    const size_t n = (size_t)ncol * 12 * g.nsite;
    if (i >= n) return;
    const int s = (int)(i % (size_t)g.nsite);
    const size_t row = i / (size_t)g.nsite;
    const int tl = s / g.L3, sp = s - tl * g.L3;
    const int par = (tl + sp % g.L + (sp / g.L) % g.L + sp / g.L2) & 1;
    const size_t j = row * (size_t)(g.nsite >> 1) + (size_t)(s >> 1);
    full[i] = (par ? od : ev)[j];
}

// Ueo[mu][k][parity][nsite / 2] (precision R) from the lattice links U[mu][k][V]
template <typename R>
__global__ __launch_bounds__(kBlock) void k_links_eo(Geo g, const cpx<double>* __restrict__ U,
                                                     cpx<R>* __restrict__ Ueo) {
    const int s = (int)(blockIdx.x * kBlock + threadIdx.x);
    if (s >= g.nsite) return;
    const int tl = s / g.L3, sp = s - tl * g.L3;
    const int t = g.t0 + tl;
    const size_t sl = (size_t)(t >= g.T ? t - g.T : t) * g.L3 + sp;
    const int par = (tl + sp % g.L + (sp / g.L) % g.L + sp / g.L2) & 1;
    const size_t nh = (size_t)(g.nsite >> 1);
    for (int row = 0; row < 36; row++) {
        const cpx<double> v = U[(size_t)row * g.vlink + sl];
        Ueo[((size_t)row * 2 + par) * nh + (size_t)(s >> 1)] = cpx<R>{(R)v.re, (R)v.im};
    }
}

// Ueo12[mu][k / 2][parity][nsite / 2][k & 1], k < 6: rows 0 and 1 of every link in FP32,
// entries paired in 16-byte units (dd_eo.h, rec_link_base);
// dev[block] = the largest difference (FP64, max norm) between a link's third
// row and the conjugated cross product of its first two, over the block's
// sites (NaN if any entry is not finite)
__global__ __launch_bounds__(kBlock) void k_links_eo12(Geo g, const cpx<double>* __restrict__ U,
                                                       cpx<float>* __restrict__ Ueo, double* __restrict__ dev) {
    const int s = (int)(blockIdx.x * kBlock + threadIdx.x);
    double d = 0;
    auto worse = [](double a, double b) { return (b > a || b != b) ? b : a; };
    if (s < g.nsite) {
        const int tl = s / g.L3, sp = s - tl * g.L3;
        const int t = g.t0 + tl;
        const size_t sl = (size_t)(t >= g.T ? t - g.T : t) * g.L3 + sp;
        const int par = (tl + sp % g.L + (sp / g.L) % g.L + sp / g.L2) & 1;
        const size_t nh = (size_t)(g.nsite >> 1);
        for (int mu = 0; mu < 4; mu++) {
            cpx<double> w[9];
            for (int k = 0; k < 9; k++) w[k] = U[(size_t)(mu * 9 + k) * g.vlink + sl];
            for (int k = 0; k < 6; k++)
                Ueo[((((size_t)(mu * 3 + k / 2) * 2 + par) * nh + (size_t)(s >> 1)) << 1) + (k & 1)] =
                    cpx<float>{(float)w[k].re, (float)w[k].im};
            const cpx<double> c[3] = {w[1] * w[5] - w[2] * w[4], w[2] * w[3] - w[0] * w[5], w[0] * w[4] - w[1] * w[3]};
            for (int k = 0; k < 3; k++) {
                d = worse(d, fabs(w[6 + k].re - c[k].re));
                d = worse(d, fabs(w[6 + k].im + c[k].im));
            }
        }
    }
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) d = worse(d, __shfl_xor(d, off, kWave));
    __shared__ double sh[kBlock / kWave];
    if (threadIdx.x % kWave == 0) sh[threadIdx.x / kWave] = d;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = sh[0];
        for (int k = 1; k < kBlock / kWave; k++) m = worse(m, sh[k]);
        dev[blockIdx.x] = m;
    }
}

constexpr int kEoNT = 256;

// workgroups per column: tiles of kEoNT pairs per slice x chunks of tc slices
int eo_blocks(const Geo& g, int tc) { return (((g.L3 >> 1) + kEoNT - 1) / kEoNT) * ((g.nt + tc - 1) / tc); }

template <typename R, int DAG, bool SELF, int KC, bool REC, bool NTS>
void launch_eo_epi(hipStream_t s, int epi, dim3 grid, const Geo& g, const cpx<R>* U, R a_self, R c_hop, int p_out,
                   const cpx<R>* in, const cpx<R>* self, cpx<R>* out, const cpx<R>* aux, int ncol, int tc,
                   int remap, int blocked, double* partial, const ColState* st) {
    const dim3 block(kEoNT);
#define DD_EO_CASE(E)                                                                                              \
    if constexpr (NTS)                                                                                             \
        hipLaunchKernelGGL((k_eo_hop_nt<R, DAG, E, kEoNT, SELF, KC, REC>), grid, block, 0, s, g, U, a_self, c_hop, \
                           p_out, in, self, out, aux, ncol, tc, remap, blocked, partial, st);                      \
    else                                                                                                           \
        hipLaunchKernelGGL((k_eo_hop<R, DAG, E, kEoNT, SELF, KC, REC>), grid, block, 0, s, g, U, a_self, c_hop,    \
                           p_out, in, self, out, aux, ncol, tc, remap, blocked, partial, st)
    switch (epi) {
        case EPI_STORE: DD_EO_CASE(EPI_STORE); break;
        case EPI_DOT_AUX: DD_EO_CASE(EPI_DOT_AUX); break;
        case EPI_TS: DD_EO_CASE(EPI_TS); break;
        case EPI_RESID: DD_EO_CASE(EPI_RESID); break;
        default: DD_EO_CASE(EPI_NORM); break;
    }
#undef DD_EO_CASE
}

// Columns per thread of the half-hop sweep that a launch may use: FP32 shares
// each link load between 2 columns (221 VGPRs, two waves per SIMD; 4 columns
// need AGPRs and were never faster); FP64 already needs the whole register
// file for one.
template <typename R>
bool eo_kc_ok(int kc, int ncol) {
    if (sizeof(R) == 8) return kc == 1;
    return (kc == 1 || kc == 2) && ncol % kc == 0;
}

template <typename R, int D, bool SF>
void launch_eo_kc(hipStream_t s, int kc, bool rec, bool nts, int epi, dim3 grid, const Geo& g, const cpx<R>* U,
                  R a_self, R c_hop, int p_out, const cpx<R>* in, const cpx<R>* self, cpx<R>* out, const cpx<R>* aux,
                  int ncol, int tc, int remap, int blocked, double* partial, const ColState* st) {
#define DD_EO_KC(K, REC, NTS)                                                                                          \
    launch_eo_epi<R, D, SF, K, REC, NTS>(s, epi, grid, g, U, a_self, c_hop, p_out, in, self, out, aux, ncol, tc, remap, \
                                         blocked, partial, st)
    if constexpr (sizeof(R) == 4) {
        if (kc == 2) {
            if (rec) {
                if (nts) DD_EO_KC(2, true, true);
                else DD_EO_KC(2, true, false);
            } else {
                if (nts) DD_EO_KC(2, false, true);
                else DD_EO_KC(2, false, false);
            }
            return;
        }
    }
    DD_EO_KC(1, false, false);
#undef DD_EO_KC
}

// The LDS-tile form applies to FP32 fields with L = 32 or 16 whose links are SU(3)
// (two rows each).
template <typename R>
bool eo_lds_ok(const Geo& g, const void* U12) {
    return sizeof(R) == 4 && U12 != nullptr && (g.L == 32 || g.L == 16);
}

template <typename R, int D, bool SF, int LH>
void launch_eo_lds_lh(hipStream_t s, int epi, bool nts, dim3 grid, const Geo& g, const cpx<R>* U12, R a_self,
                      R c_hop, int p_out, const cpx<R>* in, const cpx<R>* self, cpx<R>* out, const cpx<R>* aux,
                      int ncol, int cpw, int remap, double* partial, const ColState* st) {
    const dim3 block(kLdsNT);
#define DD_LDS_CASE(E)                                                                                              \
    if (nts)                                                                                                        \
        hipLaunchKernelGGL((k_eo_lds<R, D, E, SF, LH, true>), grid, block, 0, s, g, U12, a_self, c_hop, p_out, in, \
                           self, out, aux, ncol, cpw, remap, partial, st);                                          \
    else                                                                                                            \
        hipLaunchKernelGGL((k_eo_lds<R, D, E, SF, LH, false>), grid, block, 0, s, g, U12, a_self, c_hop, p_out, in, \
                           self, out, aux, ncol, cpw, remap, partial, st)
    if constexpr (!SF) {
        DD_LDS_CASE(EPI_STORE);  // the first half of the Schur operator
    } else {
        switch (epi) {
            case EPI_STORE: DD_LDS_CASE(EPI_STORE); break;
            case EPI_DOT_AUX: DD_LDS_CASE(EPI_DOT_AUX); break;
            case EPI_TS: DD_LDS_CASE(EPI_TS); break;
            default: DD_LDS_CASE(EPI_NORM); break;
        }
    }
#undef DD_LDS_CASE
}

// out = a_self * self + c_hop * H_{p_out, 1 - p_out} in, for ncol half-field columns,
// time chunks of tc slices, kc columns per thread (eo_kc_ok), workgroups
// optionally in XCD-contiguous ranges; tile flags `blocked`: bit 0 tiles as
// bricks (pair_site) rather than rows, bit 1 the chunks of a tile adjacent,
// bit 2 non-temporal output stores (k_eo_hop_nt; FP32 with kc > 1 only).
// U: the checkerboard links; U12 (nullable): the same links as two rows each,
// which launches with kc > 1 read instead.
//
// Tile flag bit 3 selects the LDS-tile form (eo_lds_ok; one slice per workgroup, so
// its partial slots are those of tc = 1) with kc columns per workgroup and bit 2
// for non-temporal stores; where it does not apply the time sweep runs instead.
template <typename R>
void launch_eo_hop(dd_ctx* c, const Geo& g, const cpx<R>* U, const cpx<R>* U12, double a_self, double c_hop,
                   int p_out, int dag, int epi, const cpx<R>* in, const cpx<R>* self, cpx<R>* out, const cpx<R>* aux,
                   int ncol, int tc, int kc, int remap, int blocked, double* partial, const ColState* st) {
    const bool sf = self != nullptr && a_self != 0;
    if constexpr (sizeof(R) == 4)
    if ((blocked & 8) && eo_lds_ok<R>(g, U12) && !(epi == EPI_RESID) && (sf || epi == EPI_STORE)) {
        const int cpw = std::max(1, std::min(kc, ncol));
        const bool nts = (blocked & 4) != 0;
        const int ntile = ((g.L3 >> 1) + kLdsNT - 1) / kLdsNT;
        const dim3 grid((unsigned)(ntile * g.nt * ((ncol + cpw - 1) / cpw)));
        hipEvent_t ev = nullptr;
        if (c->timing) timing_begin(c, &ev);
#define DD_LDS_LAUNCH(D, SF, LH)                                                                                    \
    launch_eo_lds_lh<R, D, SF, LH>(c->stream, epi, nts, grid, g, U12, R(a_self), R(c_hop), p_out, in, self, out, aux, \
                                   ncol, cpw, remap, partial, st)
#define DD_LDS_LH(D, SF)                 \
    if (g.L == 32) DD_LDS_LAUNCH(D, SF, 16); \
    else DD_LDS_LAUNCH(D, SF, 8)
        if (dag) {
            if (sf) DD_LDS_LH(1, true);
            else DD_LDS_LH(1, false);
        } else {
            if (sf) DD_LDS_LH(0, true);
            else DD_LDS_LH(0, false);
        }
#undef DD_LDS_LH
#undef DD_LDS_LAUNCH
        if (c->timing) {
            const double nh = (double)(g.nsite >> 1);
            const double extra = (sf || epi == EPI_TS ? 24.0 : 0.0) + (epi == EPI_DOT_AUX ? 24.0 : 0.0);
            const double bytes = nh * ((48.0 + extra) * ncol * c->bill_frac + 96.0) * sizeof(R);
            const std::string name = std::string("k_eo_lds<float, ") + std::to_string(dag ? 1 : 0) + ", " +
                                     std::to_string(epi) + (sf ? ", true, " : ", false, ") +
                                     std::to_string(g.L / 2) + (nts ? ", true>" : ", false>");
            timing_end(c, ev, name, bytes);
        }
        return;
    }
    if (blocked & 8) {  // the LDS form does not apply here: the time sweep of one slice per chunk
        blocked = 0;
        kc = 1;
    }
    if (!eo_kc_ok<R>(kc, ncol)) kc = 1;
    if (g.L % 4 != 0) blocked &= ~1;
    const bool nts = (blocked & 4) && kc > 1;
    blocked &= 3;
    const bool rec = U12 != nullptr && kc > 1;
    if (rec) U = U12;
    const dim3 grid((unsigned)(eo_blocks(g, tc) * (ncol / kc)));
    hipEvent_t ev = nullptr;
    if (c->timing) timing_begin(c, &ev);
#define DD_EO_LAUNCH(D, SF)                                                                                           \
    launch_eo_kc<R, D, SF>(c->stream, kc, rec, nts, epi, grid, g, U, R(a_self), R(c_hop), p_out, in, self, out, \
                           aux, ncol, tc, remap, blocked, partial, st)
    if (dag) {
        if (sf) DD_EO_LAUNCH(1, true);
        else DD_EO_LAUNCH(1, false);
    } else {
        if (sf) DD_EO_LAUNCH(0, true);
        else DD_EO_LAUNCH(0, false);
    }
#undef DD_EO_LAUNCH
    if (c->timing) {
        // per output half site: the input spinor, the output (+ self / aux when read), and the
        // links as stored (18 or 12 reals): every link of the field is used once by one output
        // site of a given parity
        const double nh = (double)(g.nsite >> 1);
        const double extra = (a_self != 0 || epi == EPI_TS ? 24.0 : 0.0) +
                             (epi == EPI_DOT_AUX || epi == EPI_RESID ? 24.0 : 0.0);
        const double bytes = nh * ((48.0 + extra) * ncol * c->bill_frac + (rec ? 96.0 : 144.0)) * sizeof(R);
        const std::string name = std::string(nts ? "k_eo_hop_nt<" : "k_eo_hop<") + (sizeof(R) == 8 ? "double" : "float") + ", " +
                                 std::to_string(dag ? 1 : 0) + ", " + std::to_string(epi) + ", " +
                                 std::to_string(kEoNT) + (sf ? ", true, " : ", false, ") + std::to_string(kc) +
                                 (rec ? ", true>" : ", false>");
        timing_end(c, ev, name, bytes);
    }
}

// The Schur complement of one lattice or slab: segments are the ncol even
// half-field columns; apply = two half hops through a scratch odd half field.
struct EOSystem : System {
    Geo g{};
    const cpx<double>* U64 = nullptr;  // checkerboard-ordered links of the field (Ueo)
    const cpx<float>* U32 = nullptr;
    const cpx<float>* U32c = nullptr;  // two rows per link, where the links are SU(3)
    double m = 0;  // 1 / (2 kappa)
    int dag = 0;
    int ncol = 0;
    cpx<double>* tmp64 = nullptr;
    cpx<float>* tmp32 = nullptr;
    // launch shape of the half-hop sweep per kind (0: FP64, 1: FP32): chunk length, XCD remap,
    // columns per thread, tile shape
    StencilSched sh[2];
    template <typename R>
    void schur(const cpx<R>* UR, const cpx<R>* UR12, cpx<R>* tmp, const StencilSched& sc, int d, int epi,
               const cpx<R>* in, cpx<R>* out, const cpx<R>* aux, double* partial, const ColState* st) {
        launch_eo_hop<R>(c, g, UR, UR12, 0.0, 1.0, 1, d, EPI_STORE, in, nullptr, tmp, nullptr, ncol, sc.tc, sc.kc,
                         sc.remap, sc.blocked, partial, st);
        launch_eo_hop<R>(c, g, UR, UR12, m, -0.25 / m, 0, d, epi, tmp, in, out, aux, ncol, sc.tc, sc.kc, sc.remap,
                         sc.blocked, partial, st);
    }
    void apply64(int d, int epi, const cpx<double>* in, cpx<double>* out, const cpx<double>* aux, double* partial,
                 const ColState* st) override {
        schur<double>(U64, nullptr, tmp64, sh[0], d ^ dag, epi, in, out, aux, partial, st);
    }
    void apply32(int d, int epi, const cpx<float>* in, cpx<float>* out, const cpx<float>* aux, double* partial,
                 const ColState* st) override {
        schur<float>(U32, U32c, tmp32, sh[1], d ^ dag, epi, in, out, aux, partial, st);
    }
};

// Launch shape of the half-hop sweep for one precision: timed on the Schur
// operator of this geometry and column count at first use (chunks of 1, 2,
// 4, 8 slices, workgroups in hardware order or XCD-contiguous ranges, 1 or 2
// columns per thread where allowed, row or brick tiles, tiles or chunks
// adjacent, plain or non-temporal output stores with two columns), cached in the
// context like the stencil shapes; small fields take 4 slices, no remap, one
// column, row tiles, untimed.
template <typename R>
StencilSched eo_tune(dd_ctx* c, EOSystem& S, const cpx<R>* UR, const cpx<R>* UR12, cpx<R>* tmp, const cpx<R>* in,
                     cpx<R>* out) {
    const Geo& g = S.g;
    const std::string key = std::string("eo:") + (sizeof(R) == 8 ? "0" : "1") + ":" + std::to_string(S.ncol) + ":" +
                            std::to_string(g.L) + ":" + std::to_string(g.T) + ":" + std::to_string(g.nt) + ":" +
                            std::to_string(g.whole);
    const auto hit = c->sched.find(key);
    if (hit != c->sched.end()) return hit->second;
    StencilSched best;
    best.nt = kEoNT;
    best.tc = std::min(4, g.nt);
    best.kc = 1;
    if ((size_t)g.nsite * S.ncol >= ((size_t)1 << 18)) {
        hipEvent_t a, b;
        if (hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess) {
            const int saved = c->timing;
            c->timing = 0;
            float best_ms = 1e30f;
            // the best of three timings of three Schur applications (one timing picked shapes by noise)
            auto time_shape = [&](const StencilSched& sc) {
                for (int w = 0; w < 2; w++)
                    S.schur<R>(UR, UR12, tmp, sc, 0, EPI_STORE, in, out, nullptr, nullptr, nullptr);
                float ms = 1e30f;
                for (int rep = 0; rep < 3; rep++) {
                    (void)hipEventRecord(a, c->stream);
                    for (int r = 0; r < 3; r++)
                        S.schur<R>(UR, UR12, tmp, sc, 0, EPI_STORE, in, out, nullptr, nullptr, nullptr);
                    (void)hipEventRecord(b, c->stream);
                    (void)hipEventSynchronize(b);
                    float t = 0;
                    (void)hipEventElapsedTime(&t, a, b);
                    ms = t < ms ? t : ms;
                }
                return ms;
            };
            for (int t : {1, 2, 4, 8})
                for (int rm = 0; rm < 2; rm++)
                    for (int kc : {1, 2})
                        for (int bl = 0; bl < 8; bl++) {
                            if (t > g.nt || !eo_kc_ok<R>(kc, S.ncol) || ((bl & 1) && g.L % 4 != 0)) continue;
                            if ((bl & 4) && kc == 1) continue;  // non-temporal stores: kc > 1 only
                            if ((bl & 2) && (g.nt + t - 1) / t < 2) continue;  // one chunk: the same order
                            StencilSched sc = best;
                            sc.tc = t;
                            sc.remap = rm;
                            sc.kc = kc;
                            sc.blocked = bl;
                            const float ms = time_shape(sc);
                            if (ms < best_ms) {
                                best_ms = ms;
                                best = sc;
                            }
                        }
            // the LDS-tile form: columns per workgroup, XCD remap, store form
            if (eo_lds_ok<R>(g, UR12))
                for (int cpw : {12, 6, 4, 3, 2, 1})
                    for (int rm = 0; rm < 2; rm++)
                        for (int nts = 0; nts < 2; nts++) {
                            if (cpw > S.ncol) continue;
                            StencilSched sc = best;
                            sc.tc = 1;
                            sc.remap = rm;
                            sc.kc = cpw;
                            sc.blocked = 8 | (nts ? 4 : 0);
                            const float ms = time_shape(sc);
                            if (ms < best_ms) {
                                best_ms = ms;
                                best = sc;
                            }
                        }
            c->timing = saved;
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(b);
        }
        (void)hipGetLastError();
    }
    tune_cache_store(c, key, best);
    return best;
}

}  // namespace

// A hop that wraps around the time edge of a whole lattice joins sites of the
// same parity when nt is odd, unless time_bc = 0 drops it.
bool eo_applicable(const Geo& g) { return g.L % 2 == 0 && (!g.whole || g.nt % 2 == 0 || g.bc == 0); }

dd_status links_eo12(dd_ctx* c, const Geo& g, const cpx<double>* U, cpx<float>* Ueo12, bool* su3) {
    const int nblk = (g.nsite + kBlock - 1) / kBlock;
    dd_status e = DD_OK;
    double* dev = (double*)workspace(c, W_LDEV, (size_t)nblk * sizeof(double), &e);
    if (e != DD_OK) return e;
    hipLaunchKernelGGL(k_links_eo12, dim3((unsigned)nblk), dim3(kBlock), 0, c->stream, g, U, Ueo12, dev);
    std::vector<double> h((size_t)nblk);
    DD_HIP(c, hipMemcpyAsync(h.data(), dev, h.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    DD_HIP(c, hipStreamSynchronize(c->stream));
    bool ok = true;
    for (double v : h) ok = ok && v <= 1e-6;
    *su3 = ok;
    return DD_OK;
}

template <typename R>
void launch_links_eo(dd_ctx* c, const Geo& g, const cpx<double>* U, cpx<R>* Ueo) {
    hipLaunchKernelGGL(k_links_eo<R>, dim3((unsigned)((g.nsite + kBlock - 1) / kBlock)), dim3(kBlock), 0, c->stream, g,
                       U, Ueo);
}
template void launch_links_eo<double>(dd_ctx*, const Geo&, const cpx<double>*, cpx<double>*);
template void launch_links_eo<float>(dd_ctx*, const Geo&, const cpx<double>*, cpx<float>*);

void launch_eo_split(dd_ctx* c, const Geo& g, int ncol, const cpx<double>* full, cpx<double>* ev, cpx<double>* od) {
    const size_t n = (size_t)ncol * 12 * g.nsite;
    hipLaunchKernelGGL(k_eo_split, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, c->stream, g, ncol,
                       full, ev, od);
}
void launch_eo_merge(dd_ctx* c, const Geo& g, int ncol, const cpx<double>* ev, const cpx<double>* od,
                     cpx<double>* full) {
    const size_t n = (size_t)ncol * 12 * g.nsite;
    hipLaunchKernelGGL(k_eo_merge, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, c->stream, g, ncol,
                       ev, od, full);
}
void launch_eo_hop64(dd_ctx* c, const Geo& g, const cpx<double>* Ueo, double a_self, double c_hop, int p_out, int dag,
                     const cpx<double>* in, const cpx<double>* self, cpx<double>* out, int ncol) {
    launch_eo_hop<double>(c, g, Ueo, nullptr, a_self, c_hop, p_out, dag, EPI_STORE, in, self, out, nullptr, ncol,
                          std::min(4, g.nt), 1, 0, 0, nullptr, nullptr);
}

dd_status solve_eo(dd_ctx* c, const cpx<double>* U, double kappa, const Geo& g, int ncol, const cpx<double>* b,
                   cpx<double>* x, const dd_solver_params& p, dd_solve_stats* stats, int dag) {
    const auto t_start = std::chrono::steady_clock::now();
    const size_t nh = (size_t)(g.nsite >> 1);
    const size_t nhalf = (size_t)ncol * 12 * nh;  // elements of one half field (all columns)
    const size_t nfull = 2 * nhalf;
    const double m = 1.0 / (2.0 * kappa);
    dd_status e = DD_OK;
    // b_e | b_o, later the full residual; x_e | x_o; the prepared source; the odd scratch fields
    cpx<double>* bb = (cpx<double>*)workspace(c, W_EO_B, nfull * sizeof(cpx<double>), &e);
    if (e != DD_OK) return e;
    cpx<double>* xx = (cpx<double>*)workspace(c, W_EO_X, nfull * sizeof(cpx<double>), &e);
    if (e != DD_OK) return e;
    cpx<double>* bhat = (cpx<double>*)workspace(c, W_EO_BHAT, nhalf * sizeof(cpx<double>), &e);
    if (e != DD_OK) return e;
    // checkerboard-ordered links of the field: FP64 always, FP32 for DD_MIXED
    const size_t nl = (size_t)36 * g.nsite;
    const unsigned glink = (unsigned)((g.nsite + kBlock - 1) / kBlock);
    cpx<double>* Ueo64 = (cpx<double>*)workspace(c, W_EO_U64, nl * sizeof(cpx<double>), &e);
    if (e != DD_OK) return e;
    hipLaunchKernelGGL(k_links_eo<double>, dim3(glink), dim3(kBlock), 0, c->stream, g, U, Ueo64);
    EOSystem S;
    S.pair32 = true;  // FP32 half fields with paired components (dd_eo.h)
    S.c = c;
    S.g = g;
    S.U64 = Ueo64;
    S.m = m;
    S.dag = dag;
    S.ncol = ncol;
    S.nelem = nhalf;
    S.tmp64 = (cpx<double>*)workspace(c, W_EO_T64, nhalf * sizeof(cpx<double>), &e);
    if (e != DD_OK) return e;
    if (p.prec == DD_MIXED) {
        cpx<float>* U32 = (cpx<float>*)workspace(c, W_U32, nl * sizeof(cpx<float>), &e);
        if (e != DD_OK) return e;
        hipLaunchKernelGGL(k_links_eo<float>, dim3(glink), dim3(kBlock), 0, c->stream, g, U, U32);
        S.U32 = U32;
        cpx<float>* U32c = (cpx<float>*)workspace(c, W_U32C, (size_t)24 * g.nsite * sizeof(cpx<float>), &e);
        if (e != DD_OK) return e;
        bool su3 = false;
        e = links_eo12(c, g, U, U32c, &su3);
        if (e != DD_OK) return e;
        if (su3) S.U32c = U32c;
        S.tmp32 = (cpx<float>*)workspace(c, W_EO_T32, nhalf * sizeof(cpx<float>), &e);
        if (e != DD_OK) return e;
        S.has32 = true;
    }
    // launch shapes (tuned on two half-field work vectors whose contents do not matter)
    S.sh[0] = eo_tune<double>(c, S, Ueo64, nullptr, S.tmp64, bhat, xx);
    if (S.has32) {
        cpx<float>* a32 = (cpx<float>*)workspace(c, W_R32, nhalf * sizeof(cpx<float>), &e);
        if (e != DD_OK) return e;
        cpx<float>* b32 = (cpx<float>*)workspace(c, W_RH32, nhalf * sizeof(cpx<float>), &e);
        if (e != DD_OK) return e;
        S.sh[1] = eo_tune<float>(c, S, S.U32, S.U32c, S.tmp32, a32, b32);
    }
    SegLayout lay;
    const int n = (int)(12 * nh);
    for (int k = 0; k < ncol; k++) {
        lay.off.push_back((long long)k * n);
        lay.len.push_back(n);
    }
    for (int kind = 0; kind < 2; kind++) {
        const int nblk = eo_blocks(g, S.sh[kind].tc);
        lay.sp0[kind].resize(ncol + 1);
        for (int k = 0; k <= ncol; k++) lay.sp0[kind][k] = k * nblk;
    }
    e = lay.upload(c, W_SEGS, &S);
    if (e != DD_OK) return e;
    // the partial slots of the source preparation and reconstruction (chunks of min(4, nt))
    S.nslots = std::max(S.nslots, (size_t)ncol * eo_blocks(g, std::min(4, g.nt)));

    // |b|^2 per column: the reference of every relative residual
    std::vector<double> bnorm;
    e = column_norms(c, (int)(12 * g.nsite), ncol, b, &bnorm);
    if (e != DD_OK) return e;
    for (double v : bnorm)
        if (!std::isfinite(v)) return fail(c, DD_ERR_BREAKDOWN, "non-finite values in the right-hand side");
    S.ref_norm2 = bnorm.data();

    const unsigned gsplit = (unsigned)((nfull + kBlock - 1) / kBlock);
    cpx<double>*b_e = bb, *b_o = bb + nhalf, *x_e = xx, *x_o = xx + nhalf;
    hipLaunchKernelGGL(k_eo_split, dim3(gsplit), dim3(kBlock), 0, c->stream, g, ncol, b, b_e, b_o);
    double* partial = (double*)workspace(c, W_PART, S.nslots * 3 * sizeof(double), &e);
    if (e != DD_OK) return e;
    // b_e' = b_e + (1/(2m)) H_eo b_o
    launch_eo_hop64(c, g, Ueo64, 1.0, 0.5 / m, 0, dag, b_o, b_e, bhat, ncol);

    // an initial guess (dd_block_solve with x0 = 1): its even sites start the Schur solve
    if (p.x0) hipLaunchKernelGGL(k_eo_split, dim3(gsplit), dim3(kBlock), 0, c->stream, g, ncol, x, x_e, x_o);
    SolveResult res;
    dd_status st = solve_system(S, bhat, x_e, p, &res);
    if (st != DD_OK && st != DD_ERR_NOCONV && st != DD_ERR_BREAKDOWN) return st;

    // x_o = (b_o + 1/2 H_oe x_e) / m, then the full answer and its true residual
    launch_eo_hop64(c, g, Ueo64, 1.0 / m, 0.5 / m, 1, dag, x_e, b_o, x_o, ncol);
    hipLaunchKernelGGL(k_eo_merge, dim3(gsplit), dim3(kBlock), 0, c->stream, g, ncol, x_e, x_o, x);
    cpx<double>* r = bb;  // b_e | b_o are no longer needed
    const size_t rslots = std::max(S.nslots, (size_t)ncol * stencil_slots(c, g, 0, ncol));
    partial = (double*)workspace(c, W_PART, rslots * 3 * sizeof(double), &e);
    if (e != DD_OK) return e;
    launch_dslash<double>(c, g, U, kappa, dag, EPI_RESID, x, r, b, ncol, partial, nullptr);
    DD_HIP(c, hipGetLastError());
    std::vector<double> rr;
    e = column_norms(c, (int)(12 * g.nsite), ncol, r, &rr);
    if (e != DD_OK) return e;
    bool converged = st == DD_OK, nonfinite = st == DD_ERR_BREAKDOWN;
    std::vector<double> rel(ncol, 0.0);
    for (int j = 0; j < ncol; j++) {
        if (!std::isfinite(rr[j])) nonfinite = true;
        rel[j] = bnorm[j] > 0 ? std::sqrt(rr[j] / bnorm[j]) : 0.0;
        if (!(rel[j] <= p.tol)) converged = false;
    }
    if (stats) {
        stats->nrhs = ncol;
        stats->iters = res.iters;
        stats->updates = res.updates;
        stats->restarts = res.restarts;
        for (int j = 0; j < DD_MAX_RHS; j++) stats->true_rel_resid[j] = j < ncol ? rel[j] : 0.0;
        stats->ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    }
    if (nonfinite) return fail(c, DD_ERR_BREAKDOWN, "non-finite values in the Krylov iteration");
    if (!converged) {
        double worst = 0;
        for (double v : rel) worst = std::max(worst, v);
        return fail(c, DD_ERR_NOCONV,
                    "even-odd solver stopped after " + std::to_string(res.iters) +
                        " iterations with relative residual " + std::to_string(worst) + " > tol " +
                        std::to_string(p.tol));
    }
    return DD_OK;
}

}  // namespace dd
