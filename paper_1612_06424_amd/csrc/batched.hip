// batched.hip -- solves of many independent domains together (each with its
// own lattice shape, links, kappa and sources).
//
// Every (domain, column) pair is one solver segment; the work vectors hold all
// segments back to back, so one stencil launch and one launch of each vector
// kernel cover every active domain of the batch.  The multi-domain stencil
// finds its domain from the workgroup index (binary search over the domains'
// first workgroups) and runs the same tile as the single-lattice kernel with
// that domain's geometry, links and mass.  The tile shape (workgroup size and
// time-chunk length) is tuned on the batch itself before the solve, and the
// inner Krylov iterations are captured once into a HIP graph and replayed on
// a library-owned stream.
//
// When every domain is bipartite (and even-odd preconditioning is asked for)
// the batch solves the even-site Schur complements of all domains together
// (dd_eo.h), with a multi-domain half-hop kernel; the source preparation, the
// reconstruction of the odd sites and the final check on the full operator run
// domain by domain.
#include <algorithm>
#include <chrono>
#include <cstring>

#include "dd_dslash.h"
#include "dd_eo.h"

namespace dd {

namespace {

// One domain of a batch, as the multi-domain stencil sees it in one precision.
struct BDom {
    Geo g;             // the domain's own lattice (whole = 1)
    const void* U;     // its links, cpx<R> [4][9][V]
    double mass;       // 1 / (2 kappa)
    long long voff;    // element offset of its column 0 in the work vectors
    int ncol;          // columns (segments) of the domain
    int seg0;          // its first segment
    int blk0;          // its first workgroup in the launch
    int nsb, nchunk;   // spatial blocks per slice, time chunks
    int tc;            // slices per chunk
    int slot0;         // its first partial slot
    int pad;
};
static_assert(sizeof(BDom) % 8 == 0, "descriptor layout must be the same on host and device");

template <typename R, int DAG, int EPI, int NT>
__global__ __launch_bounds__(NT) void k_bdslash(const BDom* __restrict__ doms, int ndom, const cpx<R>* __restrict__ in,
                                                cpx<R>* __restrict__ out, const cpx<R>* __restrict__ aux,
                                                double* __restrict__ partial, const ColState* __restrict__ st) {
    const int bid = (int)blockIdx.x;
    int lo = 0, hi = ndom - 1;  // last domain whose first workgroup is <= bid
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (doms[mid].blk0 <= bid) lo = mid;
        else hi = mid - 1;
    }
    const BDom& d = doms[lo];
    const int lb = bid - d.blk0;
    const int col = lb % d.ncol;
    const int rest = lb / d.ncol;
    const int sb = rest % d.nsb, tc = rest / d.nsb;
    if (st != nullptr && !st[d.seg0 + col].active) return;  // uniform over the workgroup
    const Geo g = d.g;
    const size_t off = (size_t)d.voff + (size_t)col * 12 * g.nsite;
    double* slot = partial + ((size_t)d.slot0 + (size_t)col * d.nsb * d.nchunk + (size_t)tc * d.nsb + sb) * 3;
    dslash_tile<R, DAG, EPI, NT>(g, (const cpx<R>*)d.U, R(d.mass), in + off, out + off,
                                 aux != nullptr ? aux + off : nullptr, sb, tc, d.tc, slot);
}

// One domain of an even-odd batch in one precision.
struct BEODom {
    Geo g;
    const void* Ueo;   // its checkerboard-ordered links, cpx<R>
    const void* Ueo12; // the same links as two rows each (FP32 batches whose links are SU(3)), or null
    double mass;       // 1 / (2 kappa)
    long long hoff;    // element offset of its column 0 in the half-field work vectors
    int ncol, seg0, blk0;
    int nblk;          // workgroups per column (group): ntile x chunks
    int slot0;         // its first partial slot
    int ntile;         // tiles of kBeoNT pairs per slice
    int tc;            // slices per chunk
    int blocked;       // brick tiles (pair_site)
};
static_assert(sizeof(BEODom) % 8 == 0, "descriptor layout must be the same on host and device");

constexpr int kBeoNT = 256;

// SCHUR = false: out = H_oe in (odd sites); SCHUR = true: out = m self - H_eo in / (4m) (even sites).
// A workgroup serves KC columns of its domain (every domain's ncol is a multiple of KC);
// REC: the links are read as two rows each (Ueo12, KC > 1 only).
template <typename R, int DAG, int EPI, bool SCHUR, int KC, bool REC>
__global__ __launch_bounds__(kBeoNT) void k_beo_hop(const BEODom* __restrict__ doms, int ndom,
                                                   const cpx<R>* __restrict__ in, const cpx<R>* __restrict__ self,
                                                   cpx<R>* __restrict__ out, const cpx<R>* __restrict__ aux,
                                                   int remap, double* __restrict__ partial,
                                                   const ColState* __restrict__ st) {
    const int bid = remap ? xcd_remap(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    int lo = 0, hi = ndom - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (doms[mid].blk0 <= bid) lo = mid;
        else hi = mid - 1;
    }
    const BEODom& d = doms[lo];
    const int lb = bid - d.blk0;
    const int ngrp = d.ncol / KC;
    const int col0 = (lb % ngrp) * KC, blk = lb / ngrp;
    unsigned live = 0;  // active columns of the group; the workgroup runs while one is
#pragma unroll
    for (int k = 0; k < KC; k++)
        if (st == nullptr || st[d.seg0 + col0 + k].active) live |= 1u << k;
    if (live == 0) return;  // uniform over the workgroup
    const Geo g = d.g;
    const size_t off = (size_t)d.hoff + (size_t)col0 * 12 * (size_t)(g.nsite >> 1);
    const R a_self = SCHUR ? R(d.mass) : R(0);
    const R c_hop = SCHUR ? R(-0.25 / d.mass) : R(1);
    double* slot = partial + ((size_t)d.slot0 + (size_t)col0 * d.nblk + blk) * 3;
    if constexpr (KC == 1)
        eo_sweep_tile<R, DAG, EPI, kBeoNT, SCHUR>(g, (const cpx<R>*)d.Ueo, a_self, c_hop, SCHUR ? 0 : 1, in + off,
                                                  self != nullptr ? self + off : nullptr, out + off,
                                                  aux != nullptr ? aux + off : nullptr, blk % d.ntile, blk / d.ntile,
                                                  d.tc, d.blocked, slot);
    else
        eo_sweep_cols<R, DAG, EPI, kBeoNT, SCHUR, KC, REC>(g, (const cpx<R>*)(REC ? d.Ueo12 : d.Ueo), a_self, c_hop,
                                                           SCHUR ? 0 : 1,
                                                      in + off, self != nullptr ? self + off : nullptr, out + off,
                                                      aux != nullptr ? aux + off : nullptr, live, blk % d.ntile,
                                                      blk / d.ntile, d.tc, d.blocked, slot, (size_t)d.nblk);
}

template <typename R, int DAG, bool SCHUR, int KC, bool REC>
void launch_beo_epi(hipStream_t s, int epi, unsigned nblk, const BEODom* doms, int ndom, const cpx<R>* in,
                    const cpx<R>* self, cpx<R>* out, const cpx<R>* aux, int remap, double* partial,
                    const ColState* st) {
    const dim3 grid(nblk), block(kBeoNT);
#define DD_BEO_CASE(E)                                                                                             \
    hipLaunchKernelGGL((k_beo_hop<R, DAG, E, SCHUR, KC, REC>), grid, block, 0, s, doms, ndom, in, self, out, aux, \
                       remap, partial, st)
    switch (epi) {
        case EPI_STORE: DD_BEO_CASE(EPI_STORE); break;
        case EPI_DOT_AUX: DD_BEO_CASE(EPI_DOT_AUX); break;
        case EPI_TS: DD_BEO_CASE(EPI_TS); break;
        case EPI_RESID: DD_BEO_CASE(EPI_RESID); break;
        default: DD_BEO_CASE(EPI_NORM); break;
    }
#undef DD_BEO_CASE
}

// kc columns per workgroup: 1 in FP64, 1 or 2 in FP32 (as for the single-system half hop);
// rec: kc > 1 launches read the two-row links
template <typename R, int DAG, bool SCHUR>
void launch_beo(hipStream_t s, int kc, bool rec, int epi, unsigned nblk, const BEODom* doms, int ndom,
                const cpx<R>* in, const cpx<R>* self, cpx<R>* out, const cpx<R>* aux, int remap, double* partial,
                const ColState* st) {
#define DD_BEO_KC(K, REC) \
    launch_beo_epi<R, DAG, SCHUR, K, REC>(s, epi, nblk, doms, ndom, in, self, out, aux, remap, partial, st)
    if constexpr (sizeof(R) == 4) {
        if (kc == 2) {
            if (rec) DD_BEO_KC(2, true);
            else DD_BEO_KC(2, false);
            return;
        }
    }
    DD_BEO_KC(1, false);
#undef DD_BEO_KC
}

template <typename R, int DAG, int NT>
void launch_bepi(hipStream_t s, int epi, unsigned nblk, const BDom* doms, int ndom, const cpx<R>* in, cpx<R>* out,
                 const cpx<R>* aux, double* partial, const ColState* st) {
    const dim3 grid(nblk), block(NT);
    switch (epi) {
        case EPI_STORE:
            hipLaunchKernelGGL((k_bdslash<R, DAG, EPI_STORE, NT>), grid, block, 0, s, doms, ndom, in, out, aux,
                               partial, st);
            break;
        case EPI_DOT_AUX:
            hipLaunchKernelGGL((k_bdslash<R, DAG, EPI_DOT_AUX, NT>), grid, block, 0, s, doms, ndom, in, out, aux,
                               partial, st);
            break;
        case EPI_TS:
            hipLaunchKernelGGL((k_bdslash<R, DAG, EPI_TS, NT>), grid, block, 0, s, doms, ndom, in, out, aux, partial,
                               st);
            break;
        case EPI_RESID:
            hipLaunchKernelGGL((k_bdslash<R, DAG, EPI_RESID, NT>), grid, block, 0, s, doms, ndom, in, out, aux,
                               partial, st);
            break;
        default:
            hipLaunchKernelGGL((k_bdslash<R, DAG, EPI_NORM, NT>), grid, block, 0, s, doms, ndom, in, out, aux,
                               partial, st);
            break;
    }
}

struct BSched {
    int nt = 128;  // workgroup size (spatial sites)
    int tc = 8;    // slices per time chunk (clamped to each domain's extent)
};

// One precision's launch of the multi-domain stencil: descriptors on the
// device, workgroup count and the schedule they were built for.
struct BLaunch {
    BSched sc;
    const BDom* doms = nullptr;
    unsigned nblk = 0;
    int nslot = 0;
    std::vector<BDom> host;
};

struct Item {
    Geo g;
    double kappa;
    int ncol;
    long long voff;   // element offset of column 0
    long long uoff;   // element offset of the FP32 links
    const cpx<double>* U64;
};

// Fill the descriptors for schedule sc (kind 0: FP64 links, 1: FP32 links).
void build_descs(const std::vector<Item>& items, const BSched& sc, int kind, const cpx<float>* U32, BLaunch* L) {
    L->sc = sc;
    L->host.resize(items.size());
    int blk = 0, slot = 0, seg = 0;
    for (size_t i = 0; i < items.size(); i++) {
        const Item& it = items[i];
        BDom& d = L->host[i];
        std::memset(&d, 0, sizeof(d));
        d.g = it.g;
        d.U = kind == 0 ? (const void*)it.U64 : (const void*)(U32 + it.uoff);
        d.mass = 1.0 / (2.0 * it.kappa);
        d.voff = it.voff;
        d.ncol = it.ncol;
        d.seg0 = seg;
        d.blk0 = blk;
        d.tc = std::min(sc.tc, it.g.nt);
        d.nsb = (it.g.L3 + sc.nt - 1) / sc.nt;
        d.nchunk = (it.g.nt + d.tc - 1) / d.tc;
        d.slot0 = slot;
        const int per = d.nsb * d.nchunk;
        blk += per * it.ncol;
        slot += per * it.ncol;
        seg += it.ncol;
    }
    L->nblk = (unsigned)blk;
    L->nslot = slot;
}

dd_status upload_descs(dd_ctx* c, Slot slot, BLaunch* L) {
    dd_status e = DD_OK;
    BDom* dev = (BDom*)workspace(c, slot, sizeof(BDom) * L->host.size(), &e);
    if (e != DD_OK) return e;
    DD_HIP(c, hipMemcpyAsync(dev, L->host.data(), sizeof(BDom) * L->host.size(), hipMemcpyHostToDevice, c->stream));
    DD_HIP(c, hipStreamSynchronize(c->stream));
    L->doms = dev;
    return DD_OK;
}

struct BatchSystem : System {
    BLaunch lk[2];  // kind 0: FP64, 1: FP32
    int ndom = 0;

    template <typename R>
    void launch(const BLaunch& L, int dag, int epi, const cpx<R>* in, cpx<R>* out, const cpx<R>* aux,
                double* partial, const ColState* st) {
        hipEvent_t ev = nullptr;
        if (c->timing) timing_begin(c, &ev);
        if (L.sc.nt == 256) {
            if (dag) launch_bepi<R, 1, 256>(c->stream, epi, L.nblk, L.doms, ndom, in, out, aux, partial, st);
            else launch_bepi<R, 0, 256>(c->stream, epi, L.nblk, L.doms, ndom, in, out, aux, partial, st);
        } else {
            if (dag) launch_bepi<R, 1, 128>(c->stream, epi, L.nblk, L.doms, ndom, in, out, aux, partial, st);
            else launch_bepi<R, 0, 128>(c->stream, epi, L.nblk, L.doms, ndom, in, out, aux, partial, st);
        }
        if (c->timing) {
            double sites_cols = 0, sites = 0;
            for (const BDom& d : L.host) {
                sites_cols += (double)d.g.nsite * d.ncol;
                sites += d.g.nsite;
            }
            const double extra = (epi == EPI_DOT_AUX || epi == EPI_RESID) ? 24.0 : 0.0;
            const double bytes = ((48.0 + extra) * sites_cols * c->bill_frac + 72.0 * sites) * sizeof(R);
            const std::string name = std::string("k_bdslash<") + (sizeof(R) == 8 ? "double" : "float") + ", " +
                                     std::to_string(dag ? 1 : 0) + ", " + std::to_string(epi) + ", " +
                                     std::to_string(L.sc.nt) + ">";
            timing_end(c, ev, name, bytes);
        }
    }
    void apply64(int dag, int epi, const cpx<double>* in, cpx<double>* out, const cpx<double>* aux, double* partial,
                 const ColState* st) override {
        launch<double>(lk[0], dag, epi, in, out, aux, partial, st);
    }
    void apply32(int dag, int epi, const cpx<float>* in, cpx<float>* out, const cpx<float>* aux, double* partial,
                 const ColState* st) override {
        launch<float>(lk[1], dag, epi, in, out, aux, partial, st);
    }
};

// The even-site Schur complements of every domain of a batch: segments are
// the even half-field columns, apply = two multi-domain half hops through an
// odd half-field scratch vector.
struct BatchEOSystem : System {
    const BEODom* doms[2] = {nullptr, nullptr};  // kind 0: FP64 links, 1: FP32 links
    std::vector<BEODom> host;                    // FP64 descriptors (sizes, for timing)
    int ndom = 0;
    unsigned nblk = 0;                 // workgroups of a launch while tuning
    unsigned nblk64 = 0, nblk32 = 0;   // workgroups of a launch per precision
    int remap[2] = {0, 0};             // XCD-contiguous workgroup ranges per precision
    int kc[2] = {1, 1};                // columns per workgroup per precision
    bool rec32 = false;                // FP32 descriptors carry two-row links
    cpx<double>* tmp64 = nullptr;
    cpx<float>* tmp32 = nullptr;

    template <typename R>
    void schur(const BEODom* dv, cpx<R>* tmp, int dag, int epi, const cpx<R>* in, cpx<R>* out, const cpx<R>* aux,
               double* partial, const ColState* st) {
        const unsigned nblk = this->nblk != 0 ? this->nblk : (sizeof(R) == 8 ? nblk64 : nblk32);
        const int rm = remap[sizeof(R) == 8 ? 0 : 1];
        const int k = kc[sizeof(R) == 8 ? 0 : 1];
        const bool rec = sizeof(R) == 4 && rec32 && k > 1;
        for (int half = 0; half < 2; half++) {
            const int e = half ? epi : EPI_STORE;
            hipEvent_t ev = nullptr;
            if (c->timing) timing_begin(c, &ev);
            if (half == 0) {
                if (dag)
                    launch_beo<R, 1, false>(c->stream, k, rec, e, nblk, dv, ndom, in, nullptr, tmp, nullptr, rm,
                                            partial, st);
                else
                    launch_beo<R, 0, false>(c->stream, k, rec, e, nblk, dv, ndom, in, nullptr, tmp, nullptr, rm,
                                            partial, st);
            } else {
                if (dag) launch_beo<R, 1, true>(c->stream, k, rec, e, nblk, dv, ndom, tmp, in, out, aux, rm, partial, st);
                else launch_beo<R, 0, true>(c->stream, k, rec, e, nblk, dv, ndom, tmp, in, out, aux, rm, partial, st);
            }
            if (c->timing) {
                // per output half site: input, output (+ self, + aux) spinors; every link of a domain
                // once, as stored (18 or 12 reals)
                double sc = 0, s = 0;
                for (const BEODom& d : host) {
                    sc += (double)(d.g.nsite >> 1) * d.ncol;
                    s += (double)(d.g.nsite >> 1);
                }
                const double extra = (half ? 24.0 : 0.0) + (e == EPI_DOT_AUX || e == EPI_RESID ? 24.0 : 0.0);
                const double bytes = ((48.0 + extra) * sc * c->bill_frac + (rec ? 96.0 : 144.0) * s) * sizeof(R);
                const std::string name = std::string("k_beo_hop<") + (sizeof(R) == 8 ? "double" : "float") + ", " +
                                         std::to_string(dag ? 1 : 0) + ", " + std::to_string(e) + ", " +
                                         (half ? "true, " : "false, ") + std::to_string(k) +
                                         (rec ? ", true>" : ", false>");
                timing_end(c, ev, name, bytes);
            }
        }
    }
    void apply64(int dag, int epi, const cpx<double>* in, cpx<double>* out, const cpx<double>* aux, double* partial,
                 const ColState* st) override {
        schur<double>(doms[0], tmp64, dag, epi, in, out, aux, partial, st);
    }
    void apply32(int dag, int epi, const cpx<float>* in, cpx<float>* out, const cpx<float>* aux, double* partial,
                 const ColState* st) override {
        schur<float>(doms[1], tmp32, dag, epi, in, out, aux, partial, st);
    }
};

// Pick the tile shape of one precision by timing the stencil on the batch
// itself (out-of-place on two work vectors whose contents do not matter).
// The choice is cached in the context per batch signature (precision and
// every domain's shape and column count), so repeated solves of the same
// batch use the same tiles and give bitwise the same results.
template <typename R>
dd_status tune_batch(dd_ctx* c, BatchSystem& S, const std::vector<Item>& items, int kind, const cpx<float>* U32,
                     const cpx<R>* in, cpx<R>* out, Slot slot) {
    std::string key = "batch:" + std::to_string(kind);
    for (const Item& it : items)
        key += ":" + std::to_string(it.g.T) + "x" + std::to_string(it.g.L) + "x" + std::to_string(it.ncol) + "b" +
               std::to_string(it.g.bc);
    const auto hit = c->sched.find(key);
    if (hit != c->sched.end()) {
        BSched sc;
        sc.nt = hit->second.nt;
        sc.tc = hit->second.tc;
        build_descs(items, sc, kind, U32, &S.lk[kind]);
        return upload_descs(c, slot, &S.lk[kind]);
    }
    static const int nts[] = {128, 256};
    static const int tcs[] = {4, 8, 16};
    hipEvent_t a, b;
    DD_HIP(c, hipEventCreate(&a));
    DD_HIP(c, hipEventCreate(&b));
    float best = 1e30f;
    BSched best_sc;
    const int saved = c->timing;
    c->timing = 0;
    dd_status e = DD_OK;
    for (int nt : nts) {
        for (int tc : tcs) {
            BSched sc;
            sc.nt = nt;
            sc.tc = tc;
            build_descs(items, sc, kind, U32, &S.lk[kind]);
            e = upload_descs(c, slot, &S.lk[kind]);
            if (e != DD_OK) break;
            for (int w = 0; w < 2; w++) S.launch<R>(S.lk[kind], 0, EPI_STORE, in, out, nullptr, nullptr, nullptr);
            (void)hipEventRecord(a, c->stream);
            for (int w = 0; w < 3; w++) S.launch<R>(S.lk[kind], 0, EPI_STORE, in, out, nullptr, nullptr, nullptr);
            (void)hipEventRecord(b, c->stream);
            if (hipEventSynchronize(b) != hipSuccess) {
                e = hip_fail(c, hipGetLastError(), "batched tile tuning");
                break;
            }
            float ms = 0;
            (void)hipEventElapsedTime(&ms, a, b);
            if (ms < best) {
                best = ms;
                best_sc = sc;
            }
        }
        if (e != DD_OK) break;
    }
    c->timing = saved;
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (e != DD_OK) return e;
    StencilSched keep;
    keep.nt = best_sc.nt;
    keep.tc = best_sc.tc;
    tune_cache_store(c, key, keep);
    build_descs(items, best_sc, kind, U32, &S.lk[kind]);
    return upload_descs(c, slot, &S.lk[kind]);
}

// Runs the batched solve with c->stream switched to the library's own stream
// (a graph can only be captured from a stream the library controls), ordered
// after the caller's stream on entry and waited for on exit.
class OwnStream {
  public:
    explicit OwnStream(dd_ctx* c) : c_(c), caller_(c->stream) {}
    dd_status enter() {
        if (c_->own_stream == nullptr) DD_HIP(c_, hipStreamCreateWithFlags(&c_->own_stream, hipStreamNonBlocking));
        hipEvent_t ev;
        DD_HIP(c_, hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        hipError_t e1 = hipEventRecord(ev, caller_);
        hipError_t e2 = e1 == hipSuccess ? hipStreamWaitEvent(c_->own_stream, ev, 0) : e1;
        (void)hipEventDestroy(ev);
        DD_HIP(c_, e2);
        c_->stream = c_->own_stream;
        return DD_OK;
    }
    ~OwnStream() {
        if (c_->stream != caller_) {
            (void)hipStreamSynchronize(c_->stream);
            c_->stream = caller_;
        }
    }

  private:
    dd_ctx* c_;
    hipStream_t caller_;
};

// The even-odd batch: every domain bipartite.  b is in bcat (full layout,
// offsets its[i].voff); the answer goes to xcat.
dd_status solve_batch_eo(dd_ctx* c, const std::vector<Item>& its, const dd_solver_params& p, const cpx<double>* bcat,
                         cpx<double>* xcat, SolveResult* res, std::vector<double>* rel) {
    const int n = (int)its.size();
    dd_status e = DD_OK;
    std::vector<long long> hoff(n), eoff(n), e12off(n);
    long long nhalf = 0, nl = 0, nl12 = 0;
    for (int i = 0; i < n; i++) {
        hoff[i] = nhalf;
        eoff[i] = nl;
        e12off[i] = nl12;
        nhalf += (long long)its[i].ncol * 12 * (its[i].g.nsite >> 1);
        nl += (long long)36 * its[i].g.nsite;
        nl12 += (long long)24 * its[i].g.nsite;
    }
    const bool mixed = p.prec == DD_MIXED;
    cpx<double>* U64 = (cpx<double>*)workspace(c, W_EO_U64, (size_t)nl * sizeof(cpx<double>), &e);
    if (e != DD_OK) return e;
    cpx<float>* U32 = nullptr;
    cpx<float>* U32c = nullptr;  // two rows per link, used while every domain's links are SU(3)
    if (mixed) {
        U32 = (cpx<float>*)workspace(c, W_U32, (size_t)nl * sizeof(cpx<float>), &e);
        if (e != DD_OK) return e;
        U32c = (cpx<float>*)workspace(c, W_U32C, (size_t)nl12 * sizeof(cpx<float>), &e);
        if (e != DD_OK) return e;
    }
    bool su3_all = mixed;
    cpx<double>* bb = (cpx<double>*)workspace(c, W_EO_B, 2 * (size_t)nhalf * sizeof(cpx<double>), &e);
    if (e != DD_OK) return e;
    cpx<double>* xx = (cpx<double>*)workspace(c, W_EO_X, 2 * (size_t)nhalf * sizeof(cpx<double>), &e);
    if (e != DD_OK) return e;
    cpx<double>* bhat = (cpx<double>*)workspace(c, W_EO_BHAT, (size_t)nhalf * sizeof(cpx<double>), &e);
    if (e != DD_OK) return e;
    cpx<double>*b_e = bb, *b_o = bb + nhalf, *x_e = xx, *x_o = xx + nhalf;
    for (int i = 0; i < n; i++) {
        const Item& it = its[i];
        const double m = 1.0 / (2.0 * it.kappa);
        launch_links_eo<double>(c, it.g, it.U64, U64 + eoff[i]);
        if (mixed) {
            launch_links_eo<float>(c, it.g, it.U64, U32 + eoff[i]);
            bool su3 = false;
            e = links_eo12(c, it.g, it.U64, U32c + e12off[i], &su3);
            if (e != DD_OK) return e;
            su3_all = su3_all && su3;
        }
        launch_eo_split(c, it.g, it.ncol, bcat + it.voff, b_e + hoff[i], b_o + hoff[i]);
        // b_e' = b_e + (1/(2m)) H_eo b_o
        launch_eo_hop64(c, it.g, U64 + eoff[i], 1.0, 0.5 / m, 0, 0, b_o + hoff[i], b_e + hoff[i], bhat + hoff[i],
                        it.ncol);
    }
    DD_HIP(c, hipGetLastError());

    BatchEOSystem S;
    S.c = c;
    S.ndom = n;
    S.nelem = (size_t)nhalf;
    S.graph = true;
    S.has32 = mixed;
    S.pair32 = true;  // FP32 half fields with paired components (dd_eo.h)
    S.rec32 = su3_all;
    S.tmp64 = (cpx<double>*)workspace(c, W_EO_T64, (size_t)nhalf * sizeof(cpx<double>), &e);
    if (e != DD_OK) return e;
    if (mixed) {
        S.tmp32 = (cpx<float>*)workspace(c, W_EO_T32, (size_t)nhalf * sizeof(cpx<float>), &e);
        if (e != DD_OK) return e;
    }
    // descriptors for a chunk length tc of the half-hop sweep, precision kind
    auto build = [&](int tc, int kc, int blocked, int kind, std::vector<BEODom>* h, std::vector<int>* sp0) {
        h->clear();
        sp0->clear();
        int blk = 0, slot = 0, seg = 0;
        for (int i = 0; i < n; i++) {
            const Item& it = its[i];
            BEODom d;
            std::memset(&d, 0, sizeof(d));
            d.g = it.g;
            d.Ueo = kind == 0 ? (const void*)(U64 + eoff[i]) : (const void*)(U32 + eoff[i]);
            d.Ueo12 = kind == 1 && su3_all ? (const void*)(U32c + e12off[i]) : nullptr;
            d.mass = 1.0 / (2.0 * it.kappa);
            d.hoff = hoff[i];
            d.ncol = it.ncol;
            d.seg0 = seg;
            d.blk0 = blk;
            d.ntile = ((it.g.L3 >> 1) + kBeoNT - 1) / kBeoNT;
            d.tc = std::min(tc, it.g.nt);
            d.nblk = d.ntile * ((it.g.nt + d.tc - 1) / d.tc);
            d.blocked = blocked && it.g.L % 4 == 0;
            d.slot0 = slot;
            h->push_back(d);
            for (int j = 0; j < it.ncol; j++) sp0->push_back(slot + j * d.nblk);
            blk += d.nblk * it.ncol / kc;
            slot += d.nblk * it.ncol;
            seg += it.ncol;
        }
        sp0->push_back(slot);
        return blk;
    };
    auto upload = [&](int kind, const std::vector<BEODom>& h) -> dd_status {
        dd_status ee = DD_OK;
        BEODom* dev = (BEODom*)workspace(c, kind == 0 ? W_BATCH0 : W_BATCH4, sizeof(BEODom) * n, &ee);
        if (ee != DD_OK) return ee;
        DD_HIP(c, hipMemcpyAsync(dev, h.data(), sizeof(BEODom) * n, hipMemcpyHostToDevice, c->stream));
        DD_HIP(c, hipStreamSynchronize(c->stream));  // h is pageable host memory
        S.doms[kind] = dev;
        return DD_OK;
    };
    // chunk length, columns per workgroup, tile shape and XCD remap per precision: timed on
    // the batch's Schur operator at first use (cached per batch signature), on work vectors
    // whose contents do not matter
    std::string sig;
    for (const Item& it : its)
        sig += ":" + std::to_string(it.g.T) + "x" + std::to_string(it.g.L) + "x" + std::to_string(it.ncol) + "b" +
               std::to_string(it.g.bc);
    SegLayout lay;
    std::vector<BEODom> hk;
    for (int kind = 0; kind < (mixed ? 2 : 1); kind++) {
        const std::string key = "beo:" + std::to_string(kind) + sig;
        int tc = 4, rmap = 0, kcb = 1, blk = 0;
        // columns per workgroup: FP32 may share link loads between 2 columns of a domain
        auto kc_ok = [&](int kc) {
            if (kc == 1) return true;
            if (kind == 0 || kc != 2) return false;
            for (const Item& it : its)
                if (it.ncol % kc != 0) return false;
            return true;
        };
        const auto hit = c->sched.find(key);
        if (hit != c->sched.end() && kc_ok(hit->second.kc)) {
            tc = hit->second.tc;
            rmap = hit->second.remap;
            kcb = hit->second.kc;
            blk = hit->second.blocked;
        } else {
            hipEvent_t ea, eb;
            DD_HIP(c, hipEventCreate(&ea));
            DD_HIP(c, hipEventCreate(&eb));
            const int saved = c->timing;
            c->timing = 0;
            float best = 1e30f;
            std::vector<int> sp;
            auto run = [&]() {
                if (kind == 0) S.schur<double>(S.doms[0], S.tmp64, 0, EPI_STORE, bhat, x_e, nullptr, nullptr, nullptr);
                else S.schur<float>(S.doms[1], S.tmp32, 0, EPI_STORE, (const cpx<float>*)x_o, (cpx<float>*)x_e,
                                    nullptr, nullptr, nullptr);
            };
            bool any4 = false;  // some domain can take brick tiles
            for (const Item& it : its) any4 = any4 || it.g.L % 4 == 0;
            for (int t : {1, 2, 4, 8}) {
                for (int kc : {1, 2}) {
                    for (int bl = 0; bl < (any4 ? 2 : 1); bl++) {
                        if (!kc_ok(kc)) continue;
                        S.kc[kind] = kc;
                        S.nblk = (unsigned)build(t, kc, bl, kind, &hk, &sp);
                        S.host = hk;
                        e = upload(kind, hk);
                        if (e != DD_OK) break;
                        for (int rm = 0; rm < 2; rm++) {
                            S.remap[kind] = rm;
                            run();
                            run();
                            (void)hipEventRecord(ea, c->stream);
                            for (int r = 0; r < 3; r++) run();
                            (void)hipEventRecord(eb, c->stream);
                            (void)hipEventSynchronize(eb);
                            float ms = 0;
                            (void)hipEventElapsedTime(&ms, ea, eb);
                            if (ms < best) {
                                best = ms;
                                tc = t;
                                rmap = rm;
                                kcb = kc;
                                blk = bl;
                            }
                        }
                    }
                    if (e != DD_OK) break;
                }
                if (e != DD_OK) break;
            }
            c->timing = saved;
            S.nblk = 0;  // launches size themselves from nblk64 / nblk32 again
            (void)hipEventDestroy(ea);
            (void)hipEventDestroy(eb);
            if (e != DD_OK) return e;
            StencilSched keep;
            keep.nt = kBeoNT;
            keep.tc = tc;
            keep.remap = rmap;
            keep.kc = kcb;
            keep.blocked = blk;
            tune_cache_store(c, key, keep);
        }
        S.remap[kind] = rmap;
        S.kc[kind] = kcb;
        const unsigned nb = (unsigned)build(tc, kcb, blk, kind, &hk, &lay.sp0[kind]);
        if (kind == 0) {
            S.nblk64 = nb;
            S.host = hk;
        } else {
            S.nblk32 = nb;
        }
        e = upload(kind, hk);
        if (e != DD_OK) return e;
    }
    if (!mixed) lay.sp0[1] = lay.sp0[0];
    for (const Item& it : its) {
        const int hlen = 12 * (it.g.nsite >> 1);
        for (int j = 0; j < it.ncol; j++) {
            lay.off.push_back(hoff[&it - &its[0]] + (long long)j * hlen);
            lay.len.push_back(hlen);
        }
    }
    e = lay.upload(c, W_SEGS, &S);
    if (e != DD_OK) return e;

    // relative residuals refer to the original sources
    std::vector<long long> foff;
    std::vector<int> flen;
    for (const Item& it : its)
        for (int j = 0; j < it.ncol; j++) {
            foff.push_back(it.voff + (long long)j * 12 * it.g.nsite);
            flen.push_back(12 * it.g.nsite);
        }
    std::vector<double> bnorm;
    e = segment_norms(c, foff, flen, bcat, &bnorm);
    if (e != DD_OK) return e;
    S.ref_norm2 = bnorm.data();

    const dd_status st = solve_system(S, bhat, x_e, p, res);
    if (st != DD_OK && st != DD_ERR_NOCONV && st != DD_ERR_BREAKDOWN) return st;

    // odd sites, the full answer, and its true residual domain by domain
    cpx<double>* r = bb;  // b_e | b_o are no longer needed (2 nhalf = the full size)
    size_t pslots = 0;
    for (const Item& it : its) pslots = std::max(pslots, (size_t)it.ncol * stencil_slots(c, it.g, 0, it.ncol));
    double* partial = (double*)workspace(c, W_PART, std::max(pslots, S.nslots) * 3 * sizeof(double), &e);
    if (e != DD_OK) return e;
    for (int i = 0; i < n; i++) {
        const Item& it = its[i];
        const double m = 1.0 / (2.0 * it.kappa);
        launch_eo_hop64(c, it.g, U64 + eoff[i], 1.0 / m, 0.5 / m, 1, 0, x_e + hoff[i], b_o + hoff[i], x_o + hoff[i],
                        it.ncol);
        launch_eo_merge(c, it.g, it.ncol, x_e + hoff[i], x_o + hoff[i], xcat + it.voff);
    }
    for (int i = 0; i < n; i++) {
        const Item& it = its[i];
        launch_dslash<double>(c, it.g, it.U64, it.kappa, 0, EPI_RESID, xcat + it.voff, r + it.voff, bcat + it.voff,
                              it.ncol, partial, nullptr);
    }
    DD_HIP(c, hipGetLastError());
    std::vector<double> rr;
    e = segment_norms(c, foff, flen, r, &rr);
    if (e != DD_OK) return e;
    rel->assign(rr.size(), 0.0);
    bool ok = true, nonfinite = st == DD_ERR_BREAKDOWN;
    for (size_t k = 0; k < rr.size(); k++) {
        if (!std::isfinite(rr[k])) nonfinite = true;
        (*rel)[k] = bnorm[k] > 0 ? std::sqrt(rr[k] / bnorm[k]) : 0.0;
        if (!((*rel)[k] <= p.tol)) ok = false;
    }
    if (nonfinite) return fail(c, DD_ERR_BREAKDOWN, "non-finite values in the Krylov iteration");
    if (!ok) return fail(c, DD_ERR_NOCONV, "batched even-odd solve missed tol on some column");
    return DD_OK;
}

}  // namespace

}  // namespace dd

using namespace dd;

extern "C" dd_status dd_block_solve_batched(dd_ctx* c, int n, const dd_batch_item* items,
                                            const dd_solver_params* p, dd_solve_stats* stats) {
    if (c == nullptr) return DD_ERR_ARG;
    const auto t_start = std::chrono::steady_clock::now();
    if (n < 1 || items == nullptr) return fail(c, DD_ERR_ARG, "need n >= 1 items");
    dd_status e = check_params(c, p);
    if (e != DD_OK) return e;

    // validate the items and lay them out back to back
    std::vector<Item> its(n);
    SegLayout lay;
    long long voff = 0, uoff = 0;
    for (int i = 0; i < n; i++) {
        const dd_batch_item& it = items[i];
        const std::string tag = "batch item " + std::to_string(i);
        const dd_lattice& l = it.lat;
        if (l.T < 2 || l.L < 2 || (l.time_bc != -1 && l.time_bc != 0 && l.time_bc != 1))
            return fail(c, DD_ERR_ARG, tag + ": need T >= 2, L >= 2, time_bc in {-1, 0, 1}");
        const double V = (double)l.T * l.L * l.L * l.L;
        if (V * 144.0 >= 2147483647.0) return fail(c, DD_ERR_ARG, tag + ": lattice too large");
        if (it.nrhs < 1 || it.nrhs > DD_MAX_RHS) return fail(c, DD_ERR_ARG, tag + ": need 1 <= nrhs <= 12");
        if (!(it.kappa > 0) || !std::isfinite(it.kappa)) return fail(c, DD_ERR_ARG, tag + ": kappa must be positive");
        const size_t nv = (size_t)V;
        const size_t fbytes = (size_t)it.nrhs * 12 * nv * 16;
        if (!on_device(c, it.U, 36 * nv * 16, 16) || !on_device(c, it.b, fbytes, 16) ||
            !on_device(c, it.x, fbytes, 16))
            return fail(c, DD_ERR_ARG, tag + ": U, b and x must be device memory of the context's device, "
                                             "16-byte aligned and large enough");
        Item& m = its[i];
        m.g = make_geo(l, nullptr);
        m.kappa = it.kappa;
        m.ncol = it.nrhs;
        m.voff = voff;
        m.uoff = uoff;
        m.U64 = (const cpx<double>*)it.U;
        for (int j = 0; j < it.nrhs; j++) {
            lay.off.push_back(voff + (long long)j * 12 * m.g.nsite);
            lay.len.push_back(12 * m.g.nsite);
        }
        voff += (long long)it.nrhs * 12 * m.g.nsite;
        uoff += (long long)36 * m.g.vlink;
    }
    const size_t nelem = (size_t)voff;

    OwnStream own(c);
    e = own.enter();
    if (e != DD_OK) return e;

    cpx<double>* bcat = (cpx<double>*)workspace(c, W_BATCH1, nelem * sizeof(cpx<double>), &e);
    if (e != DD_OK) return e;
    cpx<double>* xcat = (cpx<double>*)workspace(c, W_BATCH2, nelem * sizeof(cpx<double>), &e);
    if (e != DD_OK) return e;
    for (int i = 0; i < n; i++)
        DD_HIP(c, hipMemcpyAsync(bcat + its[i].voff, items[i].b, (size_t)its[i].ncol * 12 * its[i].g.nsite * 16,
                                 hipMemcpyDeviceToDevice, c->stream));
    bool eo = p->precond == DD_PRECOND_EO;
    for (const Item& it : its) eo = eo && eo_applicable(it.g);
    if (eo) {
        SolveResult res;
        std::vector<double> rel;
        const dd_status st = solve_batch_eo(c, its, *p, bcat, xcat, &res, &rel);
        if (st != DD_OK && st != DD_ERR_NOCONV && st != DD_ERR_BREAKDOWN) return st;
        for (int i = 0; i < n; i++)
            DD_HIP(c, hipMemcpyAsync(items[i].x, xcat + its[i].voff, (size_t)its[i].ncol * 12 * its[i].g.nsite * 16,
                                     hipMemcpyDeviceToDevice, c->stream));
        DD_HIP(c, hipStreamSynchronize(c->stream));
        if (stats) {
            const double ms =
                std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
            int seg = 0;
            for (int i = 0; i < n; i++) {
                dd_solve_stats& s = stats[i];
                std::memset(&s, 0, sizeof(s));
                s.nrhs = its[i].ncol;
                s.updates = res.updates;
                s.restarts = res.restarts;
                s.ms = ms;
                for (int j = 0; j < its[i].ncol; j++, seg++) {
                    s.iters = std::max(s.iters, seg < (int)res.seg_iters.size() ? res.seg_iters[seg] : 0);
                    s.true_rel_resid[j] = seg < (int)rel.size() ? rel[seg] : 0.0;
                }
            }
        }
        return st;
    }

    BatchSystem S;
    S.c = c;
    S.ndom = n;
    S.nelem = nelem;
    S.graph = true;
    cpx<float>* U32 = nullptr;
    if (p->prec == DD_MIXED) {
        U32 = (cpx<float>*)workspace(c, W_BATCH3, (size_t)uoff * sizeof(cpx<float>), &e);
        if (e != DD_OK) return e;
        for (int i = 0; i < n; i++) launch_links_to_f32(c, (size_t)36 * its[i].g.vlink, its[i].U64, U32 + its[i].uoff);
        S.has32 = true;
    }

    // tile shapes, tuned on the batch (FP64 always: residuals; FP32 for mixed)
    {
        cpx<double>* t0 = (cpx<double>*)workspace(c, W_R, nelem * sizeof(cpx<double>), &e);
        if (e != DD_OK) return e;
        e = tune_batch<double>(c, S, its, 0, U32, bcat, t0, W_BATCH0);
        if (e != DD_OK) return e;
        if (S.has32) {
            cpx<float>* a = (cpx<float>*)workspace(c, W_R32, nelem * sizeof(cpx<float>), &e);
            if (e != DD_OK) return e;
            cpx<float>* bq = (cpx<float>*)workspace(c, W_RH32, nelem * sizeof(cpx<float>), &e);
            if (e != DD_OK) return e;
            launch_zero<float>(c, nelem, a);
            e = tune_batch<float>(c, S, its, 1, U32, a, bq, W_BATCH4);
            if (e != DD_OK) return e;
        }
    }
    for (int kind = 0; kind < 2; kind++) {
        lay.sp0[kind].clear();
        if (kind == 1 && !S.has32) {
            lay.sp0[kind].assign(lay.off.size() + 1, 0);
            continue;
        }
        for (const BDom& d : S.lk[kind].host)
            for (int j = 0; j < d.ncol; j++) lay.sp0[kind].push_back(d.slot0 + j * d.nsb * d.nchunk);
        lay.sp0[kind].push_back(S.lk[kind].nslot);
    }
    e = lay.upload(c, W_SEGS, &S);
    if (e != DD_OK) return e;

    SolveResult res;
    const dd_status st = solve_system(S, bcat, xcat, *p, &res);
    if (st != DD_OK && st != DD_ERR_NOCONV && st != DD_ERR_BREAKDOWN) return st;
    for (int i = 0; i < n; i++)
        DD_HIP(c, hipMemcpyAsync(items[i].x, xcat + its[i].voff, (size_t)its[i].ncol * 12 * its[i].g.nsite * 16,
                                 hipMemcpyDeviceToDevice, c->stream));
    DD_HIP(c, hipStreamSynchronize(c->stream));
    if (stats) {
        const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
        int seg = 0;
        for (int i = 0; i < n; i++) {
            dd_solve_stats& s = stats[i];
            std::memset(&s, 0, sizeof(s));
            s.nrhs = its[i].ncol;
            s.updates = res.updates;
            s.restarts = res.restarts;
            s.ms = ms;
            for (int j = 0; j < its[i].ncol; j++, seg++) {
                s.iters = std::max(s.iters, res.seg_iters[seg]);
                s.true_rel_resid[j] = res.rel[seg];
            }
        }
    }
    return st;
}
