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
#include <algorithm>
#include <chrono>
#include <cstring>

#include "dd_dslash.h"

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
            const double bytes = ((48.0 + extra) * sites_cols + 72.0 * sites) * sizeof(R);
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

    BatchSystem S;
    S.c = c;
    S.ndom = n;
    S.nelem = nelem;
    S.graph = true;
    cpx<double>* bcat = (cpx<double>*)workspace(c, W_BATCH1, nelem * sizeof(cpx<double>), &e);
    if (e != DD_OK) return e;
    cpx<double>* xcat = (cpx<double>*)workspace(c, W_BATCH2, nelem * sizeof(cpx<double>), &e);
    if (e != DD_OK) return e;
    cpx<float>* U32 = nullptr;
    if (p->prec == DD_MIXED) {
        U32 = (cpx<float>*)workspace(c, W_BATCH3, (size_t)uoff * sizeof(cpx<float>), &e);
        if (e != DD_OK) return e;
        for (int i = 0; i < n; i++) launch_links_to_f32(c, (size_t)36 * its[i].g.vlink, its[i].U64, U32 + its[i].uoff);
        S.has32 = true;
    }
    for (int i = 0; i < n; i++)
        DD_HIP(c, hipMemcpyAsync(bcat + its[i].voff, items[i].b, (size_t)its[i].ncol * 12 * its[i].g.nsite * 16,
                                 hipMemcpyDeviceToDevice, c->stream));

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
