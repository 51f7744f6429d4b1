// abi.hip -- the extern "C" entry points declared in dd.h: argument
// validation, workspace management, and the orchestration of the hot path
// (stencil, solves, factorised propagator, correlator, adjoint) on the
// context's stream.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <vector>

#include "dd_internal.h"

namespace dd {

dd_status fail(dd_ctx* c, dd_status st, const std::string& msg) {
    if (c) c->err = msg;
    return st;
}

dd_status hip_fail(dd_ctx* c, hipError_t e, const char* what) {
    return fail(c, DD_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

void* workspace(dd_ctx* c, Slot s, size_t bytes, dd_status* st) {
    Buffer& b = c->ws[s];
    if (bytes == 0) bytes = 256;
    if (b.bytes >= bytes) return b.ptr;
    if (b.ptr) {
        (void)hipStreamSynchronize(c->stream);
        (void)hipFree(b.ptr);
        b.ptr = nullptr;
        b.bytes = 0;
    }
    hipError_t e = hipMalloc(&b.ptr, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        b.ptr = nullptr;
        *st = fail(c, DD_ERR_NOMEM, "workspace allocation of " + std::to_string(bytes) + " bytes failed");
        return nullptr;
    }
    b.bytes = bytes;
    return b.ptr;
}

Geo make_geo(const dd_lattice& lat, const dd_domain* dom) {
    Geo g;
    g.L = lat.L;
    g.L2 = lat.L * lat.L;
    g.L3 = g.L2 * lat.L;
    g.T = lat.T;
    g.vlink = lat.T * g.L3;
    g.bc = lat.time_bc;
    if (dom == nullptr) {
        g.t0 = 0;
        g.nt = lat.T;
        g.whole = 1;
    } else {
        g.t0 = dom->t0;
        g.nt = dom->nt;
        g.whole = 0;
    }
    g.nsite = g.nt * g.L3;
    return g;
}

// ---------------------------------------------------------------- timing
void timing_begin(dd_ctx* c, hipEvent_t* ev) {
    hipEvent_t a;
    if (!c->event_pool.empty()) {
        a = c->event_pool.back();
        c->event_pool.pop_back();
    } else if (hipEventCreate(&a) != hipSuccess) {
        *ev = nullptr;
        return;
    }
    (void)hipEventRecord(a, c->stream);
    *ev = a;
}

void timing_end(dd_ctx* c, hipEvent_t start, const std::string& name, double bytes) {
    if (start == nullptr) return;
    int entry = -1;
    for (size_t i = 0; i < c->timing_entries.size(); i++)
        if (c->timing_entries[i].name == name) entry = (int)i;
    if (entry < 0) {
        c->timing_entries.push_back(TimingEntry{name, 0, 0, 0});
        entry = (int)c->timing_entries.size() - 1;
    }
    hipEvent_t b;
    if (!c->event_pool.empty()) {
        b = c->event_pool.back();
        c->event_pool.pop_back();
    } else if (hipEventCreate(&b) != hipSuccess) {
        c->event_pool.push_back(start);
        return;
    }
    (void)hipEventRecord(b, c->stream);
    c->pending.push_back(TimedLaunch{start, b, entry, bytes});
    if (c->pending.size() >= 4096) timing_harvest(c);
}

void timing_harvest(dd_ctx* c) {
    if (c->pending.empty()) return;
    (void)hipStreamSynchronize(c->stream);
    for (auto& t : c->pending) {
        float ms = 0;
        if (hipEventElapsedTime(&ms, t.start, t.stop) == hipSuccess) {
            TimingEntry& te = c->timing_entries[t.entry];
            te.ms += ms;
            te.launches += 1;
            te.bytes += t.bytes;
        }
        c->event_pool.push_back(t.start);
        c->event_pool.push_back(t.stop);
    }
    c->pending.clear();
}

bool on_device(dd_ctx* c, const void* p, size_t bytes, size_t align) {
    if (p == nullptr || (reinterpret_cast<uintptr_t>(p) % align) != 0) return false;
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    if (a.type != hipMemoryTypeDevice || a.device != c->device) return false;
    hipDeviceptr_t base = nullptr;
    size_t size = 0;
    if (hipMemGetAddressRange(&base, &size, (hipDeviceptr_t)p) == hipSuccess) {
        const char* lo = (const char*)base;
        const char* q = (const char*)p;
        if (q + bytes > lo + size) return false;
    } else {
        (void)hipGetLastError();
    }
    return true;
}

dd_status check_params(dd_ctx* c, const dd_solver_params* p, bool allow_guess) {
    if (p == nullptr) return fail(c, DD_ERR_ARG, "solver params are NULL");
    if (p->x0 != 0 && !(p->x0 == 1 && allow_guess))
        return fail(c, DD_ERR_ARG, allow_guess ? "solver x0 must be 0 or 1"
                                               : "solver x0 must be 0 (only dd_block_solve takes an initial guess)");
    if (!(p->tol > 0) || p->tol >= 1 || p->max_iter < 1)
        return fail(c, DD_ERR_ARG, "need 0 < tol < 1 and max_iter >= 1");
    if (p->prec != DD_FP64 && p->prec != DD_MIXED) return fail(c, DD_ERR_ARG, "solver prec must be DD_FP64 or DD_MIXED");
    if (!(p->delta >= 0) || p->delta >= 1) return fail(c, DD_ERR_ARG, "solver delta must lie in [0, 1)");
    if (p->solver != DD_BICGSTAB && p->solver != DD_CGNR) return fail(c, DD_ERR_ARG, "unknown solver kind");
    if (p->precond != DD_PRECOND_EO && p->precond != DD_PRECOND_NONE) return fail(c, DD_ERR_ARG, "unknown precond");
    return DD_OK;
}

}  // namespace dd

using namespace dd;

// ---------------------------------------------------------------- allocation-free scratch
// A file-scope device array that serves dd_pion_correlator_noalloc as its partial-sum and
// result scratch, so that call needs no allocation (each GPU the library runs on holds
// its own copy until the process ends).  Host code never uses the array's name as an
// address: dd_create looks up its device address once per device (with that device
// current) and every later use goes through that pointer.
namespace {
constexpr size_t kScratchDoubles = (size_t)1 << 18;  // 2 MiB
__device__ __align__(256) double scratch[kScratchDoubles];
constexpr int kMaxDevices = 64;
double* g_scratch_ptr[kMaxDevices] = {};
std::mutex g_scratch_mu;

// the device address of `scratch` on device dev (current), looked up on first use
dd_status resolve_scratch(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return DD_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[dev] != nullptr) return DD_OK;
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || ptr == nullptr) {
        (void)hipGetLastError();
        return DD_ERR_HIP;
    }
    g_scratch_ptr[dev] = (double*)ptr;
    return DD_OK;
}
}  // namespace

#define CHECK_PTR(c, p, bytes, align, name)                                                         \
    do {                                                                                             \
        if (!on_device(c, p, bytes, align))                                                          \
            return fail(c, DD_ERR_ARG, std::string(name) +                                          \
                                           ": null, misaligned, too small or not device memory of " \
                                           "the context's device");                                 \
    } while (0)


namespace {

dd_status check_dom(dd_ctx* c, const dd_domain* dom) {
    if (dom == nullptr) return DD_OK;
    if (dom->t0 < 0 || dom->t0 >= c->lat.T || dom->nt < 1 || dom->nt >= c->lat.T)
        return fail(c, DD_ERR_ARG, "slab must satisfy 0 <= t0 < T and 1 <= nt < T");
    return DD_OK;
}

dd_status check_kappa(dd_ctx* c, double kappa) {
    if (!(kappa > 0) || !std::isfinite(kappa)) return fail(c, DD_ERR_ARG, "kappa must be positive and finite");
    return DD_OK;
}

size_t vlink(const dd_lattice& l) { return (size_t)l.T * l.L * l.L * l.L; }

}  // namespace

extern "C" {

dd_status dd_create(const dd_lattice* lat, void* stream, dd_ctx** out) {
    if (out == nullptr) return DD_ERR_ARG;
    *out = nullptr;
    if (lat == nullptr || lat->T < 2 || lat->L < 2 || (lat->time_bc != -1 && lat->time_bc != 0 && lat->time_bc != 1))
        return DD_ERR_ARG;
    // index arithmetic is 32-bit: 144 * V complex numbers must fit
    if ((double)lat->T * lat->L * lat->L * lat->L * 144.0 >= 2147483647.0) return DD_ERR_ARG;
    dd_ctx* c = new (std::nothrow) dd_ctx();
    if (c == nullptr) return DD_ERR_NOMEM;
    c->lat = *lat;
    c->stream = (hipStream_t)stream;
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return DD_ERR_HIP;
    }
    c->ws.resize(W_NSLOTS);
    if (resolve_scratch(c->device) != DD_OK) {
        delete c;
        return DD_ERR_HIP;
    }
    tune_cache_load(c);
    *out = c;
    return DD_OK;
}

void dd_destroy(dd_ctx* c) {
    if (c == nullptr) return;
    (void)hipStreamSynchronize(c->stream);
    for (auto& b : c->ws)
        if (b.ptr) (void)hipFree(b.ptr);
    for (auto& t : c->pending) {
        (void)hipEventDestroy(t.start);
        (void)hipEventDestroy(t.stop);
    }
    for (auto e : c->event_pool) (void)hipEventDestroy(e);
    if (c->own_stream) (void)hipStreamDestroy(c->own_stream);
    if (c->host_state) (void)hipHostFree(c->host_state);
    if (c->host_dots) (void)hipHostFree(c->host_dots);
    delete c;
}

const char* dd_last_error(const dd_ctx* c) { return c ? c->err.c_str() : "null context"; }

dd_status dd_apply_dirac(dd_ctx* c, const void* U, double kappa, const dd_domain* dom, int nrhs, const void* in,
                         void* out, int prec) {
    if (c == nullptr) return DD_ERR_ARG;
    dd_status e = check_dom(c, dom);
    if (e != DD_OK) return e;
    if ((e = check_kappa(c, kappa)) != DD_OK) return e;
    if (nrhs < 1 || nrhs > 4 * DD_MAX_RHS) return fail(c, DD_ERR_ARG, "nrhs out of range");
    if (prec != DD_FP64 && prec != DD_FP32) return fail(c, DD_ERR_ARG, "prec must be DD_FP64 or DD_FP32");
    const Geo g = make_geo(c->lat, dom);
    const size_t cs = prec == DD_FP64 ? 16 : 8;
    const size_t fbytes = (size_t)nrhs * 12 * g.nsite * cs;
    CHECK_PTR(c, U, 36 * vlink(c->lat) * cs, cs, "U");
    CHECK_PTR(c, in, fbytes, cs, "in");
    CHECK_PTR(c, out, fbytes, cs, "out");
    const char* a = (const char*)in;
    const char* b = (const char*)out;
    if (a < b + fbytes && b < a + fbytes) return fail(c, DD_ERR_ARG, "in and out overlap");
    if (prec == DD_FP64)
        launch_dslash<double>(c, g, (const cpx<double>*)U, kappa, 0, EPI_STORE, (const cpx<double>*)in,
                              (cpx<double>*)out, nullptr, nrhs, nullptr, nullptr);
    else
        launch_dslash<float>(c, g, (const cpx<float>*)U, kappa, 0, EPI_STORE, (const cpx<float>*)in,
                             (cpx<float>*)out, nullptr, nrhs, nullptr, nullptr);
    DD_HIP(c, hipGetLastError());
    return DD_OK;
}

dd_status dd_frontier_hop(dd_ctx* c, const void* U, const dd_domain* dst, const dd_domain* src, int nrhs,
                          const void* in, void* out, double alpha) {
    if (c == nullptr) return DD_ERR_ARG;
    if (dst == nullptr || src == nullptr) return fail(c, DD_ERR_ARG, "frontier hop needs two slabs");
    dd_status e;
    if ((e = check_dom(c, dst)) != DD_OK || (e = check_dom(c, src)) != DD_OK) return e;
    if (nrhs < 1 || nrhs > 4 * DD_MAX_RHS) return fail(c, DD_ERR_ARG, "nrhs out of range");
    const int T = c->lat.T;
    for (int k = 0; k < dst->nt; k++) {
        const int t = (dst->t0 + k) % T;
        if (((t - src->t0) % T + T) % T < src->nt) return fail(c, DD_ERR_ARG, "frontier hop slabs overlap");
    }
    const int L3 = c->lat.L * c->lat.L * c->lat.L;
    CHECK_PTR(c, U, 36 * vlink(c->lat) * 16, 16, "U");
    CHECK_PTR(c, in, (size_t)nrhs * 12 * src->nt * L3 * 16, 16, "in");
    CHECK_PTR(c, out, (size_t)nrhs * 12 * dst->nt * L3 * 16, 16, "out");
    launch_frontier(c, c->lat, (const cpx<double>*)U, *dst, *src, nrhs, (const cpx<double>*)in, (cpx<double>*)out,
                    alpha);
    DD_HIP(c, hipGetLastError());
    return DD_OK;
}

dd_status dd_block_solve(dd_ctx* c, const void* U, double kappa, const dd_domain* dom, int nrhs, const void* b,
                         void* x, const dd_solver_params* p, dd_solve_stats* stats) {
    if (c == nullptr) return DD_ERR_ARG;
    dd_status e;
    if ((e = check_dom(c, dom)) != DD_OK || (e = check_params(c, p, true)) != DD_OK ||
        (e = check_kappa(c, kappa)) != DD_OK)
        return e;
    if (nrhs < 1 || nrhs > DD_MAX_RHS) return fail(c, DD_ERR_ARG, "nrhs must be in [1, 12]");
    const Geo g = make_geo(c->lat, dom);
    const size_t fbytes = (size_t)nrhs * 12 * g.nsite * 16;
    CHECK_PTR(c, U, 36 * vlink(c->lat) * 16, 16, "U");
    CHECK_PTR(c, b, fbytes, 16, "b");
    CHECK_PTR(c, x, fbytes, 16, "x");
    if (b == x) return fail(c, DD_ERR_ARG, "b and x must be different fields");
    return solve(c, (const cpx<double>*)U, kappa, g, nrhs, (const cpx<double>*)b, (cpx<double>*)x, *p, stats, 0);
}

// The factorised propagator with optional quark-line projections: nproj slices
// proj_t[i] (global time) whose crossing field is replaced by P_L = sum over the
// proj_nvec[i] vectors phi_i phi_i^+ of proj_phi[i] (Sec. 3.3, Eq. 16).
static dd_status factorized(dd_ctx* c, const void* U, double kappa, const int src[4], const dd_domain* doms, int ndom,
                     int overlap, int nproj, const int* proj_t, const int* proj_nvec, const void* const* proj_phi,
                     const dd_solver_params* p, void* S_fact, void* S_exact, dd_solve_stats* stats) {
    if (c == nullptr) return DD_ERR_ARG;
    dd_status e;
    if ((e = check_params(c, p)) != DD_OK || (e = check_kappa(c, kappa)) != DD_OK) return e;
    if (overlap < 0) return fail(c, DD_ERR_ARG, "overlap must be >= 0");
    if (src == nullptr || doms == nullptr || ndom < 2) return fail(c, DD_ERR_ARG, "need a source and >= 2 slabs");
    const dd_lattice& lat = c->lat;
    const int T = lat.T, L = lat.L, L3 = L * L * L;
    if (src[0] < 0 || src[0] >= T || src[1] < 0 || src[1] >= L || src[2] < 0 || src[2] >= L || src[3] < 0 ||
        src[3] >= L)
        return fail(c, DD_ERR_ARG, "source outside the lattice");
    // the slabs must partition [0, T)
    std::vector<int> owner(T, -1);
    for (int k = 0; k < ndom; k++) {
        if ((e = check_dom(c, &doms[k])) != DD_OK) return e;
        for (int j = 0; j < doms[k].nt; j++) {
            const int t = (doms[k].t0 + j) % T;
            if (owner[t] != -1) return fail(c, DD_ERR_ARG, "slabs overlap");
            owner[t] = k;
        }
    }
    for (int t = 0; t < T; t++)
        if (owner[t] == -1) return fail(c, DD_ERR_ARG, "slabs do not cover [0, T)");
    if (owner[src[0]] != 0) return fail(c, DD_ERR_ARG, "the source must lie in doms[0]");
    // block distances on the graph of non-zero blocks of D (time hops between
    // consecutive slabs; across the time edge only if time_bc != 0)
    std::vector<std::vector<int>> adj(ndom);
    for (int t = 0; t < T; t++) {
        const int tn = (t + 1) % T;
        if (tn == 0 && lat.time_bc == 0) continue;
        const int a = owner[t], b = owner[tn];
        if (a != b) {
            if (std::find(adj[a].begin(), adj[a].end(), b) == adj[a].end()) adj[a].push_back(b);
            if (std::find(adj[b].begin(), adj[b].end(), a) == adj[b].end()) adj[b].push_back(a);
        }
    }
    std::vector<int> dist(ndom, -1), order;
    std::deque<int> q;
    dist[0] = 0;
    q.push_back(0);
    while (!q.empty()) {
        const int a = q.front();
        q.pop_front();
        order.push_back(a);
        for (int b : adj[a])
            if (dist[b] < 0) {
                dist[b] = dist[a] + 1;
                q.push_back(b);
            }
    }
    if ((int)order.size() != ndom) return fail(c, DD_ERR_ARG, "slabs are not connected by D");
    // slabs whose solution crosses a frontier outward; with overlap regions they are also
    // solved on their extension (overlap slices more on both time sides), which must stay
    // shorter than the lattice
    std::vector<char> feeds(ndom, 0);
    for (int a = 0; a < ndom; a++)
        for (int b : adj[a])
            if (dist[b] == dist[a] + 1) feeds[a] = 1;
    for (int k = 0; k < ndom; k++)
        if (overlap > 0 && feeds[k] && doms[k].nt + 2 * overlap >= T)
            return fail(c, DD_ERR_ARG, "overlap too thick for slab " + std::to_string(k));

    const size_t V = vlink(lat);
    CHECK_PTR(c, U, 36 * V * 16, 16, "U");
    CHECK_PTR(c, S_fact, 144 * V * 16, 16, "S_fact");
    if (S_exact) CHECK_PTR(c, S_exact, 144 * V * 16, 16, "S_exact");
    if (nproj < 0) return fail(c, DD_ERR_ARG, "nproj must be >= 0");
    if (nproj > 0 && (proj_t == nullptr || proj_nvec == nullptr || proj_phi == nullptr))
        return fail(c, DD_ERR_ARG, "projection arrays are NULL");
    std::vector<char> projected(T, 0);
    for (int i = 0; i < nproj; i++) {
        const int t = proj_t[i], nv = proj_nvec[i];
        if (t < 0 || t >= T) return fail(c, DD_ERR_ARG, "projection slice outside [0, T)");
        if (projected[t]) return fail(c, DD_ERR_ARG, "slice " + std::to_string(t) + " projected twice");
        projected[t] = 1;
        if (nv < 1 || nv > std::min(kMaxProjVec, 6 * L3))
            return fail(c, DD_ERR_ARG, "projection basis size must be in [1, min(256, 6 L^3)]");
        CHECK_PTR(c, proj_phi[i], (size_t)nv * 12 * L3 * 16, 16, "proj_phi");
    }

    // per-slab solutions psi_k, stored compactly one after the other
    std::vector<size_t> base(ndom);
    size_t tot = 0;
    for (int k = 0; k < ndom; k++) {
        base[k] = tot;
        tot += (size_t)144 * doms[k].nt * L3;
    }
    cpx<double>* psi = (cpx<double>*)workspace(c, W_AUX2, tot * sizeof(cpx<double>), &e);
    if (e != DD_OK) return e;
    size_t maxslab = 0;
    for (int k = 0; k < ndom; k++) maxslab = std::max(maxslab, (size_t)144 * doms[k].nt * L3);
    cpx<double>* rhs = (cpx<double>*)workspace(c, W_AUX3, std::max(maxslab, S_exact ? 144 * V : 0) * sizeof(cpx<double>), &e);
    if (e != DD_OK) return e;
    // the fields that cross frontiers (psi itself without overlap regions), and the source
    // and solution on an extended slab
    cpx<double>* hop = psi;
    cpx<double>* ext = nullptr;
    size_t maxext = 0;
    if (overlap > 0) {
        hop = (cpx<double>*)workspace(c, W_AUX0, tot * sizeof(cpx<double>), &e);
        if (e != DD_OK) return e;
        for (int k = 0; k < ndom; k++)
            if (feeds[k]) maxext = std::max(maxext, (size_t)144 * (doms[k].nt + 2 * overlap) * L3);
        ext = (cpx<double>*)workspace(c, W_AUX1, 2 * maxext * sizeof(cpx<double>), &e);
        if (e != DD_OK) return e;
    }

    const int ssp = (src[3] * L + src[2]) * L + src[1];
    dd_status worst = DD_OK;
    for (int k : order) {
        const dd_domain& dk = doms[k];
        const int nsite = dk.nt * L3;
        if (dist[k] == 0) {
            const int tl = ((src[0] - dk.t0) % T + T) % T;
            launch_point_source(c, nsite, tl * L3 + ssp, rhs);
        } else {
            launch_zero<double>(c, (size_t)144 * nsite, rhs);
            for (int j = 0; j < ndom; j++)
                if (dist[j] == dist[k] - 1 && std::find(adj[k].begin(), adj[k].end(), j) != adj[k].end())
                    launch_frontier(c, lat, (const cpx<double>*)U, dk, doms[j], 12, hop + base[j], rhs, -1.0);
        }
        DD_HIP(c, hipGetLastError());
        const Geo g = make_geo(lat, &dk);
        e = solve(c, (const cpx<double>*)U, kappa, g, 12, rhs, psi + base[k], *p, stats ? &stats[k] : nullptr, 0);
        if (e != DD_OK && e != DD_ERR_NOCONV) return e;
        if (e == DD_ERR_NOCONV) worst = e;
        launch_slab_scatter(c, lat, dk, 12, psi + base[k], (cpx<double>*)S_fact);
        if (overlap > 0 && feeds[k]) {
            // the same source on the slab grown by overlap slices on both sides; its part on
            // slab k is what crosses the frontiers (Sec. 3.2, Gamma-bar)
            const int ntb = dk.nt + 2 * overlap;
            const dd_domain dx{((dk.t0 - overlap) % T + T) % T, ntb};
            cpx<double>*rx = ext, *xx = ext + maxext;
            launch_zero<double>(c, (size_t)144 * ntb * L3, rx);
            launch_slab_embed(c, L3, ntb, overlap, dk.nt, 12, rhs, rx, 0);
            DD_HIP(c, hipGetLastError());
            dd_solve_stats sx;
            e = solve(c, (const cpx<double>*)U, kappa, make_geo(lat, &dx), 12, rx, xx, *p, stats ? &sx : nullptr, 0);
            if (e != DD_OK && e != DD_ERR_NOCONV) return e;
            if (e == DD_ERR_NOCONV) worst = e;
            if (stats) {
                dd_solve_stats& sk = stats[k];
                sk.iters += sx.iters;
                sk.updates += sx.updates;
                sk.restarts += sx.restarts;
                sk.ms += sx.ms;
                for (int j = 0; j < 12; j++) sk.true_rel_resid[j] = std::max(sk.true_rel_resid[j], sx.true_rel_resid[j]);
            }
            launch_slab_embed(c, L3, ntb, overlap, dk.nt, 12, hop + base[k], xx, 1);
        }
        // the quark line is cut on the projected slices of this slab's crossing field
        // (S_fact on the slab keeps the unprojected solution, already scattered)
        for (int i = 0; feeds[k] && i < nproj; i++) {
            const int kl = ((proj_t[i] - dk.t0) % T + T) % T;
            if (kl >= dk.nt) continue;
            e = project_slice(c, L3, dk.nt, kl, 12, hop + base[k], proj_nvec[i], (const cpx<double>*)proj_phi[i]);
            if (e != DD_OK) return e;
        }
    }
    if (S_exact) {
        launch_point_source(c, (int)V, src[0] * L3 + ssp, rhs);
        const Geo g = make_geo(lat, nullptr);
        e = solve(c, (const cpx<double>*)U, kappa, g, 12, rhs, (cpx<double>*)S_exact, *p,
                  stats ? &stats[ndom] : nullptr, 0);
        if (e != DD_OK && e != DD_ERR_NOCONV) return e;
        if (e == DD_ERR_NOCONV) worst = e;
    }
    DD_HIP(c, hipStreamSynchronize(c->stream));
    if (worst != DD_OK) return fail(c, worst, "a slab or whole-lattice solve did not converge: " + c->err);
    return DD_OK;
}

dd_status dd_factorized_propagator(dd_ctx* c, const void* U, double kappa, const int src[4], const dd_domain* doms,
                                   int ndom, int overlap, const dd_solver_params* p, void* S_fact, void* S_exact,
                                   dd_solve_stats* stats) {
    return factorized(c, U, kappa, src, doms, ndom, overlap, 0, nullptr, nullptr, nullptr, p, S_fact, S_exact,
                      stats);
}

dd_status dd_factorized_propagator_projected(dd_ctx* c, const void* U, double kappa, const int src[4],
                                             const dd_domain* doms, int ndom, int overlap, int nproj,
                                             const int* proj_t, const int* proj_nvec, const void* const* proj_phi,
                                             const dd_solver_params* p, void* S_fact, void* S_exact,
                                             dd_solve_stats* stats) {
    return factorized(c, U, kappa, src, doms, ndom, overlap, nproj, proj_t, proj_nvec, proj_phi, p, S_fact,
                      S_exact, stats);
}

dd_status dd_projection_basis(dd_ctx* c, const void* U, double kappa, const dd_domain* pi, int t_slice, int sign,
                              int nvec, int n_iter, const void* v0, void* phi, const dd_solver_params* p,
                              dd_solve_stats* stats) {
    if (c == nullptr) return DD_ERR_ARG;
    dd_status e;
    if (pi == nullptr) return fail(c, DD_ERR_ARG, "pi is NULL");
    if ((e = check_dom(c, pi)) != DD_OK || (e = check_params(c, p)) != DD_OK || (e = check_kappa(c, kappa)) != DD_OK)
        return e;
    const dd_lattice& lat = c->lat;
    const int T = lat.T, L3 = lat.L * lat.L * lat.L;
    if (t_slice < 0 || t_slice >= T) return fail(c, DD_ERR_ARG, "t_slice outside [0, T)");
    const int k = ((t_slice - pi->t0) % T + T) % T;
    if (k >= pi->nt) return fail(c, DD_ERR_ARG, "t_slice outside the slab");
    if (sign != 1 && sign != -1) return fail(c, DD_ERR_ARG, "sign must be +1 or -1");
    if (nvec < 1 || nvec > std::min(kMaxProjVec, 6 * L3))
        return fail(c, DD_ERR_ARG, "nvec must be in [1, min(256, 6 L^3)]");
    if (n_iter < 0) return fail(c, DD_ERR_ARG, "n_iter must be >= 0");
    const Geo g = make_geo(lat, pi);
    CHECK_PTR(c, U, 36 * vlink(lat) * 16, 16, "U");
    CHECK_PTR(c, v0, (size_t)nvec * 12 * g.nsite * 16, 16, "v0");
    CHECK_PTR(c, phi, (size_t)nvec * 12 * L3 * 16, 16, "phi");
    return projection_basis(c, (const cpx<double>*)U, kappa, g, k, sign, nvec, n_iter, (const cpx<double>*)v0,
                            (cpx<double>*)phi, *p, stats);
}

dd_status dd_disconnected_traces(dd_ctx* c, const void* U, double kappa, const dd_domain* doms, int ndom, int nsrc,
                                 const void* eta, int n_hop, const dd_solver_params* p, void* tau,
                                 dd_solve_stats* stats) {
    if (c == nullptr) return DD_ERR_ARG;
    dd_status e;
    if ((e = check_params(c, p)) != DD_OK || (e = check_kappa(c, kappa)) != DD_OK) return e;
    const dd_lattice& lat = c->lat;
    const int T = lat.T;
    if (nsrc < 1) return fail(c, DD_ERR_ARG, "nsrc must be >= 1");
    if (n_hop < 0 || n_hop > 16) return fail(c, DD_ERR_ARG, "n_hop must be in [0, 16]");
    if (doms == nullptr && ndom != 0) return fail(c, DD_ERR_ARG, "doms is NULL but ndom != 0");
    if (doms != nullptr) {
        if (ndom < 1) return fail(c, DD_ERR_ARG, "ndom must be >= 1");
        std::vector<char> used(T, 0);
        for (int k = 0; k < ndom; k++) {
            if ((e = check_dom(c, &doms[k])) != DD_OK) return e;
            for (int j = 0; j < doms[k].nt; j++) {
                const int t = (doms[k].t0 + j) % T;
                if (used[t]) return fail(c, DD_ERR_ARG, "domains overlap");
                used[t] = 1;
            }
        }
    }
    const size_t V = vlink(lat);
    CHECK_PTR(c, U, 36 * V * 16, 16, "U");
    CHECK_PTR(c, eta, (size_t)nsrc * 12 * V * 16, 16, "eta");
    CHECK_PTR(c, tau, (size_t)nsrc * T * 16, 16, "tau");
    return disconnected_traces(c, (const cpx<double>*)U, kappa, doms, ndom, nsrc, (const cpx<double>*)eta, n_hop, *p,
                               (cpx<double>*)tau, stats);
}

dd_status dd_disconnected_correlator(dd_ctx* c, int nsrc, const void* tau, double* C_host) {
    if (c == nullptr) return DD_ERR_ARG;
    if (nsrc < 2) return fail(c, DD_ERR_ARG, "nsrc must be >= 2 (the product runs over distinct sources)");
    if (C_host == nullptr) return fail(c, DD_ERR_ARG, "C_host is NULL");
    CHECK_PTR(c, tau, (size_t)nsrc * c->lat.T * 16, 16, "tau");
    return disconnected_correlator(c, nsrc, (const cpx<double>*)tau, C_host);
}

dd_status dd_nucleon_lines(dd_ctx* c, const void* U, double kappa, const dd_domain* gbar, const dd_domain* gstar,
                           int t_phi, int nvec, const void* phi, int x0, void* xi, void* eta,
                           const dd_solver_params* p, dd_solve_stats* stats) {
    if (c == nullptr) return DD_ERR_ARG;
    if (gbar == nullptr || gstar == nullptr) return fail(c, DD_ERR_ARG, "gbar and gstar must be slabs");
    dd_status e;
    if ((e = check_dom(c, gbar)) != DD_OK || (e = check_dom(c, gstar)) != DD_OK || (e = check_params(c, p)) != DD_OK ||
        (e = check_kappa(c, kappa)) != DD_OK)
        return e;
    const dd_lattice& lat = c->lat;
    const int T = lat.T, L3 = lat.L * lat.L * lat.L;
    auto in = [&](const dd_domain& d, int t) { return t >= 0 && t < T && ((t - d.t0) % T + T) % T < d.nt; };
    if (!in(*gbar, t_phi) || !in(*gbar, x0)) return fail(c, DD_ERR_ARG, "t_phi and x0 must lie in gbar");
    if (in(*gstar, t_phi)) return fail(c, DD_ERR_ARG, "t_phi must lie outside gstar");
    const bool before = (t_phi + 1) % T == gstar->t0, after = (gstar->t0 + gstar->nt) % T == t_phi;
    const bool wrap_ok = lat.time_bc != 0 || (before ? t_phi != T - 1 : t_phi != 0);
    if (!(before || after) || !wrap_ok) return fail(c, DD_ERR_ARG, "t_phi must be a time neighbour of gstar");
    if (nvec < 1 || nvec > std::min(kMaxProjVec, 6 * L3))
        return fail(c, DD_ERR_ARG, "nvec must be in [1, min(256, 6 L^3)]");
    const size_t V = vlink(lat);
    CHECK_PTR(c, U, 36 * V * 16, 16, "U");
    CHECK_PTR(c, phi, (size_t)nvec * 12 * L3 * 16, 16, "phi");
    CHECK_PTR(c, xi, (size_t)nvec * 12 * L3 * 16, 16, "xi");
    CHECK_PTR(c, eta, (size_t)nvec * 12 * gstar->nt * L3 * 16, 16, "eta");
    return nucleon_lines(c, (const cpx<double>*)U, kappa, *gbar, *gstar, t_phi, nvec, (const cpx<double>*)phi, x0,
                         (cpx<double>*)xi, (cpx<double>*)eta, *p, stats);
}

dd_status dd_baryon_blocks(dd_ctx* c, int nvec, int nt, const void* s, void* B) {
    if (c == nullptr) return DD_ERR_ARG;
    const int L3 = c->lat.L * c->lat.L * c->lat.L;
    if (nvec < 1 || nvec > kMaxProjVec) return fail(c, DD_ERR_ARG, "nvec must be in [1, 256]");
    if (nt < 1 || nt > c->lat.T) return fail(c, DD_ERR_ARG, "nt must be in [1, T]");
    CHECK_PTR(c, s, (size_t)nvec * 12 * nt * L3 * 16, 16, "s");
    CHECK_PTR(c, B, (size_t)nt * 4 * nvec * nvec * nvec * 16, 16, "B");
    const char* a = (const char*)s;
    const char* b = (const char*)B;
    const size_t na = (size_t)nvec * 12 * nt * L3 * 16, nb = (size_t)nt * 4 * nvec * nvec * nvec * 16;
    if (a < b + nb && b < a + na) return fail(c, DD_ERR_ARG, "s and B overlap");
    return baryon_blocks(c, nvec, nt, (const cpx<double>*)s, (cpx<double>*)B);
}

dd_status dd_nucleon_contract(dd_ctx* c, int nvec, int ntx, const void* Bx, int nty, const void* By, double* W_host) {
    if (c == nullptr) return DD_ERR_ARG;
    if (nvec < 1 || nvec > kMaxProjVec) return fail(c, DD_ERR_ARG, "nvec must be in [1, 256]");
    if (ntx < 1 || nty < 1 || ntx > c->lat.T || nty > c->lat.T) return fail(c, DD_ERR_ARG, "ntx, nty must be in [1, T]");
    if (W_host == nullptr) return fail(c, DD_ERR_ARG, "W_host is NULL");
    const size_t sl = (size_t)4 * nvec * nvec * nvec * 16;
    CHECK_PTR(c, Bx, ntx * sl, 16, "Bx");
    CHECK_PTR(c, By, nty * sl, 16, "By");
    return nucleon_contract(c, nvec, ntx, (const cpx<double>*)Bx, nty, (const cpx<double>*)By, W_host);
}

dd_status dd_pion_correlator(dd_ctx* c, const void* S, int ncol, int t_src, double* C_host) {
    if (c == nullptr) return DD_ERR_ARG;
    if (ncol < 1 || ncol > 4 * DD_MAX_RHS) return fail(c, DD_ERR_ARG, "ncol out of range");
    if (t_src < 0 || t_src >= c->lat.T) return fail(c, DD_ERR_ARG, "t_src outside [0, T)");
    if (C_host == nullptr) return fail(c, DD_ERR_ARG, "C_host is NULL");
    const size_t V = vlink(c->lat);
    CHECK_PTR(c, S, (size_t)ncol * 12 * V * 16, 16, "S");
    dd_status e = DD_OK;
    double* partial = (double*)workspace(c, W_PART, (size_t)c->lat.T * 12 * ncol * 3 * sizeof(double), &e);
    if (e != DD_OK) return e;
    double* Cd = (double*)workspace(c, W_DOTS, (size_t)c->lat.T * sizeof(double), &e);
    if (e != DD_OK) return e;
    launch_pion(c, c->lat, ncol, (const cpx<double>*)S, t_src, partial, Cd);
    DD_HIP(c, hipGetLastError());
    DD_HIP(c, hipMemcpyAsync(C_host, Cd, sizeof(double) * c->lat.T, hipMemcpyDeviceToHost, c->stream));
    DD_HIP(c, hipStreamSynchronize(c->stream));
    return DD_OK;
}

dd_status dd_pion_correlator_noalloc(dd_ctx* c, const void* S, int ncol, int t_src, double* C_host) {
    if (c == nullptr) return DD_ERR_ARG;
    if (ncol < 1 || ncol > 4 * DD_MAX_RHS) return fail(c, DD_ERR_ARG, "ncol out of range");
    if (t_src < 0 || t_src >= c->lat.T) return fail(c, DD_ERR_ARG, "t_src outside [0, T)");
    if (C_host == nullptr) return fail(c, DD_ERR_ARG, "C_host is NULL");
    const size_t V = vlink(c->lat);
    CHECK_PTR(c, S, (size_t)ncol * 12 * V * 16, 16, "S");
    const size_t T = (size_t)c->lat.T;
    const size_t npart = T * 12 * (size_t)ncol * 3;  // the pion kernels' partial sums, then C
    if (npart + T > kScratchDoubles)
        return fail(c, DD_ERR_ARG, "dd_pion_correlator_noalloc: 36 T ncol + T = " + std::to_string(npart + T) +
                                       " doubles exceed the static scratch of " + std::to_string(kScratchDoubles));
    double* base = c->device >= 0 && c->device < kMaxDevices ? g_scratch_ptr[c->device] : nullptr;
    if (base == nullptr) return fail(c, DD_ERR_HIP, "static scratch not resolved for this device");
    launch_pion(c, c->lat, ncol, (const cpx<double>*)S, t_src, base, base + npart);
    DD_HIP(c, hipGetLastError());
    DD_HIP(c, hipMemcpyAsync(C_host, base + npart, sizeof(double) * T, hipMemcpyDeviceToHost, c->stream));
    DD_HIP(c, hipStreamSynchronize(c->stream));
    return DD_OK;
}

dd_status dd_block_solve_backward(dd_ctx* c, const void* U, double kappa, const dd_domain* dom, int nrhs,
                                  const void* x, const void* grad_x, void* grad_b, void* grad_U,
                                  const dd_solver_params* p, dd_solve_stats* stats) {
    if (c == nullptr) return DD_ERR_ARG;
    dd_status e;
    if ((e = check_dom(c, dom)) != DD_OK || (e = check_params(c, p)) != DD_OK || (e = check_kappa(c, kappa)) != DD_OK)
        return e;
    if (nrhs < 1 || nrhs > DD_MAX_RHS) return fail(c, DD_ERR_ARG, "nrhs must be in [1, 12]");
    const Geo g = make_geo(c->lat, dom);
    const size_t fbytes = (size_t)nrhs * 12 * g.nsite * 16;
    CHECK_PTR(c, U, 36 * vlink(c->lat) * 16, 16, "U");
    CHECK_PTR(c, x, fbytes, 16, "x");
    CHECK_PTR(c, grad_x, fbytes, 16, "grad_x");
    CHECK_PTR(c, grad_b, fbytes, 16, "grad_b");
    if (grad_U) CHECK_PTR(c, grad_U, 36 * vlink(c->lat) * 16, 16, "grad_U");
    // D^+ lambda = grad_x
    e = solve(c, (const cpx<double>*)U, kappa, g, nrhs, (const cpx<double>*)grad_x, (cpx<double>*)grad_b, *p, stats,
              1);
    if (e != DD_OK) return e;
    // dL = -Re<lambda, dD x> = 1/2 d(-2 Re<lambda, D x>)
    if (grad_U)
        launch_link_force(c, g, nrhs, (const cpx<double>*)x, (const cpx<double>*)grad_b, 0.5, (cpx<double>*)grad_U);
    DD_HIP(c, hipGetLastError());
    DD_HIP(c, hipStreamSynchronize(c->stream));
    return DD_OK;
}

dd_status dd_domain_action(dd_ctx* c, const void* U, double kappa, const dd_domain* dom, int nrhs, const void* phi,
                           void* X, void* Y, double* S_host, const dd_solver_params* p, dd_solve_stats* stats) {
    if (c == nullptr) return DD_ERR_ARG;
    dd_status e;
    if ((e = check_dom(c, dom)) != DD_OK || (e = check_params(c, p)) != DD_OK || (e = check_kappa(c, kappa)) != DD_OK)
        return e;
    if (nrhs < 1 || nrhs > DD_MAX_RHS) return fail(c, DD_ERR_ARG, "nrhs must be in [1, 12]");
    const Geo g = make_geo(c->lat, dom);
    const size_t fbytes = (size_t)nrhs * 12 * g.nsite * 16;
    CHECK_PTR(c, U, 36 * vlink(c->lat) * 16, 16, "U");
    CHECK_PTR(c, phi, fbytes, 16, "phi");
    CHECK_PTR(c, X, fbytes, 16, "X");
    CHECK_PTR(c, Y, fbytes, 16, "Y");
    dd_solve_stats s2{};
    e = solve(c, (const cpx<double>*)U, kappa, g, nrhs, (const cpx<double>*)phi, (cpx<double>*)Y, *p, stats, 1);
    if (e != DD_OK) return e;
    e = solve(c, (const cpx<double>*)U, kappa, g, nrhs, (const cpx<double>*)Y, (cpx<double>*)X, *p, &s2, 0);
    if (stats) {
        stats->iters += s2.iters;
        stats->updates += s2.updates;
        stats->restarts += s2.restarts;
        stats->ms += s2.ms;
        for (int j = 0; j < nrhs; j++) stats->true_rel_resid[j] = std::max(stats->true_rel_resid[j], s2.true_rel_resid[j]);
    }
    if (e != DD_OK) return e;
    if (S_host) {
        std::vector<double> nn;
        e = column_norms(c, 12 * g.nsite, nrhs, (const cpx<double>*)Y, &nn);
        if (e != DD_OK) return e;
        double s = 0;
        for (double v : nn) s += v;
        *S_host = s;
    }
    DD_HIP(c, hipStreamSynchronize(c->stream));
    return DD_OK;
}

dd_status dd_domain_action_backward(dd_ctx* c, const dd_domain* dom, int nrhs, const void* X, const void* Y,
                                    double g_S, void* grad_U, void* grad_phi) {
    if (c == nullptr) return DD_ERR_ARG;
    dd_status e;
    if ((e = check_dom(c, dom)) != DD_OK) return e;
    if (nrhs < 1 || nrhs > DD_MAX_RHS) return fail(c, DD_ERR_ARG, "nrhs must be in [1, 12]");
    if (!std::isfinite(g_S)) return fail(c, DD_ERR_ARG, "g_S must be finite");
    const Geo g = make_geo(c->lat, dom);
    const size_t n = (size_t)nrhs * 12 * g.nsite;
    CHECK_PTR(c, X, n * 16, 16, "X");
    CHECK_PTR(c, Y, n * 16, 16, "Y");
    CHECK_PTR(c, grad_U, 36 * vlink(c->lat) * 16, 16, "grad_U");
    CHECK_PTR(c, grad_phi, n * 16, 16, "grad_phi");
    launch_link_force(c, g, nrhs, (const cpx<double>*)X, (const cpx<double>*)Y, g_S, (cpx<double>*)grad_U);
    launch_scale(c, n, 2.0 * g_S, (const cpx<double>*)X, (cpx<double>*)grad_phi);
    DD_HIP(c, hipGetLastError());
    return DD_OK;
}

dd_status dd_link_force(dd_ctx* c, const dd_domain* dom, int nrhs, const void* X, const void* Y, double coeff,
                        void* grad_U) {
    if (c == nullptr) return DD_ERR_ARG;
    dd_status e;
    if ((e = check_dom(c, dom)) != DD_OK) return e;
    if (nrhs < 1 || nrhs > 4 * DD_MAX_RHS) return fail(c, DD_ERR_ARG, "nrhs out of range");
    const Geo g = make_geo(c->lat, dom);
    const size_t fbytes = (size_t)nrhs * 12 * g.nsite * 16;
    CHECK_PTR(c, X, fbytes, 16, "X");
    CHECK_PTR(c, Y, fbytes, 16, "Y");
    CHECK_PTR(c, grad_U, 36 * vlink(c->lat) * 16, 16, "grad_U");
    launch_link_force(c, g, nrhs, (const cpx<double>*)X, (const cpx<double>*)Y, coeff, (cpx<double>*)grad_U);
    DD_HIP(c, hipGetLastError());
    return DD_OK;
}

dd_status dd_set_kernel_timing(dd_ctx* c, int enable) {
    if (c == nullptr) return DD_ERR_ARG;
    timing_harvest(c);
    c->timing = enable ? 1 : 0;
    c->timing_entries.clear();
    return DD_OK;
}

dd_status dd_kernel_timing_count(dd_ctx* c, int* count) {
    if (c == nullptr || count == nullptr) return DD_ERR_ARG;
    timing_harvest(c);
    *count = (int)c->timing_entries.size();
    return DD_OK;
}

dd_status dd_kernel_timing(dd_ctx* c, int index, char* name, int name_len, double* ms, long long* launches,
                           double* bytes) {
    if (c == nullptr) return DD_ERR_ARG;
    timing_harvest(c);
    if (index < 0 || index >= (int)c->timing_entries.size())
        return fail(c, DD_ERR_ARG, "timing index out of range");
    const TimingEntry& te = c->timing_entries[index];
    if (name != nullptr && name_len > 0) {
        const size_t k = std::min((size_t)name_len - 1, te.name.size());
        std::memcpy(name, te.name.data(), k);
        name[k] = 0;
    }
    if (ms) *ms = te.ms;
    if (launches) *launches = te.launches;
    if (bytes) *bytes = te.bytes;
    return DD_OK;
}

}  // extern "C"
