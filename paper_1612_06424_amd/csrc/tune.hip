// tune.hip -- per-context autotuner of the stencil launch shape.
//
// The best (workgroup size, time-chunk length, XCD remap, columns per thread,
// tile shape and order) depends on the precision, the number of columns and the
// lattice geometry (how many
// workgroups are resident per XCD against how much of the 4 MB L2 one time
// slice of them touches).  The first launch for a new key times every
// candidate on scratch buffers of the same size (best of three timings) and
// keeps the fastest; later
// launches reuse it.  Small problems use the default shape untimed.
//
// With the environment variable DD_TUNE_CACHE naming a file, a new context
// loads the choices stored there and every new choice is appended to it, so
// that separate processes (for instance the passes of a profiler) launch the
// same shapes.
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <sstream>
#include <string>

#include "dd_internal.h"

namespace dd {

namespace {

std::string key_of(const Geo& g, int kind, int ncol) {
    return std::to_string(kind) + ":" + std::to_string(ncol) + ":" + std::to_string(g.L) + ":" +
           std::to_string(g.T) + ":" + std::to_string(g.nt) + ":" + std::to_string(g.whole);
}

template <typename R>
StencilSched tune(dd_ctx* c, const Geo& g, int ncol) {
    StencilSched best = default_sched(g);
    const size_t nf = (size_t)ncol * 12 * g.nsite, nl = (size_t)36 * g.vlink;
    cpx<R>*in = nullptr, *out = nullptr, *U = nullptr;
    if (hipMalloc(&in, nf * sizeof(cpx<R>)) != hipSuccess || hipMalloc(&out, nf * sizeof(cpx<R>)) != hipSuccess ||
        hipMalloc(&U, nl * sizeof(cpx<R>)) != hipSuccess) {
        (void)hipGetLastError();
        if (in) (void)hipFree(in);
        if (out) (void)hipFree(out);
        if (U) (void)hipFree(U);
        return best;
    }
    (void)hipMemsetAsync(in, 0, nf * sizeof(cpx<R>), c->stream);
    (void)hipMemsetAsync(U, 0, nl * sizeof(cpx<R>), c->stream);
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    const int saved_timing = c->timing;
    c->timing = 0;
    float best_ms = 1e30f;
    const int tcs[] = {4, 8, 16, 1 << 20};
    for (int kc = 1; kc <= 4; kc++)
    for (int nt : {128, 256})
        for (int tcv : tcs)
            for (int remap : {0, 1})
            for (int bl = 0; bl < 4; bl++) {
                StencilSched sc;
                sc.nt = nt;
                sc.tc = tcv > g.nt ? g.nt : tcv;
                sc.remap = remap;
                sc.kc = kc;
                sc.blocked = bl;
                if (tcv != sc.tc && tcv != (1 << 20)) continue;  // same as a shorter candidate
                if (sched_kc(sc, ncol, sizeof(R), (size_t)12 * g.nsite * sizeof(cpx<R>)) != kc) continue;
                if ((bl & 1) && brick_rows(g, nt) == 0) continue;          // bricks do not fit
                if ((bl & 2) && (g.nt + sc.tc - 1) / sc.tc < 2) continue;  // one chunk: the same order
                for (int w = 0; w < 2; w++)
                    launch_dslash_sched<R>(c, g, sc, U, 0.125, 0, EPI_STORE, in, out, nullptr, ncol, nullptr, nullptr);
                // the best of three timings of three launches each (one timing picked shapes by noise)
                float ms = 1e30f;
                for (int rep = 0; rep < 3; rep++) {
                    (void)hipEventRecord(e0, c->stream);
                    for (int r = 0; r < 3; r++)
                        launch_dslash_sched<R>(c, g, sc, U, 0.125, 0, EPI_STORE, in, out, nullptr, ncol, nullptr,
                                               nullptr);
                    (void)hipEventRecord(e1, c->stream);
                    (void)hipEventSynchronize(e1);
                    float t = 0;
                    (void)hipEventElapsedTime(&t, e0, e1);
                    ms = t < ms ? t : ms;
                }
                if (ms < best_ms) {
                    best_ms = ms;
                    best = sc;
                }
            }
    c->timing = saved_timing;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(c->stream);
    (void)hipFree(in);
    (void)hipFree(out);
    (void)hipFree(U);
    (void)hipGetLastError();
    return best;
}

}  // namespace

void tune_cache_load(dd_ctx* c) {
    const char* path = std::getenv("DD_TUNE_CACHE");
    if (path == nullptr || *path == 0) return;
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        // key nt tc remap [kc [blocked]]
        std::istringstream in(line);
        std::string key;
        StencilSched sc;
        if (!(in >> key >> sc.nt >> sc.tc >> sc.remap)) continue;
        if (!(in >> sc.kc)) sc.kc = 1;
        if (!(in >> sc.blocked)) sc.blocked = 0;
        c->sched[key] = sc;
    }
}

void tune_cache_store(dd_ctx* c, const std::string& key, const StencilSched& sc) {
    c->sched[key] = sc;
    const char* path = std::getenv("DD_TUNE_CACHE");
    if (path == nullptr || *path == 0) return;
    std::ofstream f(path, std::ios::app);
    f << key << " " << sc.nt << " " << sc.tc << " " << sc.remap << " " << sc.kc << " " << sc.blocked << "\n";
}

StencilSched stencil_sched(dd_ctx* c, const Geo& g, int kind, int ncol) {
    const std::string k = key_of(g, kind, ncol);
    auto it = c->sched.find(k);
    if (it != c->sched.end()) return it->second;
    StencilSched sc = default_sched(g);
    if (c->autotune && (size_t)g.nsite * ncol >= ((size_t)1 << 18))
        sc = kind == 0 ? tune<double>(c, g, ncol) : tune<float>(c, g, ncol);
    tune_cache_store(c, k, sc);
    return sc;
}

int stencil_slots(dd_ctx* c, const Geo& g, int kind, int ncol) {
    return stencil_blocks(g, stencil_sched(c, g, kind, ncol));
}

}  // namespace dd
