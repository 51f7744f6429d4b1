// batched.hip -- solves of many independent domains (each its own lattice,
// links, kappa and sources).
#include <algorithm>
#include <chrono>

#include "dd_internal.h"

using namespace dd;

extern "C" dd_status dd_block_solve_batched(dd_ctx* c, int n, const dd_batch_item* items,
                                            const dd_solver_params* p, dd_solve_stats* stats) {
    if (c == nullptr) return DD_ERR_ARG;
    if (n < 1 || items == nullptr || p == nullptr) return fail(c, DD_ERR_ARG, "need n >= 1 items and params");
    dd_status worst = DD_OK;
    for (int i = 0; i < n; i++) {
        const dd_batch_item& it = items[i];
        if (it.lat.T < 2 || it.lat.L < 2 || it.nrhs < 1 || it.nrhs > DD_MAX_RHS || !(it.kappa > 0) ||
            it.U == nullptr || it.b == nullptr || it.x == nullptr)
            return fail(c, DD_ERR_ARG, "invalid batch item " + std::to_string(i));
        const Geo g = make_geo(it.lat, nullptr);
        dd_status e = solve(c, (const cpx<double>*)it.U, it.kappa, g, it.nrhs, (const cpx<double>*)it.b,
                            (cpx<double>*)it.x, *p, stats ? &stats[i] : nullptr, 0);
        if (e != DD_OK && e != DD_ERR_NOCONV) return e;
        if (e != DD_OK) worst = e;
    }
    return worst;
}
