// dd_internal.h -- shared definitions of the HIP library (kernels, solvers, ABI).
// gfx950 only: 64-lane wavefronts, 256 compute units in 8 XCDs.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <map>
#include <string>
#include <vector>

#include "dd.h"

namespace dd {

constexpr int kBlock = 256;   // threads per workgroup for site-parallel kernels
constexpr int kElems = 8;     // elements per thread of the solver vector kernels

// Minimum resident waves per SIMD asked of the stencil kernels (bounds their
// register use): [0] FP64, [1] FP32, for the time-sweep and the half-hop kernels.
#ifndef DD_SWEEP_WAVES64
#define DD_SWEEP_WAVES64 1
#endif
#ifndef DD_SWEEP_WAVES32
#define DD_SWEEP_WAVES32 1
#endif
#ifndef DD_EO_WAVES64
#define DD_EO_WAVES64 1
#endif
#ifndef DD_EO_WAVES32
#define DD_EO_WAVES32 1
#endif
template <typename R>
constexpr int sweep_waves() { return sizeof(R) == 8 ? DD_SWEEP_WAVES64 : DD_SWEEP_WAVES32; }
template <typename R>
constexpr int eo_waves() { return sizeof(R) == 8 ? DD_EO_WAVES64 : DD_EO_WAVES32; }
constexpr int kWave = 64;     // CDNA wavefront
constexpr int kNumXcd = 8;    // MI355X: workgroups are dealt round-robin over 8 XCDs

// Complex number with interleaved (re, im); 16-byte aligned for FP64 so that a
// component load is one dwordx4, 8-byte aligned (dwordx2) for FP32.
template <typename R>
struct alignas(2 * sizeof(R)) cpx {
    R re, im;
};

template <typename R>
__host__ __device__ inline cpx<R> mk(R a, R b) { return cpx<R>{a, b}; }
template <typename R>
__device__ inline cpx<R> operator+(cpx<R> a, cpx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <typename R>
__device__ inline cpx<R> operator-(cpx<R> a, cpx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <typename R>
__device__ inline cpx<R> operator-(cpx<R> a) { return {-a.re, -a.im}; }
template <typename R>
__device__ inline cpx<R> operator*(cpx<R> a, cpx<R> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename R>
__device__ inline cpx<R> operator*(R s, cpx<R> a) { return {s * a.re, s * a.im}; }
// conj(a) * b
template <typename R>
__device__ inline cpx<R> cmulc(cpx<R> a, cpx<R> b) {
    return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
// i * a
template <typename R>
__device__ inline cpx<R> imul(cpx<R> a) { return {-a.im, a.re}; }

// Geometry of one field: a time slab [t0, t0+nt) of a T x L^3 lattice, or the
// whole lattice (whole = 1, t0 = 0, nt = T).  Field sites are local, links global.
struct Geo {
    int L, L2, L3;   // L, L^2, L^3
    int T;           // lattice time extent (link array covers T*L3 sites)
    int t0, nt;      // slab
    int nsite;       // nt * L3
    int whole;       // 1: hops across the slab's time ends wrap (whole lattice)
    int bc;          // time-edge factor for wrapping hops: -1, 0 (dropped), +1
    int vlink;       // T * L3
};

// XCD-aware workgroup index: the hardware deals consecutive workgroup ids to
// the 8 XCDs round-robin; remap so that each XCD (own L2) walks a contiguous
// range of logical blocks, keeping stencil neighbours and shared links in one L2.
__device__ inline int xcd_remap(int bid, int nblk) {
    const int q = nblk / kNumXcd, r = nblk % kNumXcd;
    const int xcd = bid % kNumXcd, loc = bid / kNumXcd;
    return (xcd < r) ? xcd * (q + 1) + loc : r * (q + 1) + (xcd - r) * q + loc;
}

// ------------------------------------------------------------------ solver scalars
// Per-column scalars of the Krylov iterations, kept on the device so that the
// iteration runs without host round trips.
struct ColState {
    double rho_re, rho_im;      // <r^, r>
    double alpha_re, alpha_im;
    double omega_re, omega_im;
    double beta_re, beta_im;
    double rr;                  // |r|^2 (recursive)
    double bb;                  // |b|^2 of the current system
    double stop2;               // stop when rr <= stop2
    double zz;                  // CGNR: |D^+ r|^2
    double rh2;                 // |r^|^2 of the shadow residual
    int active;                 // 1 while iterating
    int iters;                  // iterations done by this column
    int breakdown;              // 1: stalled (rho, <r^,v> or omega vanished), 2: non-finite
    int xdue;                   // CGNR: alpha p of the current iteration still to be added to x
};

// ------------------------------------------------------------------ context
struct Buffer {
    void* ptr = nullptr;
    size_t bytes = 0;
};

// Launch shape of the time-sweep stencil: workgroup size (spatial sites),
// time-chunk length and whether workgroups are remapped to XCD-contiguous ranges.
struct StencilSched {
    int nt = 128;
    int tc = 8;
    int remap = 0;
    int kc = 1;       // columns per thread
    int blocked = 0;  // tile flags: bit 0 tiles as (y, z) bricks of x rows (even-odd: 4 x 4),
                      // bit 1 the time chunks of a tile in adjacent workgroups, bit 2 non-temporal
                      // output stores (half hop, two columns per thread) or, for the full stencil,
                      // x hops loaded rather than taken from neighbouring lanes; bit 3 the half
                      // hop's LDS-tile form
};

struct TimedLaunch {
    hipEvent_t start, stop;
    int entry;  // index into dd_ctx::timing_entries
    double bytes;
};

// Accumulated HIP-event time of one kernel instance.
struct TimingEntry {
    std::string name;  // the instance as a profiler names it, e.g. "k_dslash<float, 1, 4, 128>"
    double ms = 0;
    long long launches = 0;
    double bytes = 0;
};

}  // namespace dd

struct dd_ctx {
    dd_lattice lat;
    hipStream_t stream;
    int device;
    std::string err;
    std::vector<dd::Buffer> ws;  // workspace slots, grown on demand
    // kernel timing
    int timing = 0;
    std::vector<dd::TimedLaunch> pending;
    std::vector<hipEvent_t> event_pool;
    std::vector<dd::TimingEntry> timing_entries;
    // autotuned stencil launch shapes, keyed by (precision, ncol, geometry)
    std::map<std::string, dd::StencilSched> sched;
    int autotune = 1;
    // library-owned stream for work captured into HIP graphs (created on first use)
    hipStream_t own_stream = nullptr;
    // pinned host mirrors of per-column state and of small reductions
    dd::ColState* host_state = nullptr;
    double* host_dots = nullptr;
    int host_n = 0;
    // fraction of a launch's columns whose spinor bytes the kernel timing bills: solvers set
    // it to the share of columns active when they launch (a stopped column's workgroups
    // return at once); 1 outside solves
    double bill_frac = 1.0;
};

namespace dd {

// Workspace slots (each is one lazily grown device allocation).
enum Slot {
    W_R = 0, W_RH, W_P, W_V, W_S, W_T,          // Krylov vectors, FP64
    W_R32, W_RH32, W_P32, W_V32, W_S32, W_T32,  // Krylov vectors, FP32
    W_B32, W_X32, W_U32, W_RES64,
    W_PART, W_STATE, W_STATE32, W_DOTS,
    W_AUX0, W_AUX1, W_AUX2, W_AUX3, W_AUX4,
    W_SEGS, W_SEGN, W_EO_B, W_EO_X, W_EO_BHAT, W_EO_T64, W_EO_T32, W_EO_U64, W_BATCH0, W_BATCH1, W_BATCH2, W_BATCH3, W_BATCH4,
    W_U32C, W_LDEV, W_PROJ_V, W_PROJ_G, W_PROJ_R, W_DISC0, W_DISC1, W_DISC2, W_DISC3,
    W_NSLOTS
};

dd_status fail(dd_ctx* c, dd_status st, const std::string& msg);
dd_status hip_fail(dd_ctx* c, hipError_t e, const char* what);
void* workspace(dd_ctx* c, Slot s, size_t bytes, dd_status* st);

#define DD_HIP(ctx, call)                                         \
    do {                                                          \
        hipError_t e_ = (call);                                   \
        if (e_ != hipSuccess) return ::dd::hip_fail(ctx, e_, #call); \
    } while (0)

Geo make_geo(const dd_lattice& lat, const dd_domain* dom);
// p is device memory of the context's device, aligned, with bytes available
bool on_device(dd_ctx* c, const void* p, size_t bytes, size_t align);
// allow_guess: the entry point honours dd_solver_params::x0 (dd_block_solve only)
dd_status check_params(dd_ctx* c, const dd_solver_params* p, bool allow_guess = false);

// ---------------------------------------------------------------- stencil launchers
// Epilogues fused into the stencil (one pass over the output):
enum Epi {
    EPI_STORE = 0,   // out = M in
    EPI_DOT_AUX,     // out = M in; partial <aux, out>
    EPI_TS,          // out = M in; partials <out, in>, |out|^2
    EPI_RESID,       // out = aux - M in; partial |out|^2
    EPI_NORM,        // out = M in; partial |out|^2
    EPI_HOP          // out = kappa D_hop in = in - 2 kappa D in (no mass term, no partials; dag = 0)
};

// M = D (dag = 0) or D^+ = gamma5 D gamma5 (dag = 1) on the field geometry g.
// partial: [ncol][nsb][3] doubles (nsb = site blocks); active: nullable per-column mask.
template <typename R>
void launch_dslash(dd_ctx* c, const Geo& g, const cpx<R>* U, double kappa, int dag, int epi,
                   const cpx<R>* in, cpx<R>* out, const cpx<R>* aux, int ncol,
                   double* partial, const ColState* state);

// Number of partial-sum slots per column written by one stencil launch.
StencilSched stencil_sched(dd_ctx* c, const Geo& g, int kind, int ncol);
int stencil_slots(dd_ctx* c, const Geo& g, int kind, int ncol);
// Tuned shapes shared across processes through the file named by DD_TUNE_CACHE.
void tune_cache_load(dd_ctx* c);
void tune_cache_store(dd_ctx* c, const std::string& key, const StencilSched& sc);
StencilSched default_sched(const Geo& g);
int stencil_blocks(const Geo& g, const StencilSched& sc);
int sched_kc(const StencilSched& sc, int ncol, size_t real_bytes, size_t col_bytes);
int brick_rows(const Geo& g, int nt);
template <typename R>
void launch_dslash_sched(dd_ctx* c, const Geo& g, const StencilSched& sc, const cpx<R>* U, double kappa,
                         int dag, int epi, const cpx<R>* in, cpx<R>* out, const cpx<R>* aux, int ncol,
                         double* partial, const ColState* st);
inline int site_blocks(int nsite) { return (nsite + kBlock - 1) / kBlock; }

// ---------------------------------------------------------------- solver segments
// A solve advances many columns ("segments") together: the columns of one
// lattice or slab, or every column of every domain of a batch.  Segments lie
// back to back in each work vector and may differ in length.  Device tables:
struct Segs {
    const long long* off;  // [nseg] first element (complex) of each segment
    const int* len;        // [nseg] elements of each segment (12 x sites)
    const int* eb0;        // [nseg + 1] first elementwise workgroup of each segment
    const int* eseg;       // [neb] segment of each elementwise workgroup
    int nseg, neb;
    int paired;            // FP32 vectors are even-odd half fields with paired components (dd_eo.h)
};

// Vector kernels of the Krylov solvers over segments; reductions write one
// partial slot per elementwise workgroup (slots of segment k: [eb0[k], eb0[k+1])).
template <typename R>
void launch_bicg_p(dd_ctx* c, const Segs& S, const cpx<R>* r, cpx<R>* p, const cpx<R>* v, const ColState* st);
template <typename R>
void launch_bicg_s(dd_ctx* c, const Segs& S, const cpx<R>* r, const cpx<R>* v, cpx<R>* s, const ColState* st);
template <typename R>
void launch_bicg_xr(dd_ctx* c, const Segs& S, cpx<R>* x, cpx<R>* r, const cpx<R>* p, const cpx<R>* s,
                    const cpx<R>* t, const cpx<R>* rh, double* partial, const ColState* st);
template <typename R>
void launch_cg_r(dd_ctx* c, const Segs& S, cpx<R>* r, const cpx<R>* w, double* partial, const ColState* st);
template <typename R>
void launch_cg_px(dd_ctx* c, const Segs& S, cpx<R>* x, cpx<R>* p, const cpx<R>* z, const ColState* st);
template <typename R>
void launch_norm2(dd_ctx* c, const Segs& S, const cpx<R>* a, double* partial);
template <typename R>
void launch_copy_segs(dd_ctx* c, const Segs& S, const cpx<R>* a, cpx<R>* b, const ColState* st);
template <typename R>
void launch_fold_x(dd_ctx* c, const Segs& S, cpx<double>* x, cpx<R>* xk, const int* mask);
template <typename R>
void launch_set_resid(dd_ctx* c, const Segs& S, const cpx<double>* r64, cpx<R>* rk, const int* mask);
template <typename R>
void launch_restart_dirs(dd_ctx* c, const Segs& S, const cpx<R>* r, cpx<R>* rh, cpx<R>* p, cpx<R>* v,
                         const int* mask);
template <typename R>
void launch_cg_shift(dd_ctx* c, const Segs& S, cpx<R>* p, cpx<R>* z, const cpx<R>* t, const int* mask);
// a = 0 on the segments with mask[seg] != 0
void launch_zero_segs(dd_ctx* c, const Segs& S, cpx<double>* a, const int* mask);

// finalize kinds (one workgroup per segment reduces its partial slots, then
// updates that segment's scalars)
enum Fin {
    FIN_ALPHA = 0,   // dots = <r^,v>        -> alpha = rho / <r^,v>
    FIN_OMEGA,       // dots = <t,s>, |t|^2  -> omega
    FIN_RHO,         // dots = <r^,r>, |r|^2 -> beta, rho, rr, convergence
    FIN_CG_ALPHA,    // dots = |w|^2         -> alpha = zz / |w|^2
    FIN_CG_RR,       // dots = |r|^2         -> rr, convergence
    FIN_CG_BETA,     // dots = |z|^2         -> beta = zz_new / zz
    FIN_CG_ZZ,       // dots = |z|^2         -> zz
    FIN_STORE        // dots -> out[seg*3 + k] (plain reduction)
};
// p0: device [nseg + 1] prefix of the partial slots of each segment.
void launch_finalize(dd_ctx* c, int fin, int nseg, const int* p0, const double* partial, ColState* st,
                     double* out);

// The operator side of a solve: nseg independent systems M_k x_k = b_k.
// apply runs the stencil of every segment in precision R with a fused
// epilogue (dag = 1: D^+); the partial slots of segment k written by such a
// launch are [sp0[kind][k], sp0[kind][k+1]) with kind 0 = FP64, 1 = FP32.
struct System {
    dd_ctx* c = nullptr;
    int nseg = 0;
    size_t nelem = 0;                      // complex elements of one work vector
    Segs seg{};                            // elementwise segment tables
    const int* sp0[2] = {nullptr, nullptr};
    size_t nslots = 0;                     // partial slots needed by any launch
    bool graph = false;                    // replay the inner iterations from a captured HIP graph
    bool has32 = false;                    // FP32 stencil available (links converted)
    bool pair32 = false;                   // FP32 vectors are half fields with paired components
    const double* ref_norm2 = nullptr;     // host [nseg]: |.|^2 that residuals are relative to (default |b|^2)
    virtual ~System() {}
    virtual void apply64(int dag, int epi, const cpx<double>* in, cpx<double>* out, const cpx<double>* aux,
                         double* partial, const ColState* st) = 0;
    virtual void apply32(int dag, int epi, const cpx<float>* in, cpx<float>* out, const cpx<float>* aux,
                         double* partial, const ColState* st) = 0;
    void apply(int dag, int epi, const cpx<double>* in, cpx<double>* out, const cpx<double>* aux,
               double* partial, const ColState* st) {
        apply64(dag, epi, in, out, aux, partial, st);
    }
    void apply(int dag, int epi, const cpx<float>* in, cpx<float>* out, const cpx<float>* aux, double* partial,
               const ColState* st) {
        apply32(dag, epi, in, out, aux, partial, st);
    }
};

// Host and device copies of a segment layout.  upload() places the device
// tables in workspace slot `slot` and waits for the copy.
struct SegLayout {
    std::vector<long long> off;
    std::vector<int> len;
    std::vector<int> sp0[2];  // stencil partial prefixes per kind, filled by the caller
    std::vector<int> eb0, eseg;
    dd_status upload(dd_ctx* c, Slot slot, System* S);
};

// Outcome of solve_system per segment and overall.
struct SolveResult {
    int iters = 0;                  // lockstep iterations
    int updates = 0;                // rounds of reliable updates
    int restarts = 0;
    std::vector<double> rel;        // true |b - M x| / |b| per segment
    std::vector<int> seg_iters;     // iterations each segment was active
};

// Solve every segment of S to p.tol (true FP64 residual); b and x are work
// vectors laid out as S.seg.  Returns DD_ERR_NOCONV / DD_ERR_BREAKDOWN with the
// result filled.
dd_status solve_system(System& S, const cpx<double>* b, cpx<double>* x, const dd_solver_params& p,
                       SolveResult* res);

// Even-odd preconditioned solve of one lattice or slab (evenodd.hip); usable
// when the lattice is bipartite: L even, and nt even for a whole lattice.
bool eo_applicable(const Geo& g);
// FP32 checkerboard links of field g as two rows each (Ueo12[mu][k < 6][parity][nsite / 2]);
// *su3 tells whether every link's third row is the conjugated cross product of
// the first two within 1e-6 (so that the two rows determine the link to FP32
// precision).
dd_status links_eo12(dd_ctx* c, const Geo& g, const cpx<double>* U, cpx<float>* Ueo12, bool* su3);
// checkerboard-ordered links of the field g (Ueo[mu][k][parity][nsite/2]) from U[mu][k][V]
template <typename R>
void launch_links_eo(dd_ctx* c, const Geo& g, const cpx<double>* U, cpx<R>* Ueo);
// full field [ncol][12][nsite] <-> even / odd half fields [ncol][12][nsite/2]
void launch_eo_split(dd_ctx* c, const Geo& g, int ncol, const cpx<double>* full, cpx<double>* ev, cpx<double>* od);
void launch_eo_merge(dd_ctx* c, const Geo& g, int ncol, const cpx<double>* ev, const cpx<double>* od,
                     cpx<double>* full);
// out = a_self * self + c_hop * H_{p_out, 1 - p_out} in (FP64, no epilogue); self may be NULL
void launch_eo_hop64(dd_ctx* c, const Geo& g, const cpx<double>* Ueo, double a_self, double c_hop, int p_out, int dag,
                     const cpx<double>* in, const cpx<double>* self, cpx<double>* out, int ncol);
dd_status solve_eo(dd_ctx* c, const cpx<double>* U, double kappa, const Geo& g, int ncol, const cpx<double>* b,
                   cpx<double>* x, const dd_solver_params& p, dd_solve_stats* stats, int dag);

// |a_k|^2 of the segments [off[k], off[k] + len[k]) of a, into out; synchronises.
dd_status segment_norms(dd_ctx* c, const std::vector<long long>& off, const std::vector<int>& len,
                        const cpx<double>* a, std::vector<double>* out);
// |a_j|^2 of the ncol columns of a (each n elements), into out; synchronises.
dd_status column_norms(dd_ctx* c, int n, int ncol, const cpx<double>* a, std::vector<double>* out);

void launch_links_to_f32(dd_ctx* c, size_t n, const cpx<double>* src, cpx<float>* dst);
template <typename R>
void launch_gamma5(dd_ctx* c, int n, int ncol, const cpx<R>* in, cpx<R>* out);
template <typename R>
void launch_zero(dd_ctx* c, size_t n, cpx<R>* a);
// b = s a over n complex128 elements (b may be a)
void launch_scale(dd_ctx* c, size_t n, double s, const cpx<double>* a, cpx<double>* b);

// frontier: out(dst) += alpha * P_dst D P_src in(src), time hops across the frontier
void launch_frontier(dd_ctx* c, const dd_lattice& lat, const cpx<double>* U, const dd_domain& dst,
                     const dd_domain& src, int ncol, const cpx<double>* in, cpx<double>* out,
                     double alpha);
// copy a compact slab field into / out of a whole-lattice field
void launch_slab_scatter(dd_ctx* c, const dd_lattice& lat, const dd_domain& dom, int ncol,
                         const cpx<double>* part, cpx<double>* whole);
void launch_slab_gather(dd_ctx* c, const dd_lattice& lat, const dd_domain& dom, int ncol,
                        const cpx<double>* whole, cpx<double>* part);
// compact slab field (nt slices) <-> the slices [off, off + nt) of a compact slab
// field of nt_big slices; dir 0: part -> big, 1: big -> part
void launch_slab_embed(dd_ctx* c, int L3, int nt_big, int off, int nt, int ncol, cpx<double>* part,
                       cpx<double>* big, int dir);
void launch_point_source(dd_ctx* c, int nsite, int site, cpx<double>* eta);
// pion correlator: per-slice partial sums then fixed-order reduction
void launch_pion(dd_ctx* c, const dd_lattice& lat, int ncol, const cpx<double>* S, int t_src,
                 double* partial, double* C);
// link force: grad_U += coeff * g(X, Y) on the slab geometry
void launch_link_force(dd_ctx* c, const Geo& g, int ncol, const cpx<double>* X,
                       const cpx<double>* Y, double coeff, cpx<double>* grad);

// ---------------------------------------------------------------- timing
void timing_begin(dd_ctx* c, hipEvent_t* ev);
void timing_end(dd_ctx* c, hipEvent_t ev, const std::string& name, double bytes);
void timing_harvest(dd_ctx* c);

// ---------------------------------------------------------------- solver
dd_status solve(dd_ctx* c, const cpx<double>* U, double kappa, const Geo& g, int ncol,
                const cpx<double>* b, cpx<double>* x, const dd_solver_params& p,
                dd_solve_stats* stats, int dag);

// ---------------------------------------------------------------- quark-line projection
constexpr int kMaxProjVec = 256;  // vectors per projection basis
// phi ([nvec][12][L^3]) = orthonormal basis for the quark line leaving slice k of
// the slab g forward (sign +1) or backward (-1), by n_iter inverse iterations
// from v0 ([nvec][12][g.nsite])
dd_status projection_basis(dd_ctx* c, const cpx<double>* U, double kappa, const Geo& g, int k, int sign, int nvec,
                           int n_iter, const cpx<double>* v0, cpx<double>* phi, const dd_solver_params& p,
                           dd_solve_stats* stats);
// slice k of field ([ncol][12][nt L^3]) <- sum_i phi_i phi_i^+ (that slice)
dd_status project_slice(dd_ctx* c, int L3, int nt, int k, int ncol, cpx<double>* field, int nvec,
                        const cpx<double>* phi);

// ---------------------------------------------------------------- disconnected contraction
// tau ([nsrc][T], device) = per-source, per-slice estimates of tr{gamma5 D_Lambda^-1} with
// n_hop powers of kappa D_hop, over the slabs doms (NULL: the whole lattice); eta
// [nsrc][12][V].  stats: NULL or one entry per domain.  Synchronises.
dd_status disconnected_traces(dd_ctx* c, const cpx<double>* U, double kappa, const dd_domain* doms, int ndom,
                              int nsrc, const cpx<double>* eta, int n_hop, const dd_solver_params& p,
                              cpx<double>* tau, dd_solve_stats* stats);
// C_host[y0][x0] (complex, T x T) = the two-trace product over distinct sources
dd_status disconnected_correlator(dd_ctx* c, int nsrc, const cpx<double>* tau, double* C_host);

// ---------------------------------------------------------------- nucleon contraction
// xi ([nvec][12][L^3], slice x0 of gbar) and eta ([nvec][12][|gstar|]) of the lines cut by phi
// on slice t_phi; stats: NULL or 2 entries (the gbar and the gstar solves).  Synchronises.
dd_status nucleon_lines(dd_ctx* c, const cpx<double>* U, double kappa, const dd_domain& gbar, const dd_domain& gstar,
                        int t_phi, int nvec, const cpx<double>* phi, int x0, cpx<double>* xi, cpx<double>* eta,
                        const dd_solver_params& p, dd_solve_stats* stats);
// B[t][k][alpha][i][j] of the n fields s ([n][12][nt L^3]), summed per time slice
dd_status baryon_blocks(dd_ctx* c, int n, int nt, const cpx<double>* s, cpx<double>* B);
// W_host[w][y][x] (complex) = W1 (w = 0), W2 (w = 1) of the blocks Bx (ntx slices), By (nty)
dd_status nucleon_contract(dd_ctx* c, int n, int ntx, const cpx<double>* Bx, int nty, const cpx<double>* By,
                           double* W_host);

}  // namespace dd
