// nucleon.hip -- the factorised nucleon contraction with projected quark lines
// (Sec. 4.2, Eqs. 22-26).
//
// Each quark line from x in Gbar to y in Gstar is cut by the projector on N_m
// vectors phi_i living on the slice t_phi just outside Gstar:
//   D^-1(y, x) -> - sum_i eta_i(y) xi_i^T(x),
//   xi_i^T(x) = [phi_i^+ D_Gbar^-1](x)  = conj([D_Gbar^-1+ phi_i](x)),
//   eta_i(y)  = [D_Gstar^-1 D_{Gstar,dGstar} phi_i](y),
// so the Wick contractions factorise into colourless spinors (Eq. 25)
//   B[s_i, s_j, s_k](x)_alpha = eps^{abc} (s_i^{aT} C gamma5 s_j^b)(x) s_k^c_alpha(x),
// summed over each time slice, one set built from three xi's at the source and
// one from three eta's at every sink slice, contracted through the spin matrix
// P_+ = (1 + gamma_0)/2 (Eqs. 23-24, whose gamma5 P_- belongs to conventions the
// text does not print: with this operator, (1 - gamma_mu) on the forward hop,
// and xi^T = phi^+ D^-1 without gamma5, a forward-propagating quark carries
// (1 + gamma_0)/2 and B_x^T gamma5 P_-+ B_y vanishes at leading order).
//
// Blocks per slice are a dense contraction over the sites x and colours c:
//   B[(k, alpha)][(i, j)] = sum_{x, c} E_c[(i, j)](x) s_k^c_alpha(x),
//   E_c = eps^{abc} sum_{beta, gamma} s_i^a_beta (C gamma5)_{beta gamma} s_j^b_gamma,
// a (P x 3 X) by (3 X x 4 N_m) matrix product per chunk of X sites, over the
// P = N_m (N_m + 1) / 2 pairs i <= j only: B is symmetric in (i, j) (C gamma5 and
// eps are both antisymmetric).  The diquarks E (HBM-bound) and the packed quark
// matrix are written per chunk; the product is a complex FP64 GEMM on the matrix
// cores (k_zgemm_mfma: 64 x 64 tiles of four 16 x 16 x 4 FP64 MFMA blocks per
// wavefront, operands staged through LDS, the k range split so that the grid
// fills the chip, the splits added in a fixed order by k_zgemm_reduce)
// accumulating into the slice's packed blocks, and a last kernel writes both
// (i, j) and (j, i).  About N_m / 2 flops per byte of E, so the product, not the
// diquarks, bounds the time.
//
// Basis: chiral, component = spin * 3 + colour; gamma_0 = [[0, -1], [-1, 0]]
// (2 x 2 blocks), gamma5 = diag(1, 1, -1, -1), C = gamma_0 gamma_2 (C gamma_mu
// C^-1 = -gamma_mu^T), so C gamma5 has (0,1) = -1, (1,0) = +1, (2,3) = -1,
// (3,2) = +1 and P_+ = (1 + gamma_0)/2 = 1/2 [[1, -1], [-1, 1]].
#include <algorithm>
#include <chrono>
#include <cstdlib>
#include <cstring>

#include "dd_internal.h"
#include "dd_wilson.h"

namespace dd {

namespace {

constexpr int kNB = 256;
constexpr int kXT = 1;                   // sites per workgroup of the diquark kernel (LDS: 49 KB at 256 vectors)
constexpr int kMaxN = kMaxProjVec;       // vectors per set of lines
constexpr int kCChunk = 1 << 16;         // flat block entries per contraction workgroup

__device__ inline cpx<double> cj(cpx<double> a) { return {a.re, -a.im}; }

// xi[col][c][s] = conj(w[col][c][slice kx, s])
__global__ __launch_bounds__(kNB) void k_conj_slice(int L3, int nsite, int kx, const cpx<double>* __restrict__ w,
                                                    cpx<double>* __restrict__ xi) {
    const int s = blockIdx.x * kNB + threadIdx.x;
    const int cc = blockIdx.y;  // col * 12 + component
    if (s >= L3) return;
    xi[(size_t)cc * L3 + s] = cj(w[(size_t)cc * nsite + (size_t)kx * L3 + s]);
}

// Sp (column-major, 3X x 4n): row c X + x, column q = 4 k + alpha  <-  s_k^{alpha, c}(off + x)
__global__ __launch_bounds__(kNB) void k_pack_quarks(int n, long long nsite, long long off, int X,
                                                     const cpx<double>* __restrict__ s, cpx<double>* __restrict__ Sp) {
    const int x = blockIdx.x * kNB + threadIdx.x;
    const int qc = blockIdx.y;  // q * 3 + c
    if (x >= X) return;
    const int q = qc / 3, c = qc % 3;
    const int k = q >> 2, al = q & 3;
    Sp[(size_t)q * 3 * X + (size_t)c * X + x] = s[((size_t)k * 12 + al * 3 + c) * nsite + off + x];
}

// row p of the packed pairs i <= j, p = i n - i (i - 1) / 2 + (j - i)
__device__ inline long long pair_start(int i, int n) { return (long long)i * n - (long long)i * (i - 1) / 2; }
__device__ inline void pair_of(long long p, int n, int& i, int& j) {
    const double d = 2.0 * n + 1.0;
    int a = (int)((d - sqrt(d * d - 8.0 * (double)p)) * 0.5);
    a = max(0, min(a, n - 1));
    while (a > 0 && pair_start(a, n) > p) a--;
    while (a < n - 1 && pair_start(a + 1, n) <= p) a++;
    i = a;
    j = a + (int)(p - pair_start(a, n));
}

// diquark of the colour pair (a, b): sum_{beta, gamma} s_i^a_beta (C gamma5)_{beta gamma} s_j^b_gamma
__device__ inline cpx<double> diquark(const cpx<double>* si, const cpx<double>* sj, int a, int b) {
    // (C gamma5): (0,1) = -1, (1,0) = +1, (2,3) = -1, (3,2) = +1
    return si[3 + a] * sj[b] - si[a] * sj[3 + b] + si[9 + a] * sj[6 + b] - si[6 + a] * sj[9 + b];
}

// E (column-major, P x 3X): row p(i, j), column c X + x  <-  eps^{abc} diquark(a, b) at site off + x
__global__ __launch_bounds__(kNB) void k_diquarks(int n, long long nsite, long long off, int X,
                                                  const cpx<double>* __restrict__ s, cpx<double>* __restrict__ E) {
    __shared__ cpx<double> sq[kXT][kMaxN][12];
    const int x0 = blockIdx.x * kXT;
    for (int e = threadIdx.x; e < kXT * n * 12; e += kNB) {
        const int xt = e % kXT, rest = e / kXT;
        const int comp = rest % 12, k = rest / 12;
        const int x = x0 + xt;
        sq[xt][k][comp] = x < X ? s[((size_t)k * 12 + comp) * nsite + off + x] : cpx<double>{0.0, 0.0};
    }
    __syncthreads();
    const size_t M = (size_t)n * (n + 1) / 2;
    for (int r = threadIdx.x; r < (int)M; r += kNB) {
        int i, j;
        pair_of(r, n, i, j);
#pragma unroll
        for (int xt = 0; xt < kXT; xt++) {
            const int x = x0 + xt;
            if (x >= X) break;
            const cpx<double>* si = sq[xt][i];
            const cpx<double>* sj = sq[xt][j];
            // eps^{abc}: c = 0 from (1, 2), c = 1 from (2, 0), c = 2 from (0, 1), minus the swapped pair
            E[r + (size_t)(0 * X + x) * M] = diquark(si, sj, 1, 2) - diquark(si, sj, 2, 1);
            E[r + (size_t)(1 * X + x) * M] = diquark(si, sj, 2, 0) - diquark(si, sj, 0, 2);
            E[r + (size_t)(2 * X + x) * M] = diquark(si, sj, 0, 1) - diquark(si, sj, 1, 0);
        }
    }
}

// ------------------------------------------------------------------ complex FP64 GEMM
// C (M x N) = A (M x K) B (K x N), all column-major complex FP64 (lda = M, ldb = K,
// ldc = M), on the matrix cores.  v_mfma_f64_16x16x4f64 multiplies a 16 x 4 block
// (lane l holds A[l % 16][l / 16]) by a 4 x 16 block (lane l holds B[l / 16][l % 16])
// into a 16 x 16 accumulator (lane l holds rows l / 16 + 4 e, e = 0..3, of column l % 16).
// A complex product is four real ones: re += ar br + ai (-bi), im += ar bi + ai br.
// A workgroup (four wavefronts, 2 x 2) owns a 64 x 64 tile of C and one of nsplit
// ranges of k (kps steps of 16); per step the 64 x 16 panel of A and the 16 x 64
// panel of B go through LDS (the next step's panels are loaded into registers while
// the current one is multiplied), and each wavefront runs 16 MFMAs per 4 values of
// k on its 32 x 32 quarter (132 registers: three wavefronts per SIMD; a form holding
// the step's operands up front took 212 and ran 16 % slower).  Each split writes its own partial C; k_zgemm_reduce
// adds them in a fixed order, so the result does not depend on scheduling.
typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef double dbl2 __attribute__((ext_vector_type(2)));
constexpr int kGM = 64, kGN = 64, kGK = 16;  // workgroup tile (complex entries) and k step
constexpr int kGThreads = 256;

__device__ __forceinline__ dbl2 gload2(rsrc_t r, uint32_t voff) {
    return __builtin_bit_cast(dbl2, __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, 0, 0));
}

__global__ __launch_bounds__(kGThreads, 2) void k_zgemm_mfma(int M, int N, int K, int kps,
                                                             const cpx<double>* __restrict__ A,
                                                             const cpx<double>* __restrict__ B,
                                                             cpx<double>* __restrict__ Cpart) {
    __shared__ dbl2 As[kGK][kGM + 1];  // As[k][m]; one entry of padding per row
    __shared__ dbl2 Bs[kGK][kGN + 1];  // Bs[k][n]
    const int tm = (M + kGM - 1) / kGM, tn = (N + kGN - 1) / kGN;
    // XCD-contiguous work ranges, the column tiles of one (row tile, split) adjacent: they share the A panel
    const int w = xcd_remap((int)blockIdx.x, (int)gridDim.x);
    const int nt = w % tn, mt = (w / tn) % tm, sp = w / (tn * tm);
    const int m0 = mt * kGM, n0 = nt * kGN;
    const int nkt = (K + kGK - 1) / kGK;
    const int kt0 = sp * kps, kt1 = min(nkt, kt0 + kps);
    const rsrc_t ra = make_rsrc(A, (uint32_t)((size_t)M * K * sizeof(cpx<double>)));
    const rsrc_t rb = make_rsrc(B, (uint32_t)((size_t)K * N * sizeof(cpx<double>)));

    const int tid = (int)threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int wm = wv & 1, wn = wv >> 1;
    // global -> LDS roles: A entries (m = tid % 64, k = tid / 64 + 4 r), B entries (k = tid % 16, n = tid / 16 + 16 r)
    const int am = tid & 63, ak = tid >> 6;
    const int bk = tid & 15, bn = tid >> 4;
    dbl2 ga[4], gb[4];
    auto fetch = [&](int kt) {
        const int k0 = kt * kGK;
#pragma unroll
        for (int r = 0; r < 4; r++) {
            const int m = m0 + am, k = k0 + ak + 4 * r;
            const bool ok = m < M && k < K;
            const dbl2 v = gload2(ra, ok ? (uint32_t)(((size_t)k * M + m) * sizeof(cpx<double>)) : 0u);
            ga[r] = ok ? v : dbl2{0.0, 0.0};
        }
#pragma unroll
        for (int r = 0; r < 4; r++) {
            const int k = k0 + bk, n = n0 + bn + 16 * r;
            const bool ok = k < K && n < N;
            const dbl2 v = gload2(rb, ok ? (uint32_t)(((size_t)n * K + k) * sizeof(cpx<double>)) : 0u);
            gb[r] = ok ? v : dbl2{0.0, 0.0};
        }
    };
    auto stash = [&]() {
#pragma unroll
        for (int r = 0; r < 4; r++) As[ak + 4 * r][am] = ga[r];
#pragma unroll
        for (int r = 0; r < 4; r++) Bs[bk][bn + 16 * r] = gb[r];
    };

    dbl4 cr[2][2], ci[2][2];
#pragma unroll
    for (int i = 0; i < 2; i++)
#pragma unroll
        for (int j = 0; j < 2; j++) cr[i][j] = ci[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};

    if (kt0 < kt1) {
        fetch(kt0);
        stash();
        __syncthreads();
    }
    for (int kt = kt0; kt < kt1; kt++) {
        if (kt + 1 < kt1) fetch(kt + 1);  // in flight while this step is multiplied
#pragma unroll
        for (int ks = 0; ks < kGK / 4; ks++) {
            const int kk = 4 * ks + (lane >> 4);
            double ar[2], ai[2], br[2], bi[2], bm[2];
#pragma unroll
            for (int i = 0; i < 2; i++) {
                const dbl2 a = As[kk][wm * 32 + i * 16 + (lane & 15)];
                ar[i] = a.x;
                ai[i] = a.y;
                const dbl2 b = Bs[kk][wn * 32 + i * 16 + (lane & 15)];
                br[i] = b.x;
                bi[i] = b.y;
                bm[i] = -b.y;
            }
            // consecutive MFMAs go to different accumulators
#pragma unroll
            for (int i = 0; i < 2; i++)
#pragma unroll
                for (int j = 0; j < 2; j++) cr[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[i], br[j], cr[i][j], 0, 0, 0);
#pragma unroll
            for (int i = 0; i < 2; i++)
#pragma unroll
                for (int j = 0; j < 2; j++) ci[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[i], bi[j], ci[i][j], 0, 0, 0);
#pragma unroll
            for (int i = 0; i < 2; i++)
#pragma unroll
                for (int j = 0; j < 2; j++) cr[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[i], bm[j], cr[i][j], 0, 0, 0);
#pragma unroll
            for (int i = 0; i < 2; i++)
#pragma unroll
                for (int j = 0; j < 2; j++) ci[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[i], br[j], ci[i][j], 0, 0, 0);
        }
        __syncthreads();  // every wavefront is done with the panels
        if (kt + 1 < kt1) {
            stash();
            __syncthreads();
        }
    }

    // this split's partial C: two 8-byte stores per entry (re, then im through the scalar offset)
    const size_t MN = (size_t)M * N;
    const rsrc_t rc = make_rsrc(Cpart + (size_t)sp * MN, (uint32_t)(MN * sizeof(cpx<double>)));
#pragma unroll
    for (int i = 0; i < 2; i++)
#pragma unroll
        for (int j = 0; j < 2; j++)
#pragma unroll
            for (int e = 0; e < 4; e++) {
                const int row = m0 + wm * 32 + i * 16 + (lane >> 4) + 4 * e;
                const int col = n0 + wn * 32 + j * 16 + (lane & 15);
                if (row < M && col < N) {
                    const uint32_t vo = (uint32_t)(((size_t)col * M + row) * sizeof(cpx<double>));
                    // the elements go through scalars: a bit cast of a vector element expression
                    // compiled to element 0 of the vector here
                    const double re = cr[i][j][e];
                    const double im = ci[i][j][e];
                    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, re), rc, (int)vo, 0, 0);
                    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, im), rc, (int)vo, 8, 0);
                }
            }
}

// C (+)= sum over the splits of Cpart, in split order
__global__ __launch_bounds__(kNB) void k_zgemm_reduce(size_t MN, int nsplit, int acc,
                                                      const cpx<double>* __restrict__ Cpart,
                                                      cpx<double>* __restrict__ C) {
    const size_t f = (size_t)blockIdx.x * kNB + threadIdx.x;
    if (f >= MN) return;
    double re = 0.0, im = 0.0;
    if (acc) {
        re = C[f].re;
        im = C[f].im;
    }
    for (int s = 0; s < nsplit; s++) {
        const cpx<double> v = Cpart[(size_t)s * MN + f];
        re += v.re;
        im += v.im;
    }
    C[f].re = re;
    C[f].im = im;
}

// B[t][k][al][i][j] = Bp[t][(4 k + al) P + p(min(i, j), max(i, j))]
__global__ __launch_bounds__(kNB) void k_unpack_blocks(int n, size_t P, const cpx<double>* __restrict__ Bp,
                                                       cpx<double>* __restrict__ B) {
    const size_t f = (size_t)blockIdx.x * kNB + threadIdx.x;
    const size_t n2 = (size_t)n * n;
    if (f >= 4 * n2 * n) return;
    const int j = (int)(f % n), i = (int)((f / n) % n);
    const size_t q = f / n2;  // 4 k + al
    const int a = min(i, j), b = max(i, j);
    B[f] = Bp[q * P + (size_t)(pair_start(a, n) + (b - a))];
}

// P1[k][al][i][j] = B[k][al][j][i],  P2[k][al][i][j] = B[j][al][k][i]  (one slice, n^3 4 entries)
__global__ __launch_bounds__(kNB) void k_block_perms(int n, const cpx<double>* __restrict__ B,
                                                     cpx<double>* __restrict__ P1, cpx<double>* __restrict__ P2) {
    const size_t f = (size_t)blockIdx.x * kNB + threadIdx.x;
    const size_t n2 = (size_t)n * n, tot = 4 * n2 * n;
    if (f >= tot) return;
    const int j = (int)(f % n), i = (int)((f / n) % n), al = (int)((f / n2) % 4), k = (int)(f / (4 * n2));
    P1[f] = B[(((size_t)k * 4 + al) * n + j) * n + i];
    P2[f] = B[(((size_t)j * 4 + al) * n + k) * n + i];
}

// partial sums over a chunk of the flat index f = ((k 4 + al) n + i) n + j of
//   sum P_x[f] (P_+ By_y)[f]  for W1 (P1) and W2 (P2)
__global__ __launch_bounds__(kNB) void k_nucleon_partial(int n, int nchunk, int ntx, const cpx<double>* __restrict__ By,
                                                         const cpx<double>* __restrict__ P1,
                                                         const cpx<double>* __restrict__ P2,
                                                         double* __restrict__ partial) {
    const int chunk = blockIdx.x, yy = blockIdx.y, xx = blockIdx.z;
    const size_t n2 = (size_t)n * n, sl = 4 * n2 * n;
    const cpx<double>* by = By + (size_t)yy * sl;
    const cpx<double>* p1 = P1 + (size_t)xx * sl;
    const cpx<double>* p2 = P2 + (size_t)xx * sl;
    const size_t f0 = (size_t)chunk * kCChunk, f1 = std::min(sl, f0 + kCChunk);
    double a1r = 0, a1i = 0, a2r = 0, a2i = 0;
    for (size_t f = f0 + threadIdx.x; f < f1; f += kNB) {
        const int al = (int)((f / n2) % 4);
        // (P_+)_{al, be} = +1/2 for be = al, -1/2 for be = al +- 2
        const size_t base = f - (size_t)al * n2;  // the al = 0 entry of this (k, i, j)
        const cpx<double> u = by[base + (size_t)(al & 1) * n2], v = by[base + (size_t)((al & 1) + 2) * n2];
        const double h = al < 2 ? 0.5 : -0.5;
        const cpx<double> m = {h * (u.re - v.re), h * (u.im - v.im)};
        const cpx<double> b1 = p1[f], b2 = p2[f];
        a1r += b1.re * m.re - b1.im * m.im;
        a1i += b1.re * m.im + b1.im * m.re;
        a2r += b2.re * m.re - b2.im * m.im;
        a2i += b2.re * m.im + b2.im * m.re;
    }
    __shared__ double sh[kNB / kWave][4];
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
        a1r += __shfl_xor(a1r, off, kWave);
        a1i += __shfl_xor(a1i, off, kWave);
        a2r += __shfl_xor(a2r, off, kWave);
        a2i += __shfl_xor(a2i, off, kWave);
    }
    const int w = threadIdx.x / kWave, l = threadIdx.x % kWave;
    if (l == 0) {
        sh[w][0] = a1r;
        sh[w][1] = a1i;
        sh[w][2] = a2r;
        sh[w][3] = a2i;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        double acc = 0;
        for (int k = 0; k < kNB / kWave; k++) acc += sh[k][threadIdx.x];
        partial[(((size_t)yy * ntx + xx) * nchunk + chunk) * 4 + threadIdx.x] = acc;
    }
}

// W[w][y][x] (complex) = - sum of the chunk partials, in chunk order
__global__ __launch_bounds__(kNB) void k_nucleon_final(int nty, int ntx, int nchunk, const double* __restrict__ partial,
                                                       double* __restrict__ W) {
    const int e = blockIdx.x * kNB + threadIdx.x;  // (y * ntx + x) * 2 + w
    if (e >= nty * ntx * 2) return;
    const int w = e % 2, yx = e / 2;
    double re = 0, im = 0;
    for (int c = 0; c < nchunk; c++) {
        re += partial[((size_t)yx * nchunk + c) * 4 + 2 * w];
        im += partial[((size_t)yx * nchunk + c) * 4 + 2 * w + 1];
    }
    W[((size_t)w * nty * ntx + yx) * 2] = -re;
    W[((size_t)w * nty * ntx + yx) * 2 + 1] = -im;
}

}  // namespace


dd_status nucleon_lines(dd_ctx* c, const cpx<double>* U, double kappa, const dd_domain& gbar, const dd_domain& gstar,
                        int t_phi, int nvec, const cpx<double>* phi, int x0, cpx<double>* xi, cpx<double>* eta,
                        const dd_solver_params& p, dd_solve_stats* stats) {
    const dd_lattice& lat = c->lat;
    const int T = lat.T, L3 = lat.L * lat.L * lat.L;
    const Geo gb = make_geo(lat, &gbar), gs = make_geo(lat, &gstar);
    const int kp = ((t_phi - gbar.t0) % T + T) % T, kx = ((x0 - gbar.t0) % T + T) % T;
    const size_t nb = (size_t)DD_MAX_RHS * 12 * std::max(gb.nsite, gs.nsite);
    dd_status e = DD_OK;
    cpx<double>* rhs = (cpx<double>*)workspace(c, W_DISC0, nb * sizeof(cpx<double>), &e);
    if (e != DD_OK) return e;
    cpx<double>* w = (cpx<double>*)workspace(c, W_DISC1, nb * sizeof(cpx<double>), &e);
    if (e != DD_OK) return e;
    dd_solve_stats tot[2];
    std::memset(tot, 0, sizeof(tot));
    tot[0].nrhs = tot[1].nrhs = nvec;
    dd_status worst = DD_OK;
    const dd_domain src{t_phi, 1};
    for (int a0 = 0; a0 < nvec; a0 += DD_MAX_RHS) {
        const int nc = std::min(DD_MAX_RHS, nvec - a0);
        const cpx<double>* ph = phi + (size_t)a0 * 12 * L3;
        // xi: D_Gbar^+ w = phi (placed on slice t_phi), xi = conj(w) on slice x0
        launch_zero<double>(c, (size_t)nc * 12 * gb.nsite, rhs);
        launch_slab_embed(c, L3, gb.nt, kp, 1, nc, const_cast<cpx<double>*>(ph), rhs, 0);
        DD_HIP(c, hipGetLastError());
        for (int side = 0; side < 2; side++) {
            dd_solve_stats st;
            if (side == 0) {
                e = solve(c, U, kappa, gb, nc, rhs, w, p, &st, 1);
            } else {
                // eta: D_Gstar eta = D_{Gstar, dGstar} phi
                launch_zero<double>(c, (size_t)nc * 12 * gs.nsite, rhs);
                launch_frontier(c, lat, U, gstar, src, nc, ph, rhs, 1.0);
                DD_HIP(c, hipGetLastError());
                e = solve(c, U, kappa, gs, nc, rhs, eta + (size_t)a0 * 12 * gs.nsite, p, &st, 0);
            }
            if (e != DD_OK && e != DD_ERR_NOCONV) return e;
            if (e == DD_ERR_NOCONV) worst = e;
            tot[side].iters += st.iters;
            tot[side].updates += st.updates;
            tot[side].restarts += st.restarts;
            tot[side].ms += st.ms;
            for (int j = 0; j < nc; j++)
                tot[side].true_rel_resid[(a0 + j) % DD_MAX_RHS] =
                    std::max(tot[side].true_rel_resid[(a0 + j) % DD_MAX_RHS], st.true_rel_resid[j]);
            if (side == 0) {
                hipLaunchKernelGGL(k_conj_slice, dim3((unsigned)((L3 + kNB - 1) / kNB), (unsigned)(12 * nc)), dim3(kNB),
                                   0, c->stream, L3, gb.nsite, kx, w, xi + (size_t)a0 * 12 * L3);
                DD_HIP(c, hipGetLastError());
            }
        }
    }
    if (stats) {
        stats[0] = tot[0];
        stats[1] = tot[1];
    }
    DD_HIP(c, hipStreamSynchronize(c->stream));
    if (worst != DD_OK) return fail(c, worst, "a nucleon line solve did not converge: " + c->err);
    return DD_OK;
}

dd_status baryon_blocks(dd_ctx* c, int n, int nt, const cpx<double>* s, cpx<double>* B) {
    const int L3 = c->lat.L * c->lat.L * c->lat.L;
    const long long nsite = (long long)nt * L3;
    const size_t M = (size_t)n * (n + 1) / 2;  // pairs i <= j
    // sites per chunk: the diquarks of a chunk stay below 2 GiB
    int X = (int)std::min<size_t>((size_t)L3, std::max<size_t>(64, ((size_t)1 << 31) / (M * 3 * sizeof(cpx<double>))));
    // the packed quarks too (the product addresses both through 32-bit buffer offsets)
    X = (int)std::min<size_t>((size_t)X, ((size_t)1 << 31) / ((size_t)3 * 4 * n * sizeof(cpx<double>)));
    if (const char* env = std::getenv("DD_BLOCK_CHUNK")) X = std::max(1, std::min(X, std::atoi(env)));  // tests
    dd_status e = DD_OK;
    cpx<double>* E = (cpx<double>*)workspace(c, W_DISC2, (M * 3 * X + M * 4 * n) * sizeof(cpx<double>), &e);
    if (e != DD_OK) return e;
    cpx<double>* Bp = E + M * 3 * X;  // the packed blocks of one slice
    cpx<double>* Sp = (cpx<double>*)workspace(c, W_DISC3, (size_t)3 * X * 4 * n * sizeof(cpx<double>), &e);
    if (e != DD_OK) return e;
    // the k range of a chunk's product is split so that about 16 workgroups per CU run in all
    const int N = 4 * n;
    const int ntile = (int)(((M + kGM - 1) / kGM) * ((N + kGN - 1) / kGN));
    const int nkt_max = (3 * X + kGK - 1) / kGK;
    const int nsplit_max = std::max(1, std::min(nkt_max, (16 * 256 + ntile - 1) / ntile));
    cpx<double>* Cpart =
        (cpx<double>*)workspace(c, W_DISC1, (size_t)nsplit_max * M * N * sizeof(cpx<double>), &e);
    if (e != DD_OK) return e;
    const size_t nfull = (size_t)4 * n * n * n;
    for (int t = 0; t < nt; t++) {
        for (int x0 = 0; x0 < L3; x0 += X) {
            const int xc = std::min(X, L3 - x0);
            const long long off = (long long)t * L3 + x0;
            hipLaunchKernelGGL(k_pack_quarks, dim3((unsigned)((xc + kNB - 1) / kNB), (unsigned)(12 * n)), dim3(kNB), 0,
                               c->stream, n, nsite, off, xc, s, Sp);
            hipLaunchKernelGGL(k_diquarks, dim3((unsigned)((xc + kXT - 1) / kXT)), dim3(kNB), 0, c->stream, n, nsite,
                               off, xc, s, E);
            // Bp (P x 4n, column-major) (+)= E (P x 3 xc) Sp (3 xc x 4n)
            const int K = 3 * xc;
            const int nkt = (K + kGK - 1) / kGK;
            const int kps = (nkt + nsplit_max - 1) / nsplit_max;
            const int nsplit = (nkt + kps - 1) / kps;
            hipLaunchKernelGGL(k_zgemm_mfma, dim3((unsigned)(ntile * nsplit)), dim3(kGThreads), 0, c->stream, (int)M, N,
                               K, kps, E, Sp, Cpart);
            hipLaunchKernelGGL(k_zgemm_reduce, dim3((unsigned)((M * N + kNB - 1) / kNB)), dim3(kNB), 0, c->stream,
                               M * (size_t)N, nsplit, x0 == 0 ? 0 : 1, Cpart, Bp);
            DD_HIP(c, hipGetLastError());
        }
        hipLaunchKernelGGL(k_unpack_blocks, dim3((unsigned)((nfull + kNB - 1) / kNB)), dim3(kNB), 0, c->stream, n, M,
                           Bp, B + (size_t)t * nfull);
    }
    DD_HIP(c, hipGetLastError());
    return DD_OK;
}

dd_status nucleon_contract(dd_ctx* c, int n, int ntx, const cpx<double>* Bx, int nty, const cpx<double>* By,
                           double* W_host) {
    const size_t sl = (size_t)4 * n * n * n;
    const int nchunk = (int)((sl + kCChunk - 1) / kCChunk);
    dd_status e = DD_OK;
    cpx<double>* P = (cpx<double>*)workspace(c, W_DISC2, 2 * (size_t)ntx * sl * sizeof(cpx<double>), &e);
    if (e != DD_OK) return e;
    cpx<double>* P1 = P;
    cpx<double>* P2 = P + (size_t)ntx * sl;
    double* part = (double*)workspace(c, W_DISC3, ((size_t)nty * ntx * nchunk * 4 + (size_t)nty * ntx * 4) *
                                                      sizeof(double), &e);
    if (e != DD_OK) return e;
    double* Wd = part + (size_t)nty * ntx * nchunk * 4;
    for (int x = 0; x < ntx; x++)
        hipLaunchKernelGGL(k_block_perms, dim3((unsigned)((sl + kNB - 1) / kNB)), dim3(kNB), 0, c->stream, n,
                           Bx + (size_t)x * sl, P1 + (size_t)x * sl, P2 + (size_t)x * sl);
    hipLaunchKernelGGL(k_nucleon_partial, dim3((unsigned)nchunk, (unsigned)nty, (unsigned)ntx), dim3(kNB), 0,
                       c->stream, n, nchunk, ntx, By, P1, P2, part);
    hipLaunchKernelGGL(k_nucleon_final, dim3((unsigned)((nty * ntx * 2 + kNB - 1) / kNB)), dim3(kNB), 0, c->stream,
                       nty, ntx, nchunk, part, Wd);
    DD_HIP(c, hipGetLastError());
    DD_HIP(c, hipMemcpyAsync(W_host, Wd, (size_t)nty * ntx * 4 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    DD_HIP(c, hipStreamSynchronize(c->stream));
    return DD_OK;
}

}  // namespace dd
