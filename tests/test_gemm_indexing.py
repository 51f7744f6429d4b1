"""Host emulation of the index arithmetic of the baryon-block product k_zgemm_mfma.

The kernel computes C = A B in complex FP64 (column-major, lda = M, ldb = K, ldc = M) on
v_mfma_f64_16x16x4f64.  A workgroup decodes its XCD-remapped index into (column tile
fastest, row tile, k split), stages 64 x 16 panels of A and 16 x 64 panels of B in LDS
(thread t: A entries (t % 64, t / 64 + 4 r), B entries (t % 16, t / 16 + 16 r)), and each of
its four wavefronts multiplies a 32 x 32 quarter as 2 x 2 blocks of 16 x 16, four real MFMAs
per complex block.  The MFMA lane layout used here is the one read off an in-bounds probe on
the MI355X: lane l holds A[l % 16][l / 16] and B[l / 16][l % 16], and rows l / 16 + 4 e
(e = 0..3) of column l % 16 of the result.  This module restates that arithmetic with
numpy and checks, on ragged shapes and several split counts, that every entry of every
split's partial C is written exactly once, that the workgroup decode covers every
(tile, split) once, and that the splits add up to A B; a planted wrong result layout
(rows 4 (l / 16) + e) must fail.
"""
import numpy as np
import pytest

GM = GN = 64
GK = 16
NXCD = 8


def xcd_remap(bid, nblk):
    q, r = divmod(nblk, NXCD)
    xcd, loc = bid % NXCD, bid // NXCD
    return xcd * (q + 1) + loc if xcd < r else r * (q + 1) + (xcd - r) * q + loc


def mfma(a, b, c, rows_of):
    """One 16 x 16 x 4 FP64 MFMA on per-lane operands a, b (64,) and accumulator c (64, 4)."""
    A = np.zeros((16, 4))
    B = np.zeros((4, 16))
    lanes = np.arange(64)
    A[lanes % 16, lanes // 16] = a
    B[lanes // 16, lanes % 16] = b
    D = A @ B
    out = c.copy()
    for e in range(4):
        out[:, e] += D[rows_of(lanes, e), lanes % 16]
    return out


def measured_rows(lanes, e):
    return lanes // 16 + 4 * e


def emulate(A, B, nsplit_max, rows_of=measured_rows):
    M, K = A.shape
    N = B.shape[1]
    tm, tn = -(-M // GM), -(-N // GN)
    nkt = -(-K // GK)
    kps = -(-nkt // nsplit_max)
    nsplit = -(-nkt // kps)
    grid = tm * tn * nsplit
    Cp = np.zeros((nsplit, M, N), complex)
    written = np.zeros((nsplit, M, N), int)
    work = [xcd_remap(b, grid) for b in range(grid)]
    assert sorted(work) == list(range(grid)), "the remap is a permutation"
    lanes = np.arange(64)
    for w in work:
        nt, mt, sp = w % tn, (w // tn) % tm, w // (tn * tm)
        m0, n0 = mt * GM, nt * GN
        cr = np.zeros((4, 2, 2, 64, 4))
        ci = np.zeros((4, 2, 2, 64, 4))
        for kt in range(sp * kps, min(nkt, sp * kps + kps)):
            k0 = kt * GK
            As = np.zeros((GK, GM), complex)
            Bs = np.zeros((GK, GN), complex)
            for t in range(256):
                for r in range(4):
                    m, k = m0 + (t & 63), k0 + (t >> 6) + 4 * r
                    As[(t >> 6) + 4 * r, t & 63] = A[m, k] if m < M and k < K else 0
                    k, n = k0 + (t & 15), n0 + (t >> 4) + 16 * r
                    Bs[t & 15, (t >> 4) + 16 * r] = B[k, n] if k < K and n < N else 0
            for wv in range(4):
                wm, wn = wv & 1, wv >> 1
                for ks in range(GK // 4):
                    kk = 4 * ks + (lanes >> 4)
                    a = [As[kk, wm * 32 + i * 16 + (lanes & 15)] for i in range(2)]
                    b = [Bs[kk, wn * 32 + j * 16 + (lanes & 15)] for j in range(2)]
                    for i in range(2):
                        for j in range(2):
                            cr[wv, i, j] = mfma(a[i].real, b[j].real, cr[wv, i, j], rows_of)
                            ci[wv, i, j] = mfma(a[i].real, b[j].imag, ci[wv, i, j], rows_of)
                            cr[wv, i, j] = mfma(a[i].imag, -b[j].imag, cr[wv, i, j], rows_of)
                            ci[wv, i, j] = mfma(a[i].imag, b[j].real, ci[wv, i, j], rows_of)
        for wv in range(4):
            wm, wn = wv & 1, wv >> 1
            for i in range(2):
                for j in range(2):
                    for e in range(4):
                        row = m0 + wm * 32 + i * 16 + (lanes >> 4) + 4 * e
                        col = n0 + wn * 32 + j * 16 + (lanes & 15)
                        ok = (row < M) & (col < N)
                        Cp[sp, row[ok], col[ok]] = cr[wv, i, j, ok, e] + 1j * ci[wv, i, j, ok, e]
                        np.add.at(written, (sp, row[ok], col[ok]), 1)
    return Cp, written


def _matrices(M, N, K, seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((M, K)) + 1j * rng.standard_normal((M, K))
    B = rng.standard_normal((K, N)) + 1j * rng.standard_normal((K, N))
    return A, B


@pytest.mark.parametrize("M,N,K,nsplit_max", [(1, 4, 48, 3), (15, 20, 30, 3), (78, 48, 21, 2), (130, 70, 50, 4),
                                              (64, 64, 64, 1)])
def test_every_entry_once_and_the_product(M, N, K, nsplit_max):
    A, B = _matrices(M, N, K, M + N + K)
    Cp, written = emulate(A, B, nsplit_max)
    assert (written == 1).all()
    C = Cp.sum(0)
    ref = A @ B
    assert np.abs(C - ref).max() < 1e-12 * np.abs(ref).max()


def test_a_wrong_result_layout_is_caught():
    A, B = _matrices(15, 20, 30, 7)
    Cp, _ = emulate(A, B, 3, rows_of=lambda lanes, e: 4 * (lanes // 16) + e)
    # the kernel's stores follow the measured layout, so the planted one scrambles the rows
    assert np.abs(Cp.sum(0) - A @ B).max() > 1e-3
