"""Host emulation of the index arithmetic of the even-odd time-sweep half hop.

The half-hop kernels (k_eo_hop on one lattice or slab, k_beo_hop on a batch of domains)
decode a workgroup into (domain, group of KC columns, tile of NT site pairs of a slice,
chunk of time slices); a thread owns one pair (xh, y, z) and sweeps the chunk, writing the
output site of its parity on every slice and carrying the projected backward time
neighbours of the next two slices in registers (cA serves slice t, cB slice t + 1, the
spinor loaded for the forward hop of slice t serves slice t + 2).  This module restates
that arithmetic with numpy and checks, over the geometries the library runs (the 96
uneven domains of the batched workload, the 16 x 32^3 slabs and the whole 64 x 32^3
lattice, small odd cases), for KC = 1 and 2, every chunk length the tuners try, plain and
brick tiles, tile-major and chunk-major orders, XCD remap on and off and both parities:

  - every output half site of every column is written exactly once per launch, and it has
    the parity asked for;
  - every neighbour read is in range, of the other parity, and the lattice neighbour of the
    output site (periodic in space; across the time edge only on a whole lattice);
  - the carried backward neighbour a slice consumes is the spinor at (x(t), t - 1) of that
    same thread, loaded earlier in the chunk or at its start, never a value of another
    slice or column;
  - the workgroup decode covers every (column group, tile, chunk) of every domain once.
"""
import numpy as np
import pytest

from paper_1612_06424_amd.inputs import batched_domains

NT = 256
NXCD = 8


def pair_site(pr, Lh, L, blocked):
    """(xh, y, z) of pair index pr within a slice (plain rows, or 4 x 4 (y, z) bricks)."""
    pr = np.asarray(pr)
    if blocked:
        per = Lh * 16
        b, r = pr // per, pr % per
        q, nby = r // Lh, L >> 2
        return r - q * Lh, (b % nby) * 4 + (q & 3), (b // nby) * 4 + (q >> 2)
    yz = pr // Lh
    return pr - yz * Lh, yz % L, yz // L


def xcd_remap(bid, nblk):
    q, r = nblk // NXCD, nblk % NXCD
    xcd, loc = bid % NXCD, bid // NXCD
    return np.where(xcd < r, xcd * (q + 1) + loc, r * (q + 1) + (xcd - r) * q + loc)


def sweep_writes(L, nt, whole, tc, blocked, chunk_major, p_out, slip=None):
    """Emulates one column group of a launch and checks every write and read; slip plants
    one mistake (for the test that the checks catch it)."""
    L3, L2 = L ** 3, L * L
    Lh, L3h = L // 2, L3 // 2
    nh = nt * L3 // 2
    ntile = (L3h + NT - 1) // NT
    nchunk = (nt + tc - 1) // tc
    blks = np.arange(ntile * nchunk)
    tile = blks // nchunk if chunk_major else blks % ntile
    chunk = blks % nchunk if chunk_major else blks // ntile
    if slip == "decode":
        chunk = blks // ntile if chunk_major else blks % nchunk
    # the (tile, chunk) decode is a bijection onto the tiles x chunks
    assert len(set(zip(tile.tolist(), chunk.tolist()))) == ntile * nchunk
    assert tile.max() == ntile - 1 and chunk.max() == nchunk - 1
    # a thread's pair depends on its tile only, so the chunks are emulated with every
    # thread of every tile at once (tiles are disjoint ranges of pair indices)
    pr = np.arange(ntile * NT)
    pr = pr[pr < L3h]
    xh, y, z = pair_site(pr, Lh, L, blocked)
    yz = z * L + y
    assert len(set((yz * Lh + xh).tolist())) == L3h  # every pair of the slice once

    def xof(t):
        return 2 * xh + ((p_out + t + y + z + (slip == "parity")) & 1)

    def site(t, x):  # local site index of (t, x, y, z)
        return t * L3 + yz * L + x

    def load_bw(t):  # the carry for slice t: site (x(t), t - 1), -1 for zero
        if t < nt and (t > 0 or whole):
            tm = t - 1 if t > 0 else nt - 1
            return site(tm, xof(t))
        return np.full(pr.shape, -1)

    zero = np.full(pr.shape, -1)
    written = []
    for ch in range(nchunk):
        tb = ch * tc
        te = min(nt, tb + tc - (slip == "chunk"))
        cA = load_bw(tb) if tb < te else zero
        cB = load_bw(tb + 1) if tb + 1 < te else zero
        for t in range(tb, te):
            x = xof(t)
            s = site(t, x)
            assert np.all(((t + x + y + z) & 1) == p_out)
            written.append(s >> 1)
            if t > 0 or whole:  # the backward time hop consumes the carry
                tm = t - 1 if t > 0 else nt - 1
                assert np.array_equal(cA, site(tm, x)), (t, tb)
            endt = t == nt - 1
            nb2 = zero
            if not endt or whole:
                fwd = yz * L + x if endt else s + L3
                assert np.array_equal(fwd, site(0 if endt else t + 1, x))
                if not endt:
                    nb2 = fwd
            # spatial neighbours: periodic, of the other parity, in range
            steps = ((np.where(x == L - 1, -(L - 1), 1), (1, 0, 0)), (np.where(x == 0, L - 1, -1), (-1, 0, 0)),
                     (np.where(y == L - 1, -(L - 1) * L, L), (0, 1, 0)), (np.where(y == 0, (L - 1) * L, -L), (0, -1, 0)),
                     (np.where(z == L - 1, -(L - 1) * L2, L2), (0, 0, 1)),
                     (np.where(z == 0, (L - 1) * L2, -L2), (0, 0, -1)))
            for d, (dx, dy, dz) in steps:
                nb = s + d
                want = site(t, (x + dx) % L) + ((y + dy) % L - y) * L + ((z + dz) % L - z) * L2
                assert np.array_equal(nb, want)
                assert np.all(nb >= 0) and np.all((nb >> 1) < nh)
            if slip == "carry":
                cA, cB = nb2, cB
            else:
                cA, cB = cB, nb2
    w = np.concatenate(written)
    assert np.array_equal(np.sort(w), np.arange(nh)), "each output half site exactly once"
    return ntile * nchunk


GEOMS = sorted({(d["L"], d["T"], 1) for d in batched_domains(96)}) + [(32, 16, 0), (6, 8, 1), (4, 6, 0)]


@pytest.mark.parametrize("L,nt,whole", GEOMS)
@pytest.mark.parametrize("p_out", [0, 1])
def test_every_site_once_and_carries_match(L, nt, whole, p_out):
    for tc in (1, 2, 3, 4, 8):
        for blocked in ((0, 1) if L % 4 == 0 else (0,)):
            for chunk_major in (False, True):
                sweep_writes(L, nt, whole, min(tc, nt), blocked, chunk_major, p_out)


def test_whole_64x32_lattice():
    """The whole 64 x 32^3 lattice at the chunk lengths the shipped launch shapes use."""
    for tc, blocked, chunk_major in ((1, 1, True), (4, 1, False), (4, 1, True)):
        for p_out in (0, 1):
            sweep_writes(32, 64, 1, tc, blocked, chunk_major, p_out)


@pytest.mark.parametrize("kc", [1, 2])
@pytest.mark.parametrize("remap", [0, 1])
def test_batched_workgroup_decode(kc, remap):
    """k_beo_hop's decode: workgroup -> (domain by binary search over first workgroups,
    group of KC columns, block) over the 96 uneven domains with 12 columns each."""
    doms = batched_domains(96)
    for tc in (1, 2, 4, 8):
        blk0, descs, blk = [], [], 0
        for d in doms:
            L, T = d["L"], d["T"]
            ntile = (L ** 3 // 2 + NT - 1) // NT
            tcd = min(tc, T)
            nblk = ntile * ((T + tcd - 1) // tcd)
            blk0.append(blk)
            descs.append((ntile, nblk))
            blk += nblk * 12 // kc
        bids = np.arange(blk)
        lb_all = xcd_remap(bids, blk) if remap else bids
        assert np.array_equal(np.sort(lb_all), bids)  # the remap is a permutation
        blk0 = np.array(blk0)
        dom = np.searchsorted(blk0, lb_all, side="right") - 1
        seen = set()
        for b, i in zip(lb_all.tolist(), dom.tolist()):
            ntile, nblk = descs[i]
            lb = b - blk0[i]
            ngrp = 12 // kc
            col0, bk = (lb % ngrp) * kc, lb // ngrp
            assert 0 <= bk < nblk and 0 <= col0 <= 12 - kc
            for k in range(kc):
                key = (i, col0 + k, bk)
                assert key not in seen
                seen.add(key)
        assert len(seen) == sum(12 * nblk for _, nblk in descs)


@pytest.mark.parametrize("slip", ["carry", "chunk", "parity", "decode"])
def test_emulation_catches_planted_slips(slip):
    """The checks have teeth: carries rotated the wrong way, a chunk one slice short, the
    output parity flipped, tile and chunk decoded with the other order's divisor."""
    with pytest.raises(AssertionError):
        sweep_writes(16, 16, 1, 4, 1, True, 0, slip=slip)  # 8 tiles x 4 chunks
