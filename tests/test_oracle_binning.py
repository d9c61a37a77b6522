"""Pins for the oracle's binning and order: brute-force tile overlap, Python's
own sort on (tile, depth bits, id) tuples, and invariants."""

import numpy as np

import synth
from oracle.binning import bin_and_sort, depth_bits
from oracle.projection import project


def _proj(seed=0, W=128, H=128):
    P, cam, _ = synth.cfg1_inputs(seed, width=W, height=H)
    return project(P, cam), cam


def test_tile_sets_match_brute_force_overlap():
    # Independent statement of the rectangle rule: tile (tx, ty) overlaps the
    # square [u-r, u+r] x [v-r, v+r] iff u + r >= tx*16 and u - r < (tx+1)*16
    # (same in y), restricted to tiles of the image.
    for W, H in [(128, 128), (100, 75)]:
        proj, cam = _proj(1, W, H)
        bins = bin_and_sort(proj)
        TX, TY = proj["tiles"]
        for t in range(TX * TY):
            tx, ty = t % TX, t // TX
            s, e = bins["ranges"][t]
            got = set(bins["values"][s:e].tolist())
            want = set()
            for g in np.nonzero(proj["visible"])[0]:
                u, v, r = proj["u"][g], proj["v"][g], proj["radius"][g]
                if (u + r >= tx * 16 and u - r < (tx + 1) * 16 and
                        v + r >= ty * 16 and v - r < (ty + 1) * 16):
                    want.add(int(g))
            assert got == want, t


def test_order_is_python_sort_of_tuples():
    proj, _ = _proj(2)
    bins = bin_and_sort(proj)
    TX, TY = proj["tiles"]
    dbits = depth_bits(proj["depth32"])
    tuples = []
    for g in np.nonzero(proj["visible"])[0]:
        x0, y0, x1, y1 = proj["rect"][g]
        for ty in range(y0, y1 + 1):
            for tx in range(x0, x1 + 1):
                tuples.append((ty * TX + tx, int(dbits[g]), int(g)))
    tuples.sort()
    assert [t[2] for t in tuples] == bins["values"].tolist()
    assert [(t[0] << 32) | t[1] for t in tuples] == [int(k) for k in bins["keys"]]


def test_invariants():
    proj, _ = _proj(3)
    bins = bin_and_sort(proj)
    k = bins["keys"]
    assert (k[1:] >= k[:-1]).all()
    lens = bins["ranges"][:, 1] - bins["ranges"][:, 0]
    assert lens.sum() == bins["num_pairs"] == proj["tiles_touched"].sum()
    pairs = set(zip((k >> np.uint64(32)).tolist(), bins["values"].tolist()))
    assert len(pairs) == bins["num_pairs"]          # each (tile, Gaussian) once
    # depth is positive, so float bits order like values
    d = proj["depth32"][proj["visible"]]
    o = np.argsort(d, kind="stable")
    assert (np.diff(depth_bits(d[o]).astype(np.int64)) >= 0).all()


def test_empty_and_single():
    proj, _ = _proj(0)
    for k in ("visible",):
        proj = dict(proj)
    proj["visible"] = np.zeros_like(proj["visible"])
    b = bin_and_sort(proj)
    assert b["num_pairs"] == 0 and (b["ranges"] == 0).all()
