"""Pins for the oracle's lattice geometry (Sec. 2.1, Fig. 1 caption, Sec. 3.3)."""
import itertools

import numpy as np
import pytest

import oracle
from oracle import Lattice

LATTICES = [(2, (2, 2)), (2, (3, 3)), (2, (3, 4)), (2, (2, 7)), (2, (4, 4)), (3, (2, 2, 2)),
            (3, (2, 2, 3)), (3, (3, 3, 3))]


def test_caption_plaquettes(golden):
    """Caption of Fig. 1 lists two plaquettes of each lattice (1-based link numbers)."""
    g = golden["fig1_caption_plaquettes"]
    for key, d, L in (("2x2x2", 3, (2, 2, 2)), ("3x3", 2, (3, 3))):
        lat = Lattice(d, L)
        have = {tuple(sorted(int(x) + 1 for x in p)) for p in lat.plaq}
        for want in g[key]:
            assert tuple(sorted(want)) in have


def test_counts(golden):
    g = golden["lattice_counts"]
    assert (Lattice(3, (2, 2, 2)).n_links, Lattice(3, (2, 2, 2)).n_plaq) == (
        g["2x2x2"]["n_links"], g["2x2x2"]["n_plaq"])
    assert (Lattice(2, (3, 3)).n_links, Lattice(2, (3, 3)).n_plaq) == (
        g["3x3"]["n_links"], g["3x3"]["n_plaq"])
    for d, L in LATTICES:
        lat = Lattice(d, L)
        V = int(np.prod(L))
        assert lat.n_links == d * V          # N_l = d L^d
        assert lat.n_plaq == lat.n_links * (d - 1) // 2   # N_p = N_l (d-1)/2


@pytest.mark.parametrize("d,L", LATTICES)
def test_incidence(d, L):
    lat = Lattice(d, L)
    # every plaquette has 4 distinct links, every star 2d distinct links
    assert all(len(set(p.tolist())) == 4 for p in lat.plaq)
    assert all(len(set(s.tolist())) == 2 * d for s in lat.stars)
    # each link borders 2(d-1) plaquettes (Sec. 2.2 error counting) and ends at 2 sites
    cnt_p = np.bincount(lat.plaq.ravel(), minlength=lat.n_links)
    cnt_s = np.bincount(lat.stars.ravel(), minlength=lat.n_links)
    assert np.all(cnt_p == 2 * (d - 1))
    assert np.all(cnt_s == 2)
    # every plaquette boundary is closed: each of its corner sites touches 0 or 2 of its links
    star_sets = [set(s.tolist()) for s in lat.stars]
    for p in lat.plaq:
        for s in star_sets:
            assert len(s & set(p.tolist())) in (0, 2)


def _mask(links):
    m = 0
    for q in links:
        m ^= 1 << int(q)
    return m


def test_cube_faces_multiply_to_one():
    """In 3D the six faces of an elementary cube share every edge twice: prod U_p = 1."""
    lat = Lattice(3, (2, 2, 3))
    faces = {}
    for i, p in enumerate(lat.plaq):
        faces[i] = _mask(p)
    # plaquettes indexed by (site, plane) with planes (x,y), (x,z), (y,z)
    for s in range(lat.n_sites):
        x = [s % 2, (s // 2) % 2, s // 4]
        def P(site_x, plane):
            return faces[3 * lat.site(site_x) + plane]
        m = 0
        m ^= P(x, 0) ^ P([x[0], x[1], x[2] + 1], 0)
        m ^= P(x, 1) ^ P([x[0], x[1] + 1, x[2]], 1)
        m ^= P(x, 2) ^ P([x[0] + 1, x[1], x[2]], 2)
        assert m == 0


def _gf2_rank(rows):
    rows = list(rows)
    rank = 0
    bit = 0
    while rows and bit < 64:
        piv = next((r for r in rows if (r >> bit) & 1), None)
        if piv is not None:
            rows.remove(piv)
            rows = [r ^ piv if (r >> bit) & 1 else r for r in rows]
            rank += 1
        bit += 1
    return rank


@pytest.mark.parametrize("d,L", LATTICES)
def test_gauge_subspace_dimension(d, L):
    """Independent Gauss laws: all stars but one (their product is the identity).

    The gauge-invariant subspace then has dimension 2^(N_l - N_sites + 1).
    """
    lat = Lattice(d, L)
    star_masks = [_mask(s) for s in lat.stars]
    assert _gf2_rank(star_masks) == lat.n_sites - 1
    # every plaquette commutes with every star (even overlap), Sec. 2.2
    for p in lat.plaq:
        pm = _mask(p)
        for sm in star_masks:
            assert bin(pm & sm).count("1") % 2 == 0


def _z_support(lat):
    """All values of Z = -sum_p U_p over the 2^N_l basis states (brute force)."""
    N = lat.N
    b = np.arange(1 << N, dtype=np.int64)
    z = np.zeros(1 << N, dtype=np.int64)
    for p in lat.plaq:
        par = np.zeros_like(b)
        for q in p:
            par ^= (b >> int(q)) & 1
        z += np.where(par == 1, 1, -1)   # Z_p = -U_p
    return sorted(set(z.tolist()))


def test_z_spectrum_supports(golden):
    """Sec. 3.3: Z takes +-24, +-16, +-12, +-8, +-4, 0 on 2x2x2 and -9..7 step 4 on 3x3."""
    g = golden["z_spectrum"]
    assert _z_support(Lattice(2, (3, 3))) == g["3x3"]
    assert _z_support(Lattice(3, (2, 2, 2))) == g["2x2x2"]


def _x_support_trivial_sector(lat, tHooft_lines):
    """Values of X = -sum sigma^x over basis states in the sigma^x basis that obey
    every Gauss law and every 't Hooft constraint V = +1 (brute force)."""
    N = lat.N
    b = np.arange(1 << N, dtype=np.int64)
    ok = np.ones(1 << N, dtype=bool)
    for s in list(lat.stars) + list(tHooft_lines):
        par = np.zeros_like(b)
        for q in s:
            par ^= (b >> int(q)) & 1
        ok &= par == 0
    # bit = 1 means sigma^x = -1 on that link
    pop = np.array([bin(v).count("1") for v in b[ok]])
    return sorted(set((-N + 2 * pop).tolist()))


def _tHooft(lat):
    """V_mu: sigma^x over the mu-links that start on the plane x_mu = 0."""
    out = []
    for mu in range(lat.d):
        links = []
        for s in range(lat.n_sites):
            x = []
            t = s
            for nu in range(lat.d):
                x.append(t % lat.L[nu]); t //= lat.L[nu]
            if x[mu] == 0:
                links.append(lat.d * s + (lat.d - 1 - mu))
        out.append(links)
    return out


def test_x_spectrum_supports(golden):
    g = golden["x_spectrum"]
    l3 = Lattice(3, (2, 2, 2))
    assert _x_support_trivial_sector(l3, _tHooft(l3)) == g["2x2x2"]
    l2 = Lattice(2, (3, 3))
    sup = _x_support_trivial_sector(l2, _tHooft(l2))
    assert set(sup) <= set(g["3x3_superset"])
    assert not set(sup) & set(g["3x3_forbidden"])
    assert all((x + 18) % 4 == 0 for x in sup)


def test_walk_loops():
    lat = Lattice(2, (3, 3))
    # a 1x1 walk is a plaquette
    have = {tuple(sorted(p.tolist())) for p in lat.plaq}
    for s in range(lat.n_sites):
        assert tuple(sorted(lat.rect_loop(s, 0, 1, 1, 1).tolist())) in have
    # a 2x2 loop has 8 links and equals the product of its 4 plaquettes
    w = lat.rect_loop(0, 0, 1, 2, 2)
    assert len(w) == 8
    m = 0
    for x, y in itertools.product(range(2), range(2)):
        m ^= _mask(lat.rect_loop(lat.site([x, y]), 0, 1, 1, 1))
    assert m == _mask(w)
    # non-contractible line has L links all of one direction
    line = lat.line(0, 1)
    assert len(line) == 3


@pytest.mark.parametrize("d,L", [(2, (3, 3)), (2, (4, 4)), (3, (2, 2, 2))], ids=["3x3", "4x4", "2x2x2"])
def test_wilson_contours(d, L):
    """Sec. 3.1: c1, c2, c3 have perimeters in the ratios 1 : 1.5 : 2 and enclose 1 : 2 : 3
    plaquettes.  Each walk is a closed contractible loop (even overlap with every 't Hooft
    surface), its length is the perimeter, and its links are exactly the boundary (the
    symmetric difference) of a chain of 1, 2, 3 plaquettes of the lattice's plaquette list."""
    lat = Lattice(d, L)
    plaq_sets = [set(int(q) for q in p) for p in lat.plaq]
    for k, per in ((1, 4), (2, 6), (3, 8)):
        c = set(int(q) for q in lat.contour(k))
        assert len(c) == per
        for mu in range(d):
            assert len(c & set(lat.thooft(mu))) % 2 == 0
        # some chain of k distinct plaquettes has c as its boundary (brute force)
        found = False
        for combo in itertools.combinations(range(lat.n_plaq), k):
            b = set()
            for p in combo:
                b ^= plaq_sets[p]
            if b == c:
                found = True
                break
        assert found, k
    # the area ratios distinguish the laws: no chain of fewer plaquettes bounds c2 or c3
    for k in (2, 3):
        c = set(int(q) for q in lat.contour(k))
        for j in range(1, k):
            for combo in itertools.combinations(range(lat.n_plaq), j):
                b = set()
                for p in combo:
                    b ^= plaq_sets[p]
                assert b != c
