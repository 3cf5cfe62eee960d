// Lattice geometry for the engine (Sec. 2.1 of arXiv:1910.08020).
//
// Sites are numbered with the x coordinate fastest and a neighbour table is
// built from per-direction strides.  Link l(s, mu) = d s + (d-1-mu): with
// 1-based numbers this makes links 3s+1, 3s+2, 3s+3 the z, y, x links of site
// s in 3D (2s+1, 2s+2 the y, x links in 2D), which reproduces the plaquettes
// quoted in the caption of Fig. 1.
#include <cstring>

#include "lgt_internal.hpp"

namespace lgt {

std::string build_lattice(int d, const int *L, Lattice &out)
{
    if (d != 2 && d != 3) return "d must be 2 or 3";
    if (!L) return "null extents";
    Lattice lat;
    lat.d = d;
    long long V = 1;
    for (int mu = 0; mu < d; ++mu) {
        if (L[mu] < 2) return "every extent must be >= 2";
        if (L[mu] > 64) return "extent too large";
        lat.L[mu] = L[mu];
        V *= L[mu];
    }
    if (d * V > kMaxLinks) return "too many links for one GPU state (max 34)";
    lat.n_sites = (int)V;
    lat.n_links = d * (int)V;
    lat.n_plaq = (int)V * d * (d - 1) / 2;
    if (lat.n_plaq > kMaxPlaq) return "too many plaquettes (max 32)";

    // neighbour tables from strides
    int stride[3] = {1, 1, 1};
    for (int mu = 1; mu < d; ++mu) stride[mu] = stride[mu - 1] * lat.L[mu - 1];
    lat.fwd.assign((size_t)V * d, 0);
    lat.bwd.assign((size_t)V * d, 0);
    for (int s = 0; s < V; ++s)
        for (int mu = 0; mu < d; ++mu) {
            int xm = (s / stride[mu]) % lat.L[mu];
            lat.fwd[s * d + mu] = (xm + 1 < lat.L[mu]) ? s + stride[mu]
                                                         : s - (lat.L[mu] - 1) * stride[mu];
            lat.bwd[s * d + mu] = (xm > 0) ? s - stride[mu] : s + (lat.L[mu] - 1) * stride[mu];
        }

    // plaquettes: per site, planes (mu, nu) with mu < nu in lexicographic order
    for (int s = 0; s < V; ++s)
        for (int mu = 0; mu < d; ++mu)
            for (int nu = mu + 1; nu < d; ++nu) {
                int l0 = lat.link(s, mu);
                int l1 = lat.link(lat.fwd[s * d + mu], nu);
                int l2 = lat.link(lat.fwd[s * d + nu], mu);
                int l3 = lat.link(s, nu);
                lat.plaq_links.insert(lat.plaq_links.end(), {l0, l1, l2, l3});
                lat.plaq_mask.push_back((1ull << l0) | (1ull << l1) | (1ull << l2) | (1ull << l3));
            }
    // stars: the 2d links ending at each site (Gauss law)
    for (int s = 0; s < V; ++s) {
        uint64_t m = 0;
        for (int mu = 0; mu < d; ++mu) {
            m |= 1ull << lat.link(s, mu);
            m |= 1ull << lat.link(lat.bwd[s * d + mu], mu);
        }
        lat.star_mask.push_back(m);
    }
    lat.link_plaqs.assign(lat.n_links, 0u);
    for (int p = 0; p < lat.n_plaq; ++p)
        for (int k = 0; k < 4; ++k) lat.link_plaqs[lat.plaq_links[4 * p + k]] |= 1u << p;
    out = std::move(lat);
    return "";
}

// Boundary of an a x b block of plaquettes: the product of the plaquettes inside.
uint64_t region_mask(const Lattice &lat, int site, int mu, int nu, int a, int b)
{
    const int d = lat.d;
    // plaquette index of (s; mu, nu): plane ordinal among pairs mu<nu
    int plane = 0;
    for (int m = 0; m < d; ++m)
        for (int n = m + 1; n < d; ++n) {
            if (m == mu && n == nu) goto found;
            ++plane;
        }
found:
    const int planes = d * (d - 1) / 2;
    uint64_t mask = 0;
    int row = site;
    for (int j = 0; j < b; ++j) {
        int s = row;
        for (int i = 0; i < a; ++i) {
            mask ^= lat.plaq_mask[(size_t)s * planes + plane];
            s = lat.fwd[s * d + mu];
        }
        row = lat.fwd[row * d + nu];
    }
    return mask;
}

// The three contours of Sec. 3.1, c1, c2, c3, with perimeters 4 : 6 : 8 and enclosed areas
// 1 : 2 : 3, each the boundary of a chain of k plaquettes from site 0 (the product of the
// plaquettes).  2D: one plaquette, two side by side along x, then one more on top of the
// second (an L).  3D, where a planar 1 x 2 block wraps around an extent of 2: the xy
// plaquette, the xz plaquette sharing its x link, then the xy plaquette one step up in z
// (a bent strip).  Returns 0 where the chain's boundary is not a loop of 2k + 2 links (a
// block that wraps, e.g. c2 on a 2 x L torus).
uint64_t contour_mask(const Lattice &lat, int k)
{
    const int d = lat.d, planes = d * (d - 1) / 2;
    auto plaq = [&](int s, int plane) { return lat.plaq_mask[(size_t)s * planes + plane]; };
    uint64_t m = 0;
    if (d == 2) {
        const int s1 = lat.fwd[0 * d + 0], s2 = lat.fwd[s1 * d + 1];
        const int chain[3] = {0, s1, s2};
        for (int i = 0; i < k; ++i) m ^= plaq(chain[i], 0);
    } else {
        // planes of a 3D site: 0 = (x, y), 1 = (x, z), 2 = (y, z)
        const int up = lat.fwd[0 * d + 2];
        const int site[3] = {0, 0, up}, plane[3] = {0, 1, 0};
        for (int i = 0; i < k; ++i) m ^= plaq(site[i], plane[i]);
    }
    return __builtin_popcountll(m) == 2 * k + 2 ? m : 0;
}

uint64_t line_mask(const Lattice &lat, int site, int mu)
{
    uint64_t m = 0;
    int s = site;
    for (int k = 0; k < lat.L[mu]; ++k) {
        m |= 1ull << lat.link(s, mu);
        s = lat.fwd[s * lat.d + mu];
    }
    return m;
}

uint64_t thooft_mask(const Lattice &lat, int mu)
{
    // the mu-links of the sites on the plane x_mu = 0: every link that pierces the closed
    // dual surface between the planes x_mu = 0 and x_mu = 1
    int stride = 1;
    for (int nu = 0; nu < mu; ++nu) stride *= lat.L[nu];
    uint64_t m = 0;
    for (int s = 0; s < lat.n_sites; ++s)
        if ((s / stride) % lat.L[mu] == 0) m |= 1ull << lat.link(s, mu);
    return m;
}

void build_parity_tables(const Lattice &lat, uint32_t tab[kParityBytes][256])
{
    for (int k = 0; k < kParityBytes; ++k)
        for (int v = 0; v < 256; ++v) {
            uint32_t acc = 0;
            for (int i = 0; i < 8; ++i) {
                int q = 8 * k + i;
                if ((v >> i) & 1 && q < lat.n_links) acc ^= lat.link_plaqs[q];
            }
            tab[k][v] = acc;
        }
}

}  // namespace lgt
