// Per-mesh precompute on the host (once per mesh, outside the stepped path):
// orientation, edge table, geometry and the optimal convex decomposition.
//
//  - Notation of Sec. 2 (Fig. MeshK): vertices counter-clockwise, local edge i is
//    opposite local vertex i; it runs from vertex i+1 to vertex i+2, so a shared
//    edge is traversed in opposite directions by its two cells.
//  - Affine map x - x_1 = J_K (xi, eta) (below eq. basisfunc); J^{-1} is stored.
//  - Decomposition (Sec. 4.3): edges sorted by decreasing length (stable),
//    P1 limiter points are the vertices opposite the two longest edges
//    (eq. 1944), P2 internal nodes have barycentric coordinates beta_{s,i} of
//    eq. 1139 with lhat of eq. 1703; C^DCW_{K,1} = 2/(3(l1+l2)) (eq. 1692),
//    C^DCW_{K,2} = 2/(9 lbar + 3 lhat) (eq. 1713).
//
// Compiled with -ffp-contract=off so lengths and the stable sort are reproducible.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "oedg.h"
#include "oedg_internal.h"

namespace oedg {

namespace {

struct HalfEdge {
    uint64_t key;   // (min vertex id << 32) | max vertex id
    int32_t cell;
    int32_t edge;
};

// Which cell of each interior edge inside a tile does the filter's edge work (the
// "owner"; the other one receives its share through the tile's LDS).  A cell owns
// every edge to a neighbour outside the tile, and the in-tile edges are oriented so
// that a cell owns at most two edges where the forced ones allow it (the lanes of a
// wave then run two rounds of edge work instead of three) and at most two in-tile
// edges in any case (what a lane keeps in registers for its partners).  Start: the
// lower index owns; then, while a cell is over a bound, reverse a shortest path of
// owned in-tile edges from it to a cell under the bound (one edge less at the start,
// one more at the end, the same in between).  Every subgraph of a mesh of triangles
// has at most 3/2 edges per cell, so two per cell is always reachable for the in-tile
// edges (Hakimi's orientation theorem).  own[3 * (c - c0) + i] = 1 when cell c owns
// its local edge i (i an in-tile edge); deterministic for a given mesh.
void orient_tile(const std::vector<int32_t>& nbr, size_t c0, size_t c1, std::vector<uint8_t>& own) {
    const size_t n = c1 - c0;
    own.assign(3 * n, 0);
    std::vector<int> out(n, 0), in_tile(n, 0);
    auto inside = [&](int32_t x) { return x >= 0 && (size_t)x >= c0 && (size_t)x < c1; };
    for (size_t c = 0; c < n; ++c)
        for (int i = 0; i < 3; ++i) {
            const int32_t x = nbr[3 * (c0 + c) + i];
            if (x < 0) continue;
            if (!inside(x)) {
                ++out[c];
            } else if (c0 + c < (size_t)x) {
                own[3 * c + i] = 1;
                ++out[c];
                ++in_tile[c];
            }
        }
    std::vector<int> prev_cell(n), prev_edge(n), queue;
    std::vector<char> seen(n);
    // cnt: the count to bring down to `cap`
    auto reduce = [&](std::vector<int>& cnt, int cap) {
        for (size_t s = 0; s < n; ++s) {
            while (cnt[s] > cap) {
                std::fill(seen.begin(), seen.end(), 0);
                queue.assign(1, (int)s);
                seen[s] = 1;
                int found = -1;
                for (size_t q = 0; q < queue.size() && found < 0; ++q) {
                    const int u = queue[q];
                    for (int i = 0; i < 3 && found < 0; ++i) {
                        if (!own[3 * u + i]) continue;
                        const int v = nbr[3 * (c0 + u) + i] - (int)c0;
                        if (seen[v]) continue;
                        seen[v] = 1;
                        prev_cell[v] = u;
                        prev_edge[v] = i;
                        queue.push_back(v);
                        if (cnt[v] < cap) found = v;
                    }
                }
                if (found < 0) break;
                for (int v = found; v != (int)s;) {
                    const int u = prev_cell[v], i = prev_edge[v];
                    own[3 * u + i] = 0;
                    for (int j = 0; j < 3; ++j)
                        if (nbr[3 * (c0 + v) + j] == (int32_t)(c0 + u)) own[3 * v + j] = 1;
                    v = u;
                }
                --out[s];
                --in_tile[s];
                ++out[found];
                ++in_tile[found];
            }
        }
    };
    reduce(out, 2);
    reduce(in_tile, 2);
}

// barycentric coordinates of the two P2 internal nodes, in the sorted labelling
void p2_nodes(double l1, double l2, double l3, double beta[2][3], double* cdcw) {
    const double s3 = std::sqrt(3.0);
    const double lb = (l1 + l2 + l3) / 3.0;
    const double lh = std::sqrt(l1 * l1 + l2 * l2 + l3 * l3 - 2.0 / 3.0 * (l1 * l2 + l2 * l3 + l3 * l1));
    // M_{s,i} (symmetric) and c_{s,i}, eq. 1139
    const double M[2][3][6] = {
        // entries (11, 22, 33, 12, 13, 23)
        {{6, 2 * s3 + 6, 6, 1, -2, -s3 - 2},
         {6, 12, 6, -s3 - 2, -2, s3 - 2},
         {6, 6 - 2 * s3, 6, s3 - 2, -2, 1}},
        {{6, 6 - 2 * s3, 6, 1, -2, s3 - 2},
         {6, 12, 6, s3 - 2, -2, -s3 - 2},
         {6, 2 * s3 + 6, 6, -s3 - 2, -2, 1}}};
    const double c[2][3] = {{3 * l1 + 3 * l2 + s3 * (l2 - l3), 6 * l2 + s3 * (l3 - l1), 3 * l2 + 3 * l3 + s3 * (l1 - l2)},
                            {3 * l1 + 3 * l2 + s3 * (l3 - l2), 6 * l2 + s3 * (l1 - l3), 3 * l2 + 3 * l3 + s3 * (l2 - l1)}};
    const double den = 18.0 * (lb + lh) * (l2 + lh);
    for (int s = 0; s < 2; ++s)
        for (int i = 0; i < 3; ++i) {
            const double* m = M[s][i];
            const double q = m[0] * l1 * l1 + m[1] * l2 * l2 + m[2] * l3 * l3 +
                             2.0 * (m[3] * l1 * l2 + m[4] * l1 * l3 + m[5] * l2 * l3);
            beta[s][i] = (q + 2.0 * c[s][i] * lh) / den;
        }
    *cdcw = 2.0 / (9.0 * lb + 3.0 * lh);
}

}  // namespace

int build_mesh(int k, int32_t n_vert, const double* xy, int32_t n_cell, const int32_t* tri_in,
               const double* cell_xy, const int32_t* edge_bc, HostMesh& m, std::string& err) {
    if (n_cell <= 0 || n_vert <= 0) { err = "mesh has no cells or no vertices"; return -2; }
    m.n_cell = n_cell;
    m.k = k;
    const size_t nc = static_cast<size_t>(n_cell);
    m.tri.assign(3 * nc, 0);
    m.nbr.assign(3 * nc, -1);
    m.nbe.assign(3 * nc, -1);
    m.perm.assign(3 * nc, 0);
    m.jinv.assign(4 * nc, 0.0);
    m.area.assign(nc, 0.0);
    m.len.assign(3 * nc, 0.0);
    m.node_ref.assign(4 * nc, 0.0);
    m.ck.assign(nc, 0.0);
    m.ck_zxs.assign(nc, 0.0);
    std::vector<unsigned char> swapped(nc, 0);
    m.link.assign(3 * nc, -1);
    m.vx.assign(6 * nc, 0.0);
    std::vector<double> vx(6 * nc);

    for (size_t c = 0; c < nc; ++c) {
        int32_t id[3];
        double p[6];
        for (int q = 0; q < 3; ++q) {
            id[q] = tri_in[3 * c + q];
            if (id[q] < 0 || id[q] >= n_vert) { err = "vertex id out of range"; return -2; }
            if (cell_xy) {
                p[2 * q] = cell_xy[6 * c + 2 * q];
                p[2 * q + 1] = cell_xy[6 * c + 2 * q + 1];
            } else {
                p[2 * q] = xy[2 * static_cast<size_t>(id[q])];
                p[2 * q + 1] = xy[2 * static_cast<size_t>(id[q]) + 1];
            }
        }
        const double twice_area = (p[2] - p[0]) * (p[5] - p[1]) - (p[4] - p[0]) * (p[3] - p[1]);
        if (!(twice_area != 0.0) || !std::isfinite(twice_area)) { err = "degenerate cell"; return -2; }
        if (twice_area < 0) {
            swapped[c] = 1;
            std::swap(id[1], id[2]);
            std::swap(p[2], p[4]);
            std::swap(p[3], p[5]);
        }
        for (int q = 0; q < 3; ++q) m.tri[3 * c + q] = id[q];
        std::memcpy(&vx[6 * c], p, sizeof(p));
        for (int q = 0; q < 6; ++q) m.vx[q * nc + c] = p[q];
    }

    // edge table: sort half-edges by their unordered vertex pair
    std::vector<unsigned char> wall(3 * nc, 0);
    std::vector<HalfEdge> he(3 * nc);
    for (size_t c = 0; c < nc; ++c)
        for (int i = 0; i < 3; ++i) {
            const uint32_t a = static_cast<uint32_t>(m.tri[3 * c + (i + 1) % 3]);
            const uint32_t b = static_cast<uint32_t>(m.tri[3 * c + (i + 2) % 3]);
            const uint64_t lo = std::min(a, b), hi = std::max(a, b);
            he[3 * c + i] = HalfEdge{(lo << 32) | hi, static_cast<int32_t>(c), i};
        }
    std::sort(he.begin(), he.end(), [](const HalfEdge& x, const HalfEdge& y) {
        if (x.key != y.key) return x.key < y.key;
        return x.cell != y.cell ? x.cell < y.cell : x.edge < y.edge;
    });
    for (size_t r = 0; r < he.size();) {
        size_t s = r + 1;
        while (s < he.size() && he[s].key == he[r].key) ++s;
        if (s - r > 2) { err = "edge shared by more than two cells"; return -2; }
        if (s - r == 2) {
            const HalfEdge& x = he[r];
            const HalfEdge& y = he[r + 1];
            if (x.cell == y.cell) { err = "cell adjacent to itself"; return -2; }
            m.nbr[3 * x.cell + x.edge] = y.cell;
            m.nbe[3 * x.cell + x.edge] = y.edge;
            m.nbr[3 * y.cell + y.edge] = x.cell;
            m.nbe[3 * y.cell + y.edge] = x.edge;
        } else if (edge_bc) {
            // the tag names the edge opposite the input vertex; orienting swapped 1 and 2
            const size_t c = static_cast<size_t>(he[r].cell);
            const int e = he[r].edge, in = swapped[c] && e > 0 ? 3 - e : e;
            const int32_t tag = edge_bc[3 * c + in];
            if (tag != DG_BC_TRANSMISSIVE && tag != DG_BC_REFLECTIVE) {
                err = "unknown boundary tag";
                return -1;
            }
            if (tag == DG_BC_REFLECTIVE) wall[3 * c + e] = 1;
        }
        r = s;
    }
    if (static_cast<uint64_t>(n_cell) * 8 >= (1ull << 30)) { err = "too many cells"; return -1; }
    for (size_t c = 0; c < nc; ++c)
        for (int i = 0; i < 3; ++i) {
            const int32_t nb = m.nbr[3 * c + i];
            m.link[i * nc + c] = nb >= 0 ? (nb << 2) | m.nbe[3 * c + i] : (wall[3 * c + i] ? kLinkWall : kLinkOpen);
        }

    // Halo map of the tiles of kTileCells consecutive cells: the distinct out-of-tile
    // neighbours of each tile, sorted, at most kHaloCap of them (a neighbour beyond the
    // cap is reached in global memory), and every interior edge's link re-expressed
    // as the neighbour's slot in the tile's LDS image (see kLinkGlobal).
    {
        const size_t n_tiles = (nc + kTileCells - 1) / kTileCells;
        m.halo_ptr.assign(n_tiles + 1, 0);
        m.halo_cell.clear();
        m.llink.assign(3 * nc, 0);
        std::vector<int32_t> halo;
        std::vector<uint8_t> own;
        for (size_t t = 0; t < n_tiles; ++t) {
            const size_t c0 = t * kTileCells, c1 = std::min(nc, c0 + kTileCells);
            halo.clear();
            for (size_t c = c0; c < c1; ++c)
                for (int i = 0; i < 3; ++i) {
                    const int32_t nb = m.nbr[3 * c + i];
                    if (nb >= 0 && ((size_t)nb < c0 || (size_t)nb >= c1)) halo.push_back(nb);
                }
            std::sort(halo.begin(), halo.end());
            halo.erase(std::unique(halo.begin(), halo.end()), halo.end());
            if (halo.size() > (size_t)kHaloCap) halo.resize(kHaloCap);
            m.halo_cell.insert(m.halo_cell.end(), halo.begin(), halo.end());
            m.halo_ptr[t + 1] = (int32_t)m.halo_cell.size();
            orient_tile(m.nbr, c0, c1, own);
            for (size_t c = c0; c < c1; ++c)
                for (int i = 0; i < 3; ++i) {
                    const int32_t nb = m.nbr[3 * c + i];
                    int32_t v = m.link[i * nc + c];
                    if (nb >= 0) {
                        const int32_t tag = ((size_t)nb < c ? 0 : 4) | m.nbe[3 * c + i];
                        if ((size_t)nb >= c0 && (size_t)nb < c1) {
                            v = ((int32_t)(nb - c0) << 3) | tag | (own[3 * (c - c0) + i] ? 0 : kLinkRecv);
                        } else {
                            const auto it = std::lower_bound(halo.begin(), halo.end(), nb);
                            if (it != halo.end() && *it == nb)
                                v = ((int32_t)(kTileCells + (it - halo.begin())) << 3) | tag;
                            else
                                v = kLinkGlobal | (nb << 3) | tag;
                        }
                    }
                    m.llink[i * nc + c] = v;
                }
            // every in-tile edge has exactly one owner, and no cell keeps more than two
            // records for partners (the filter's registers)
            for (size_t c = c0; c < c1; ++c) {
                int kept = 0;
                for (int i = 0; i < 3; ++i) {
                    const int32_t nb = m.nbr[3 * c + i];
                    if (nb < 0 || (size_t)nb < c0 || (size_t)nb >= c1) continue;
                    const bool recv = (m.llink[i * nc + c] & kLinkRecv) != 0;
                    const bool recv_nb = (m.llink[m.nbe[3 * c + i] * nc + (size_t)nb] & kLinkRecv) != 0;
                    if (recv == recv_nb) { err = "internal: edge orientation"; return -1; }
                    kept += recv ? 0 : 1;
                }
                if (kept > 2) { err = "internal: edge orientation"; return -1; }
            }
        }
    }

    // geometry and decomposition
    const double ref[3][2] = {{0, 0}, {1, 0}, {0, 1}};
    double minck = INFINITY, minck_zxs = INFINITY;
    for (size_t c = 0; c < nc; ++c) {
        const double* p = &vx[6 * c];
        const double a = p[2] - p[0], b = p[4] - p[0], cc = p[3] - p[1], d = p[5] - p[1];
        const double det = a * d - b * cc;
        m.area[c] = 0.5 * det;
        m.jinv[0 * nc + c] = d / det;     // d xi / dx
        m.jinv[1 * nc + c] = -b / det;    // d xi / dy
        m.jinv[2 * nc + c] = -cc / det;   // d eta / dx
        m.jinv[3 * nc + c] = a / det;     // d eta / dy
        double l[3];
        for (int i = 0; i < 3; ++i) {
            const double* s = p + 2 * ((i + 1) % 3);
            const double* e = p + 2 * ((i + 2) % 3);
            const double dx = e[0] - s[0], dy = e[1] - s[1];
            l[i] = std::sqrt(dx * dx + dy * dy);
            m.len[i * nc + c] = l[i];
        }
        int o[3] = {0, 1, 2};
        std::stable_sort(o, o + 3, [&](int x, int y) { return l[x] > l[y]; });
        for (int i = 0; i < 3; ++i) m.perm[3 * c + i] = o[i];
        double cd;
        if (k == 1) {
            cd = 2.0 / (3.0 * (l[o[0]] + l[o[1]]));
            for (int s = 0; s < 2; ++s) {
                m.node_ref[(2 * s) * nc + c] = ref[o[s]][0];
                m.node_ref[(2 * s + 1) * nc + c] = ref[o[s]][1];
            }
        } else {
            double beta[2][3];
            p2_nodes(l[o[0]], l[o[1]], l[o[2]], beta, &cd);
            for (int s = 0; s < 2; ++s) {
                double xi = 0, eta = 0;
                for (int i = 0; i < 3; ++i) {   // sorted vertex i is local vertex o[i]
                    xi += beta[s][i] * ref[o[i]][0];
                    eta += beta[s][i] * ref[o[i]][1];
                }
                m.node_ref[(2 * s) * nc + c] = xi;
                m.node_ref[(2 * s + 1) * nc + c] = eta;
            }
        }
        m.ck[c] = cd * m.area[c];
        minck = std::min(minck, m.ck[c]);
        // classical decomposition: 1/(9 lbar) (P1), 1/(27 lbar) (P2), lbar the mean edge length
        const double lbar = (l[0] + l[1] + l[2]) / 3.0;
        m.ck_zxs[c] = m.area[c] / ((k == 1 ? 9.0 : 27.0) * lbar);
        minck_zxs = std::min(minck_zxs, m.ck_zxs[c]);
        m.area_sum += m.area[c];
    }
    m.minck = minck;
    m.minck_zxs = minck_zxs;
    return 0;
}

}  // namespace oedg
