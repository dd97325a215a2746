// Host mesh construction: uniform grids and adaptively refined quad/octrees with 2:1
// balance and hanging-node constraints; node-graph sparsity in SELL-C layout and the
// node-centric assembly tables.
#include "mesh.h"

#include <algorithm>
#include <array>
#include <cmath>
#include <string>
#include <unordered_set>

#include "common.h"

namespace fr {
namespace {

struct Leaf {
    int level;
    int64_t o[3];   // lower corner in finest-lattice units
};

struct LeafKey {
    size_t operator()(const std::pair<int, std::array<int64_t, 3>>& k) const {
        uint64_t h = 1469598103934665603ull ^ static_cast<uint64_t>(k.first);
        for (int i = 0; i < 3; ++i) h = (h ^ static_cast<uint64_t>(k.second[i])) * 1099511628211ull;
        return static_cast<size_t>(h);
    }
};

using LeafSet = std::unordered_set<std::pair<int, std::array<int64_t, 3>>, LeafKey>;

// Distance from the box [a, b] to the crack (segment in 2d, disk in 3d).
double crack_distance(const fr_mesh_desc& d, const double* a, const double* b) {
    const double* c = d.crack_center;
    const double l = d.crack_half_len;
    if (d.dim == 2) {
        double dx = std::max(0.0, std::max((c[0] - l) - b[0], a[0] - (c[0] + l)));
        double dy = std::max(0.0, std::max(c[1] - b[1], a[1] - c[1]));
        return std::sqrt(dx * dx + dy * dy);
    }
    double px = std::min(std::max(c[0], a[0]), b[0]);
    double py = std::min(std::max(c[1], a[1]), b[1]);
    double rxy = std::sqrt((px - c[0]) * (px - c[0]) + (py - c[1]) * (py - c[1]));
    double dxy = std::max(0.0, rxy - l);
    double dz = std::max(0.0, std::max(c[2] - b[2], a[2] - c[2]));
    return std::sqrt(dxy * dxy + dz * dz);
}

}  // namespace

static void validate(const fr_mesh_desc& d) {
    if (d.dim != 2 && d.dim != 3) fail(FR_EINVAL, "mesh: dim must be 2 or 3");
    if (d.levels < 0 || d.levels > 12) fail(FR_EINVAL, "mesh: levels must be in [0, 12]");
    double h0 = 0;
    for (int k = 0; k < d.dim; ++k) {
        if (d.base[k] < 1) fail(FR_EINVAL, "mesh: base cells per axis must be >= 1");
        if (!(d.hi[k] > d.lo[k])) fail(FR_EINVAL, "mesh: need hi > lo on every axis");
        double h = (d.hi[k] - d.lo[k]) / d.base[k];
        if (k == 0) h0 = h;
        else if (std::fabs(h - h0) > 1e-12 * h0) fail(FR_EINVAL, "mesh: cells must be cubes (equal edge on all axes)");
    }
    int64_t cells = 1;
    for (int k = 0; k < d.dim; ++k) cells *= d.base[k];
    if (cells > (int64_t(1) << 30)) fail(FR_EINVAL, "mesh: too many base cells");
    if (d.levels > 0 && !(d.refine_radius >= 0)) fail(FR_EINVAL, "mesh: refine_radius must be >= 0");
}

HostMesh build_mesh(const fr_mesh_desc& d) {
    validate(d);
    HostMesh m;
    const int dim = d.dim;
    m.dim = dim;
    m.nv = 1 << dim;
    for (int k = 0; k < 3; ++k) { m.lo[k] = d.lo[k]; m.hi[k] = d.hi[k]; }
    const int L = d.levels;
    const int64_t S = int64_t(1) << L;                 // lattice units per base cell
    const double h_base = (d.hi[0] - d.lo[0]) / d.base[0];
    m.h_min = h_base / double(S);
    int64_t ext[3] = {1, 1, 1};                         // lattice extent (points per axis - 1)
    for (int k = 0; k < dim; ++k) ext[k] = int64_t(d.base[k]) * S;

    // ---- leaves ---------------------------------------------------------------------
    std::vector<Leaf> leaves;
    if (L == 0) {
        int64_t n0 = d.base[0], n1 = d.base[1], n2 = dim == 3 ? d.base[2] : 1;
        leaves.reserve(size_t(n0 * n1 * n2));
        for (int64_t k = 0; k < n2; ++k)
            for (int64_t j = 0; j < n1; ++j)
                for (int64_t i = 0; i < n0; ++i) leaves.push_back(Leaf{0, {i, j, k}});
    } else {
        // refine towards the crack
        LeafSet set;
        std::vector<Leaf> work;
        int64_t n0 = d.base[0], n1 = d.base[1], n2 = dim == 3 ? d.base[2] : 1;
        for (int64_t k = 0; k < n2; ++k)
            for (int64_t j = 0; j < n1; ++j)
                for (int64_t i = 0; i < n0; ++i) work.push_back(Leaf{0, {i * S, j * S, k * S}});
        auto box = [&](const Leaf& c, double* a, double* b) {
            int64_t s = S >> c.level;
            for (int q = 0; q < dim; ++q) {
                a[q] = d.lo[q] + double(c.o[q]) * m.h_min;
                b[q] = d.lo[q] + double(c.o[q] + s) * m.h_min;
            }
        };
        std::vector<Leaf> out;
        while (!work.empty()) {
            Leaf c = work.back();
            work.pop_back();
            double a[3], b[3];
            box(c, a, b);
            if (c.level < L && crack_distance(d, a, b) <= d.refine_radius) {
                int64_t s = (S >> c.level) / 2;
                for (int ch = 0; ch < (1 << dim); ++ch) {
                    Leaf n{c.level + 1, {c.o[0], c.o[1], c.o[2]}};
                    for (int q = 0; q < dim; ++q) n.o[q] += ((ch >> q) & 1) * s;
                    work.push_back(n);
                }
            } else {
                out.push_back(c);
            }
        }
        for (auto& c : out) set.insert({c.level, {c.o[0], c.o[1], c.o[2]}});
        // 2:1 balance across faces, edges and corners
        auto find_leaf = [&](const int64_t* q, int max_level, int& lev, std::array<int64_t, 3>& org) -> bool {
            for (int l = 0; l <= max_level; ++l) {
                int64_t s = S >> l;
                std::array<int64_t, 3> o{0, 0, 0};
                for (int k = 0; k < dim; ++k) o[k] = (q[k] / s) * s;
                if (set.count({l, o})) { lev = l; org = o; return true; }
            }
            return false;
        };
        bool changed = true;
        while (changed) {
            changed = false;
            std::vector<std::pair<int, std::array<int64_t, 3>>> to_split;
            for (const auto& e : set) {
                int lev = e.first;
                if (lev < 2) continue;
                int64_t s = S >> lev;
                int nd = 1;
                for (int k = 0; k < dim; ++k) nd *= 3;
                for (int dir = 0; dir < nd; ++dir) {
                    int t = dir;
                    int64_t q[3] = {0, 0, 0};
                    bool self = true, inside = true;
                    for (int k = 0; k < dim; ++k) {
                        int o = t % 3 - 1;
                        t /= 3;
                        if (o != 0) self = false;
                        // a lattice point strictly inside the neighbouring cell of the same size
                        q[k] = e.second[k] + o * s + s / 2;
                        if (s == 1) q[k] = e.second[k] + o * s;   // finest: use its corner
                        if (q[k] < 0 || q[k] >= ext[k]) inside = false;
                    }
                    if (self || !inside) continue;
                    int nl;
                    std::array<int64_t, 3> no;
                    if (find_leaf(q, lev, nl, no) && nl < lev - 1) to_split.push_back({nl, no});
                }
            }
            std::sort(to_split.begin(), to_split.end());
            to_split.erase(std::unique(to_split.begin(), to_split.end()), to_split.end());
            for (auto& c : to_split) {
                if (!set.erase(c)) continue;
                int64_t s = (S >> c.first) / 2;
                for (int ch = 0; ch < (1 << dim); ++ch) {
                    std::array<int64_t, 3> o = c.second;
                    for (int q = 0; q < dim; ++q) o[q] += ((ch >> q) & 1) * s;
                    set.insert({c.first + 1, o});
                }
                changed = true;
            }
        }
        leaves.reserve(set.size());
        for (auto& e : set) leaves.push_back(Leaf{e.first, {e.second[0], e.second[1], e.second[2]}});
        // deterministic cell order: by lower corner (z, y, x), then level
        std::sort(leaves.begin(), leaves.end(), [&](const Leaf& a, const Leaf& b) {
            for (int k = dim - 1; k >= 0; --k)
                if (a.o[k] != b.o[k]) return a.o[k] < b.o[k];
            return a.level < b.level;
        });
    }

    // ---- nodes and cells ------------------------------------------------------------
    const int nv = m.nv;
    m.n_cells = int64_t(leaves.size());
    m.cells.resize(size_t(m.n_cells) * nv);
    m.cell_lo.resize(size_t(m.n_cells) * dim);
    m.cell_h.resize(size_t(m.n_cells));
    const int64_t P0 = ext[0] + 1, P1 = ext[1] + 1;
    auto key_of = [&](const int64_t* q) -> int64_t { return q[0] + P0 * (q[1] + P1 * (dim == 3 ? q[2] : 0)); };

    if (L == 0) {
        // uniform: lexicographic nodes, x fastest
        int64_t np[3] = {ext[0] + 1, ext[1] + 1, dim == 3 ? ext[2] + 1 : 1};
        m.n_nodes = np[0] * np[1] * np[2];
        m.coords.resize(size_t(m.n_nodes) * dim);
        m.lattice.resize(size_t(m.n_nodes) * dim);
        for (int64_t k = 0; k < np[2]; ++k)
            for (int64_t j = 0; j < np[1]; ++j)
                for (int64_t i = 0; i < np[0]; ++i) {
                    int64_t n = i + np[0] * (j + np[1] * k);
                    int64_t q[3] = {i, j, k};
                    for (int c = 0; c < dim; ++c) {
                        m.lattice[n * dim + c] = q[c];
                        m.coords[n * dim + c] = d.lo[c] + double(q[c]) * m.h_min;
                    }
                }
        for (int64_t c = 0; c < m.n_cells; ++c) {
            const Leaf& lf = leaves[size_t(c)];
            for (int a = 0; a < nv; ++a) {
                int64_t q[3] = {lf.o[0], lf.o[1], lf.o[2]};
                for (int k = 0; k < dim; ++k) q[k] += (a >> k) & 1;
                m.cells[size_t(c) * nv + a] = int32_t(key_of(q));
            }
            for (int k = 0; k < dim; ++k) m.cell_lo[size_t(c) * dim + k] = d.lo[k] + double(lf.o[k]) * m.h_min;
            m.cell_h[size_t(c)] = m.h_min;
        }
    } else {
        std::vector<int64_t> keys;
        keys.reserve(size_t(m.n_cells) * nv);
        for (const Leaf& lf : leaves) {
            int64_t s = S >> lf.level;
            for (int a = 0; a < nv; ++a) {
                int64_t q[3] = {lf.o[0], lf.o[1], lf.o[2]};
                for (int k = 0; k < dim; ++k) q[k] += ((a >> k) & 1) * s;
                keys.push_back(key_of(q));
            }
        }
        std::vector<int64_t> uk(keys);
        std::sort(uk.begin(), uk.end());
        uk.erase(std::unique(uk.begin(), uk.end()), uk.end());
        m.n_nodes = int64_t(uk.size());
        if (m.n_nodes >= (int64_t(1) << 31)) fail(FR_EINVAL, "mesh: too many nodes");
        m.coords.resize(size_t(m.n_nodes) * dim);
        m.lattice.resize(size_t(m.n_nodes) * dim);
        for (int64_t n = 0; n < m.n_nodes; ++n) {
            int64_t k = uk[size_t(n)];
            int64_t q[3] = {k % P0, (k / P0) % P1, k / (P0 * P1)};
            for (int c = 0; c < dim; ++c) {
                m.lattice[n * dim + c] = q[c];
                m.coords[n * dim + c] = d.lo[c] + double(q[c]) * m.h_min;
            }
        }
        auto node_of = [&](int64_t key) -> int64_t {
            auto it = std::lower_bound(uk.begin(), uk.end(), key);
            if (it == uk.end() || *it != key) return -1;
            return int64_t(it - uk.begin());
        };
        for (int64_t c = 0; c < m.n_cells; ++c) {
            const Leaf& lf = leaves[size_t(c)];
            for (int a = 0; a < nv; ++a) m.cells[size_t(c) * nv + a] = int32_t(node_of(keys[size_t(c) * nv + a]));
            for (int k = 0; k < dim; ++k) m.cell_lo[size_t(c) * dim + k] = d.lo[k] + double(lf.o[k]) * m.h_min;
            m.cell_h[size_t(c)] = m.h_min * double(S >> lf.level);
        }
        // hanging nodes: edge midpoints (weights 1/2) and 3d face centres (weights 1/4) of
        // cells that are nodes of finer neighbours
        std::vector<std::vector<std::pair<int64_t, double>>> hang(size_t(m.n_nodes));
        std::vector<uint8_t> is_hang(size_t(m.n_nodes), 0);
        for (int64_t c = 0; c < m.n_cells; ++c) {
            const Leaf& lf = leaves[size_t(c)];
            int64_t s = S >> lf.level;
            if (s < 2) continue;
            const int32_t* cv = &m.cells[size_t(c) * nv];
            // edges: vertex pairs differing in one bit
            for (int a = 0; a < nv; ++a)
                for (int k = 0; k < dim; ++k) {
                    if ((a >> k) & 1) continue;
                    int b = a | (1 << k);
                    int64_t q[3] = {lf.o[0], lf.o[1], lf.o[2]};
                    for (int t = 0; t < dim; ++t) q[t] += ((a >> t) & 1) * s;
                    q[k] += s / 2;
                    int64_t n = node_of(key_of(q));
                    if (n >= 0 && !is_hang[size_t(n)]) {
                        is_hang[size_t(n)] = 1;
                        hang[size_t(n)] = {{cv[a], 0.5}, {cv[b], 0.5}};
                    }
                }
            if (dim == 3) {
                for (int k = 0; k < 3; ++k)
                    for (int side = 0; side < 2; ++side) {
                        int64_t q[3] = {lf.o[0] + s / 2, lf.o[1] + s / 2, lf.o[2] + s / 2};
                        q[k] = lf.o[k] + side * s;
                        int64_t n = node_of(key_of(q));
                        if (n >= 0 && !is_hang[size_t(n)]) {
                            is_hang[size_t(n)] = 1;
                            std::vector<std::pair<int64_t, double>> ms;
                            for (int a = 0; a < nv; ++a)
                                if (((a >> k) & 1) == side) ms.push_back({cv[a], 0.25});
                            hang[size_t(n)] = ms;
                        }
                    }
            }
        }
        // resolve chains (a master that is itself hanging)
        for (int64_t n = 0; n < m.n_nodes; ++n) {
            if (!is_hang[size_t(n)]) continue;
            for (int guard = 0; guard < 8; ++guard) {
                bool again = false;
                std::vector<std::pair<int64_t, double>> nx;
                for (auto& mw : hang[size_t(n)]) {
                    if (is_hang[size_t(mw.first)]) {
                        again = true;
                        for (auto& m2 : hang[size_t(mw.first)]) nx.push_back({m2.first, mw.second * m2.second});
                    } else {
                        nx.push_back(mw);
                    }
                }
                std::sort(nx.begin(), nx.end());
                std::vector<std::pair<int64_t, double>> mg;
                for (auto& e : nx) {
                    if (!mg.empty() && mg.back().first == e.first) mg.back().second += e.second;
                    else mg.push_back(e);
                }
                hang[size_t(n)] = mg;
                if (!again) break;
            }
        }
        m.free_of_node.assign(size_t(m.n_nodes), -1);
        for (int64_t n = 0; n < m.n_nodes; ++n)
            if (!is_hang[size_t(n)]) {
                m.free_of_node[size_t(n)] = int32_t(m.node_of_free.size());
                m.node_of_free.push_back(int32_t(n));
            }
        m.n_free = int64_t(m.node_of_free.size());
        m.n_hanging = m.n_nodes - m.n_free;
        m.con_ptr.assign(size_t(m.n_nodes) + 1, 0);
        for (int64_t n = 0; n < m.n_nodes; ++n) {
            if (is_hang[size_t(n)]) {
                for (auto& mw : hang[size_t(n)]) {
                    m.con_master.push_back(m.free_of_node[size_t(mw.first)]);
                    m.con_w.push_back(mw.second);
                }
            } else {
                m.con_master.push_back(m.free_of_node[size_t(n)]);
                m.con_w.push_back(1.0);
            }
            m.con_ptr[size_t(n) + 1] = int32_t(m.con_master.size());
        }
    }
    if (L == 0) {
        m.n_free = m.n_nodes;
        m.n_hanging = 0;
        m.free_of_node.resize(size_t(m.n_nodes));
        m.node_of_free.resize(size_t(m.n_nodes));
        m.con_ptr.resize(size_t(m.n_nodes) + 1);
        m.con_master.resize(size_t(m.n_nodes));
        m.con_w.assign(size_t(m.n_nodes), 1.0);
        for (int64_t n = 0; n < m.n_nodes; ++n) {
            m.free_of_node[size_t(n)] = int32_t(n);
            m.node_of_free[size_t(n)] = int32_t(n);
            m.con_ptr[size_t(n)] = int32_t(n);
            m.con_master[size_t(n)] = int32_t(n);
        }
        m.con_ptr[size_t(m.n_nodes)] = int32_t(m.n_nodes);
    }
    m.dirichlet.resize(size_t(m.n_nodes));
    for (int64_t n = 0; n < m.n_nodes; ++n) {
        bool b = false;
        for (int k = 0; k < dim; ++k) {
            int64_t q = m.lattice[n * dim + k];
            if (q == 0 || q == ext[k]) b = true;
        }
        m.dirichlet[size_t(n)] = b ? 1 : 0;
    }
    return m;
}

HostMesh build_mesh_batch(const fr_mesh_desc* d, int n) {
    if (n < 1) fail(FR_EINVAL, "mesh: need at least one instance");
    if (n == 1) {
        HostMesh m = build_mesh(d[0]);
        m.node_off = {0, m.n_nodes};
        m.cell_off = {0, m.n_cells};
        m.free_off = {0, m.n_free};
        m.inst_h_min = {m.h_min};
        return m;
    }
    HostMesh u;
    u.dim = d[0].dim;
    u.nv = 1 << u.dim;
    u.n_inst = n;
    u.node_off.assign(size_t(n) + 1, 0);
    u.cell_off.assign(size_t(n) + 1, 0);
    u.free_off.assign(size_t(n) + 1, 0);
    u.h_min = 1e300;
    u.con_ptr.push_back(0);
    for (int i = 0; i < n; ++i) {
        if (d[i].dim != u.dim) fail(FR_EINVAL, "mesh: all instances of a batch must have the same dim");
        HostMesh m = build_mesh(d[i]);
        const int64_t no = u.n_nodes, fo = u.n_free;
        if (no + m.n_nodes >= (int64_t(1) << 31)) fail(FR_EINVAL, "mesh: batch has too many nodes");
        u.coords.insert(u.coords.end(), m.coords.begin(), m.coords.end());
        u.lattice.insert(u.lattice.end(), m.lattice.begin(), m.lattice.end());
        for (int32_t v : m.cells) u.cells.push_back(int32_t(v + no));
        u.cell_lo.insert(u.cell_lo.end(), m.cell_lo.begin(), m.cell_lo.end());
        u.cell_h.insert(u.cell_h.end(), m.cell_h.begin(), m.cell_h.end());
        u.dirichlet.insert(u.dirichlet.end(), m.dirichlet.begin(), m.dirichlet.end());
        for (int32_t f : m.free_of_node) u.free_of_node.push_back(f < 0 ? -1 : int32_t(f + fo));
        for (int32_t v : m.node_of_free) u.node_of_free.push_back(int32_t(v + no));
        const int32_t cbase = u.con_ptr.back();
        for (size_t k = 1; k < m.con_ptr.size(); ++k) u.con_ptr.push_back(cbase + m.con_ptr[k]);
        for (int32_t v : m.con_master) u.con_master.push_back(int32_t(v + fo));
        u.con_w.insert(u.con_w.end(), m.con_w.begin(), m.con_w.end());
        u.n_nodes += m.n_nodes;
        u.n_cells += m.n_cells;
        u.n_free += m.n_free;
        u.n_hanging += m.n_hanging;
        u.h_min = std::min(u.h_min, m.h_min);
        u.inst_h_min.push_back(m.h_min);
        u.node_off[size_t(i) + 1] = u.n_nodes;
        u.cell_off[size_t(i) + 1] = u.n_cells;
        u.free_off[size_t(i) + 1] = u.n_free;
        if (i == 0)
            for (int k = 0; k < 3; ++k) { u.lo[k] = m.lo[k]; u.hi[k] = m.hi[k]; }
    }
    return u;
}

Pattern build_pattern(const HostMesh& m, int C) {
    Pattern p;
    p.C = C;
    const int nv = m.nv;
    const int64_t nn = m.n_nodes, nf = m.n_free;
    p.n_rows = nf;
    // node -> cells adjacency
    std::vector<int32_t> nc_ptr(size_t(nn) + 1, 0);
    for (int64_t c = 0; c < m.n_cells; ++c)
        for (int a = 0; a < nv; ++a) nc_ptr[size_t(m.cells[size_t(c) * nv + a]) + 1]++;
    for (int64_t n = 0; n < nn; ++n) nc_ptr[size_t(n) + 1] += nc_ptr[size_t(n)];
    const size_t n_inc = size_t(nc_ptr[size_t(nn)]);
    std::vector<int32_t> nc_cell(n_inc), nc_a(n_inc);
    {
        std::vector<int32_t> fill(nc_ptr.begin(), nc_ptr.end() - 1);
        for (int64_t c = 0; c < m.n_cells; ++c)
            for (int a = 0; a < nv; ++a) {
                int32_t n = m.cells[size_t(c) * nv + a];
                nc_cell[static_cast<size_t>(fill[size_t(n)])] = int32_t(c);
                nc_a[static_cast<size_t>(fill[size_t(n)]++)] = a;
            }
    }
    // master -> hanging dependents
    std::vector<int32_t> dep_ptr(size_t(nf) + 1, 0);
    std::vector<int32_t> dep_node;
    std::vector<double> dep_w;
    if (m.n_hanging > 0) {
        for (int64_t n = 0; n < nn; ++n)
            if (m.free_of_node[size_t(n)] < 0)
                for (int32_t j = m.con_ptr[size_t(n)]; j < m.con_ptr[size_t(n) + 1]; ++j) dep_ptr[size_t(m.con_master[size_t(j)]) + 1]++;
        for (int64_t f = 0; f < nf; ++f) dep_ptr[size_t(f) + 1] += dep_ptr[size_t(f)];
        dep_node.resize(size_t(dep_ptr[size_t(nf)]));
        dep_w.resize(dep_node.size());
        std::vector<int32_t> fill(dep_ptr.begin(), dep_ptr.end() - 1);
        for (int64_t n = 0; n < nn; ++n)
            if (m.free_of_node[size_t(n)] < 0)
                for (int32_t j = m.con_ptr[size_t(n)]; j < m.con_ptr[size_t(n) + 1]; ++j) {
                    int32_t f = m.con_master[size_t(j)];
                    dep_node[static_cast<size_t>(fill[size_t(f)])] = int32_t(n);
                    dep_w[static_cast<size_t>(fill[size_t(f)]++)] = m.con_w[size_t(j)];
                }
    }
    // per row: entries and sorted unique columns
    std::vector<std::vector<int32_t>> cols(static_cast<size_t>(nf));
    p.ent_ptr.assign(size_t(nf) + 1, 0);
    struct Ent { int32_t cell; uint8_t a; double w; };
    std::vector<Ent> ents;
    std::vector<Ent> tmp;
    std::vector<int32_t> cand;
    int max_row = 0;
    for (int64_t f = 0; f < nf; ++f) {
        tmp.clear();
        int32_t node = m.node_of_free[size_t(f)];
        for (int32_t j = nc_ptr[size_t(node)]; j < nc_ptr[size_t(node) + 1]; ++j)
            tmp.push_back(Ent{nc_cell[size_t(j)], uint8_t(nc_a[size_t(j)]), 1.0});
        if (m.n_hanging > 0)
            for (int32_t j = dep_ptr[size_t(f)]; j < dep_ptr[size_t(f) + 1]; ++j) {
                int32_t h = dep_node[size_t(j)];
                for (int32_t t = nc_ptr[size_t(h)]; t < nc_ptr[size_t(h) + 1]; ++t)
                    tmp.push_back(Ent{nc_cell[size_t(t)], uint8_t(nc_a[size_t(t)]), dep_w[size_t(j)]});
            }
        std::sort(tmp.begin(), tmp.end(), [](const Ent& x, const Ent& y) {
            return x.cell != y.cell ? x.cell < y.cell : x.a < y.a;
        });
        cand.clear();
        for (const Ent& e : tmp) {
            ents.push_back(e);
            for (int b = 0; b < nv; ++b) {
                int32_t n = m.cells[size_t(e.cell) * nv + b];
                for (int32_t t = m.con_ptr[size_t(n)]; t < m.con_ptr[size_t(n) + 1]; ++t) cand.push_back(m.con_master[size_t(t)]);
            }
        }
        std::sort(cand.begin(), cand.end());
        cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
        if (cand.size() > 254) fail(FR_EINTERNAL, "pattern: more than 254 node neighbours in a row");
        max_row = std::max(max_row, int(cand.size()));
        cols[size_t(f)] = cand;
        p.ent_ptr[size_t(f) + 1] = int32_t(ents.size());
    }
    p.max_row = max_row;
    const size_t n_ent = ents.size();
    p.ent_cell.resize(n_ent);
    p.ent_a.resize(n_ent);
    p.ent_w.resize(n_ent);
    p.ent_k.resize(n_ent * size_t(nv));
    for (int64_t f = 0; f < nf; ++f) {
        const auto& cf = cols[size_t(f)];
        for (int32_t e = p.ent_ptr[size_t(f)]; e < p.ent_ptr[size_t(f) + 1]; ++e) {
            const Ent& en = ents[size_t(e)];
            p.ent_cell[size_t(e)] = en.cell;
            p.ent_a[size_t(e)] = en.a;
            p.ent_w[size_t(e)] = en.w;
            for (int b = 0; b < nv; ++b) {
                int32_t n = m.cells[size_t(en.cell) * nv + b];
                int32_t fb = m.free_of_node[size_t(n)];
                uint8_t k = 255;
                if (fb >= 0) k = uint8_t(std::lower_bound(cf.begin(), cf.end(), fb) - cf.begin());
                p.ent_k[size_t(e) * nv + b] = k;
            }
        }
    }
    // SELL-C layout (no row sorting: the node numbering already groups similar rows)
    p.n_slices = ceil_div(nf, C);
    p.slice_ptr.assign(size_t(p.n_slices) + 1, 0);
    p.row_len.resize(size_t(nf));
    int64_t off = 0;
    for (int64_t s = 0; s < p.n_slices; ++s) {
        int w = 0;
        for (int64_t r = s * C; r < std::min<int64_t>(nf, (s + 1) * C); ++r) w = std::max(w, int(cols[size_t(r)].size()));
        p.slice_ptr[size_t(s)] = int32_t(off);
        off += int64_t(w) * C;
        if (off >= (int64_t(1) << 31)) fail(FR_EINTERNAL, "pattern: more than 2^31 slots");
    }
    p.slice_ptr[size_t(p.n_slices)] = int32_t(off);
    p.n_slots = off;
    p.col.assign(size_t(off), 0);
    int64_t nnz = 0;
    for (int64_t r = 0; r < nf; ++r) {
        const auto& cf = cols[size_t(r)];
        int64_t s = r / C, lane = r % C;
        int w = (p.slice_ptr[size_t(s) + 1] - p.slice_ptr[size_t(s)]) / C;
        p.row_len[size_t(r)] = int32_t(cf.size());
        nnz += int64_t(cf.size());
        for (int k = 0; k < w; ++k)
            p.col[size_t(p.slice_ptr[size_t(s)] + int64_t(k) * C + lane)] = k < int(cf.size()) ? cf[size_t(k)] : int32_t(r);
    }
    // slots of padded lanes past the last row point at row 0 (any valid column)
    p.nnz = nnz;
    return p;
}

}  // namespace fr
