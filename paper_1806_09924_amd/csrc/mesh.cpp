// Host mesh construction: uniform grids and adaptively refined quad/octrees with 2:1
// balance and hanging-node constraints; node-graph sparsity in SELL-C layout and the
// node-centric assembly tables.
#include "mesh.h"

#include <algorithm>
#include <array>
#include <cmath>
#include <string>
#include <cstdint>
#include <exception>
#include <thread>

#include "common.h"

namespace fr {
namespace {

struct Leaf {
    int level;
    int64_t o[3];   // lower corner in finest-lattice units
};

// Open-addressing hash set of 64-bit keys (linear probing, load <= 1/2).
class KeySet {
public:
    explicit KeySet(size_t expect = 16) { rehash(std::max<size_t>(16, 2 * expect)); }
    bool insert(uint64_t k) {
        if (2 * (n_ + 1) > tab_.size()) rehash(2 * tab_.size());
        return put(k);
    }
    bool contains(uint64_t k) const {
        for (size_t i = mix(k) & mask_;; i = (i + 1) & mask_) {
            if (tab_[i] == kEmpty) return false;
            if (tab_[i] == k) return true;
        }
    }
    template <typename F>
    void for_each(F f) const {
        for (uint64_t v : tab_)
            if (v != kEmpty) f(v);
    }
    size_t size() const { return n_; }

private:
    static constexpr uint64_t kEmpty = ~uint64_t(0);
    static size_t mix(uint64_t k) {
        k ^= k >> 33;
        k *= 0xff51afd7ed558ccdull;
        k ^= k >> 33;
        return size_t(k);
    }
    bool put(uint64_t k) {
        for (size_t i = mix(k) & mask_;; i = (i + 1) & mask_) {
            if (tab_[i] == kEmpty) {
                tab_[i] = k;
                ++n_;
                return true;
            }
            if (tab_[i] == k) return false;
        }
    }
    void rehash(size_t cap) {
        size_t c = 16;
        while (c < cap) c <<= 1;
        std::vector<uint64_t> old;
        old.swap(tab_);
        tab_.assign(c, kEmpty);
        mask_ = c - 1;
        n_ = 0;
        for (uint64_t v : old)
            if (v != kEmpty) put(v);
    }
    std::vector<uint64_t> tab_;
    size_t mask_ = 0, n_ = 0;
};

// lattice origin (each coordinate < 2^21) packed into one key
inline uint64_t pack(const int64_t* o) {
    return uint64_t(o[0]) | (uint64_t(o[1]) << 21) | (uint64_t(o[2]) << 42);
}
inline void unpack(uint64_t k, int64_t* o) {
    o[0] = int64_t(k & 0x1FFFFF);
    o[1] = int64_t((k >> 21) & 0x1FFFFF);
    o[2] = int64_t((k >> 42) & 0x1FFFFF);
}

// Stable LSD radix sort of (key, value) pairs by key, 16-bit digits, as many passes as the
// largest key needs.
void radix_sort_pairs(std::vector<uint64_t>& key, std::vector<uint32_t>& val) {
    const size_t n = key.size();
    uint64_t mx = 0;
    for (uint64_t k : key) mx = std::max(mx, k);
    int bits = 0;
    while (bits < 64 && (mx >> bits) != 0) ++bits;
    std::vector<uint64_t> k2(n);
    std::vector<uint32_t> v2(n);
    std::vector<size_t> cnt(65537);
    for (int shift = 0; shift < bits; shift += 16) {
        std::fill(cnt.begin(), cnt.end(), 0);
        for (size_t i = 0; i < n; ++i) cnt[((key[i] >> shift) & 0xFFFF) + 1]++;
        for (size_t d = 0; d < 65536; ++d) cnt[d + 1] += cnt[d];
        for (size_t i = 0; i < n; ++i) {
            const size_t pos = cnt[(key[i] >> shift) & 0xFFFF]++;
            k2[pos] = key[i];
            v2[pos] = val[i];
        }
        key.swap(k2);
        val.swap(v2);
    }
}

// Runs f(begin, end, t) over [0, n) split into contiguous chunks, one per host thread.
template <typename F>
void parallel_ranges(int64_t n, F f) {
    const int64_t hw = std::max<int64_t>(1, std::thread::hardware_concurrency());
    const int64_t T = std::max<int64_t>(1, std::min<int64_t>({hw, 16, n / 4096 + 1}));
    std::vector<std::thread> th;
    std::vector<std::exception_ptr> err(static_cast<size_t>(T));
    for (int64_t t = 0; t < T; ++t)
        th.emplace_back([&, t]() {
            try {
                f(n * t / T, n * (t + 1) / T, int(t));
            } catch (...) {
                err[size_t(t)] = std::current_exception();
            }
        });
    for (auto& x : th) x.join();
    for (auto& e : err)
        if (e) std::rethrow_exception(e);
}

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

HostMesh build_mesh(const fr_mesh_desc& d, const RefineSeed* seed) {
    validate(d);
    HostMesh m;
    const int dim = d.dim;
    m.dim = dim;
    m.nv = 1 << dim;
    for (int k = 0; k < 3; ++k) { m.lo[k] = d.lo[k]; m.hi[k] = d.hi[k]; }
    const int L = seed ? seed->L : d.levels;
    if (L < 0 || L > 12) fail(FR_EINVAL, "mesh: levels must be in [0, 12]");
    m.desc = d;
    m.desc.levels = L;
    m.levels = L;
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
        // refined[l]: cells of level l that are split.  First the rule (split while the
        // level is below L and the box is within refine_radius of the crack), then the 2:1
        // closure level by level from the finest: every cell of level l needs the level-(l-1)
        // cell around the centre of each same-size neighbour, so the level-(l-2) cell there
        // is split (with its ancestors).  Cells of level l are never added while level l is
        // scanned, so one sweep from the finest level down is the closure.
        for (int k = 0; k < dim; ++k)
            if (ext[k] >= (int64_t(1) << 21)) fail(FR_EINVAL, "mesh: more than 2^21 finest cells per axis");
        std::vector<KeySet> refined(static_cast<size_t>(L));
        int64_t n0 = d.base[0], n1 = d.base[1], n2 = dim == 3 ? d.base[2] : 1;
        struct Item { int level; int64_t o[3]; };
        std::vector<Item> work;
        if (seed) {
            for (int l = 0; l < L && size_t(l) < seed->split.size(); ++l)
                for (uint64_t k : seed->split[size_t(l)]) refined[size_t(l)].insert(k);
        } else {
            for (int64_t k = 0; k < n2; ++k)
                for (int64_t j = 0; j < n1; ++j)
                    for (int64_t i = 0; i < n0; ++i) work.push_back(Item{0, {i * S, j * S, k * S}});
        }
        while (!work.empty()) {
            Item c = work.back();
            work.pop_back();
            const int64_t s = S >> c.level;
            double a[3] = {0, 0, 0}, b[3] = {0, 0, 0};
            for (int q = 0; q < dim; ++q) {
                a[q] = d.lo[q] + double(c.o[q]) * m.h_min;
                b[q] = d.lo[q] + double(c.o[q] + s) * m.h_min;
            }
            if (c.level < L && crack_distance(d, a, b) <= d.refine_radius) {
                refined[size_t(c.level)].insert(pack(c.o));
                for (int ch = 0; ch < (1 << dim); ++ch) {
                    Item n{c.level + 1, {c.o[0], c.o[1], c.o[2]}};
                    for (int q = 0; q < dim; ++q) n.o[q] += ((ch >> q) & 1) * (s / 2);
                    work.push_back(n);
                }
            }
        }
        // split the level-lv cell containing lattice point q, and its ancestors
        auto split_around = [&](const int64_t* q, int lv) {
            for (int l = lv; l >= 0; --l) {
                const int64_t sz = S >> l;
                int64_t o[3] = {0, 0, 0};
                for (int k = 0; k < dim; ++k) o[k] = (q[k] / sz) * sz;
                if (!refined[size_t(l)].insert(pack(o))) break;
            }
        };
        int nd = 1;
        for (int k = 0; k < dim; ++k) nd *= 3;
        for (int l = L; l >= 2; --l) {
            const int64_t s = S >> l;
            std::vector<uint64_t> parents;
            parents.reserve(refined[size_t(l - 1)].size());
            refined[size_t(l - 1)].for_each([&](uint64_t k) { parents.push_back(k); });
            for (uint64_t pk : parents) {
                int64_t po[3];
                unpack(pk, po);
                for (int ch = 0; ch < (1 << dim); ++ch) {
                    int64_t o[3] = {po[0], po[1], po[2]};
                    for (int q = 0; q < dim; ++q) o[q] += ((ch >> q) & 1) * s;
                    for (int dir = 0; dir < nd; ++dir) {
                        int t = dir;
                        int64_t q[3] = {0, 0, 0};
                        bool self = true, inside = true;
                        for (int k = 0; k < dim; ++k) {
                            const int off = t % 3 - 1;
                            t /= 3;
                            if (off != 0) self = false;
                            q[k] = o[k] + off * s + s / 2;   // inside the same-size neighbour
                            if (q[k] < 0 || q[k] >= ext[k]) inside = false;
                        }
                        if (self || !inside) continue;
                        split_around(q, l - 2);
                    }
                }
            }
        }
        // leaves: the cells of every level that are not split
        for (int64_t k = 0; k < n2; ++k)
            for (int64_t j = 0; j < n1; ++j)
                for (int64_t i = 0; i < n0; ++i) {
                    int64_t o[3] = {i * S, j * S, k * S};
                    if (L == 0 || !refined[0].contains(pack(o))) leaves.push_back(Leaf{0, {o[0], o[1], o[2]}});
                }
        for (int l = 1; l <= L; ++l) {
            const int64_t s = S >> l;
            refined[size_t(l - 1)].for_each([&](uint64_t pk) {
                int64_t po[3];
                unpack(pk, po);
                for (int ch = 0; ch < (1 << dim); ++ch) {
                    int64_t o[3] = {po[0], po[1], po[2]};
                    for (int q = 0; q < dim; ++q) o[q] += ((ch >> q) & 1) * s;
                    if (l == L || !refined[size_t(l)].contains(pack(o))) leaves.push_back(Leaf{l, {o[0], o[1], o[2]}});
                }
            });
        }
        // deterministic cell order: by lower corner (z, y, x).  Leaves do not overlap, so no two
        // share a lower corner, and the packed corner (z in the high bits) orders them.
        {
            std::vector<uint64_t> lk(leaves.size());
            std::vector<uint32_t> li(leaves.size());
            for (size_t i = 0; i < leaves.size(); ++i) {
                lk[i] = pack(leaves[i].o);
                li[i] = uint32_t(i);
            }
            radix_sort_pairs(lk, li);
            for (size_t i = 1; i < lk.size(); ++i)
                if (lk[i] == lk[i - 1]) fail(FR_EINTERNAL, "mesh: two leaves share a lower corner");
            std::vector<Leaf> sorted(leaves.size());
            for (size_t i = 0; i < leaves.size(); ++i) sorted[i] = leaves[li[i]];
            leaves.swap(sorted);
        }
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
        // vertex keys of every cell, sorted with their positions: the distinct keys are the
        // nodes (in key order), and each position learns its node id in the same sweep
        const size_t nk = size_t(m.n_cells) * size_t(nv);
        if (nk >= (size_t(1) << 32)) fail(FR_EINVAL, "mesh: too many cell vertices");
        std::vector<uint64_t> skey(nk);
        std::vector<uint32_t> spos(nk);
        for (int64_t c = 0; c < m.n_cells; ++c) {
            const Leaf& lf = leaves[size_t(c)];
            const int64_t s = S >> lf.level;
            for (int a = 0; a < nv; ++a) {
                int64_t q[3] = {lf.o[0], lf.o[1], lf.o[2]};
                for (int k = 0; k < dim; ++k) q[k] += ((a >> k) & 1) * s;
                skey[size_t(c) * nv + a] = uint64_t(key_of(q));
                spos[size_t(c) * nv + a] = uint32_t(size_t(c) * nv + a);
            }
        }
        radix_sort_pairs(skey, spos);
        std::vector<int64_t> uk;
        uk.reserve(nk / 2 + 1);
        for (size_t i = 0; i < nk; ++i) {
            if (i == 0 || skey[i] != skey[i - 1]) uk.push_back(int64_t(skey[i]));
            m.cells[spos[i]] = int32_t(uk.size() - 1);
        }
        skey = std::vector<uint64_t>();
        spos = std::vector<uint32_t>();
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
            for (int k = 0; k < dim; ++k) m.cell_lo[size_t(c) * dim + k] = d.lo[k] + double(lf.o[k]) * m.h_min;
            m.cell_h[size_t(c)] = m.h_min * double(S >> lf.level);
        }
        // hanging nodes: edge midpoints (weights 1/2) and 3d face centres (weights 1/4) of
        // cells that are nodes of finer neighbours
        std::vector<int32_t> hid(size_t(m.n_nodes), -1);           // node -> entry of `hang`
        std::vector<std::vector<std::pair<int64_t, double>>> hang;
        std::vector<uint8_t> is_hang(size_t(m.n_nodes), 0);
        auto set_hang = [&](int64_t n, std::vector<std::pair<int64_t, double>> ms) {
            is_hang[size_t(n)] = 1;
            hid[size_t(n)] = int32_t(hang.size());
            hang.push_back(std::move(ms));
        };
        // The lookups run on host threads over contiguous cell ranges and list every node found
        // with its masters; the lists are then recorded in cell order, the first cell that names
        // a node giving its masters, exactly as a serial sweep would.
        struct Cand {
            int64_t n;
            int nm;
            int64_t mst[4];
            double w;
        };
        std::vector<std::vector<Cand>> cand(16);
        parallel_ranges(m.n_cells, [&](int64_t cb, int64_t ce, int th) {
            std::vector<Cand>& out = cand[size_t(th)];
            for (int64_t c = cb; c < ce; ++c) {
                const Leaf& lf = leaves[size_t(c)];
                const int64_t s = S >> lf.level;
                if (s < 2) continue;
                const int32_t* cv = &m.cells[size_t(c) * nv];
                // edges: vertex pairs differing in one bit
                for (int a = 0; a < nv; ++a)
                    for (int k = 0; k < dim; ++k) {
                        if ((a >> k) & 1) continue;
                        const int b = a | (1 << k);
                        int64_t q[3] = {lf.o[0], lf.o[1], lf.o[2]};
                        for (int t = 0; t < dim; ++t) q[t] += ((a >> t) & 1) * s;
                        q[k] += s / 2;
                        const int64_t n = node_of(key_of(q));
                        if (n >= 0) out.push_back(Cand{n, 2, {cv[a], cv[b], 0, 0}, 0.5});
                    }
                if (dim == 3) {
                    for (int k = 0; k < 3; ++k)
                        for (int side = 0; side < 2; ++side) {
                            int64_t q[3] = {lf.o[0] + s / 2, lf.o[1] + s / 2, lf.o[2] + s / 2};
                            q[k] = lf.o[k] + side * s;
                            const int64_t n = node_of(key_of(q));
                            if (n < 0) continue;
                            Cand cd{n, 0, {0, 0, 0, 0}, 0.25};
                            for (int a = 0; a < nv; ++a)
                                if (((a >> k) & 1) == side) cd.mst[cd.nm++] = cv[a];
                            out.push_back(cd);
                        }
                }
            }
        });
        for (const auto& v : cand)
            for (const Cand& cd : v) {
                if (is_hang[size_t(cd.n)]) continue;
                std::vector<std::pair<int64_t, double>> ms;
                for (int j = 0; j < cd.nm; ++j) ms.push_back({cd.mst[j], cd.w});
                set_hang(cd.n, std::move(ms));
            }
        // resolve chains (a master that is itself hanging)
        for (int64_t n = 0; n < m.n_nodes; ++n) {
            if (!is_hang[size_t(n)]) continue;
            for (int guard = 0; guard < 8; ++guard) {
                bool again = false;
                std::vector<std::pair<int64_t, double>> nx;
                for (auto& mw : hang[size_t(hid[size_t(n)])]) {
                    if (is_hang[size_t(mw.first)]) {
                        again = true;
                        for (auto& m2 : hang[size_t(hid[size_t(mw.first)])]) nx.push_back({m2.first, mw.second * m2.second});
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
                hang[size_t(hid[size_t(n)])] = mg;
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
                for (auto& mw : hang[size_t(hid[size_t(n)])]) {
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

HostMesh refine_mesh(const HostMesh& old, const uint8_t* flags, std::vector<int32_t>& loc_cell,
                     std::vector<double>& loc_xi) {
    if (old.n_inst != 1) fail(FR_EINVAL, "mesh_refine: batched meshes are not supported");
    const int dim = old.dim, nv = old.nv;
    const int L0 = old.levels;
    const int64_t nc = old.n_cells;
    // level of every old cell from its edge in lattice units (vertex nv-1 minus vertex 0)
    std::vector<int8_t> lev(static_cast<size_t>(nc));
    bool grow = false;
    for (int64_t c = 0; c < nc; ++c) {
        const int64_t a = old.cells[size_t(c) * nv], b = old.cells[size_t(c) * nv + nv - 1];
        const int64_t s = old.lattice[size_t(b) * dim] - old.lattice[size_t(a) * dim];
        int l = L0;
        for (int64_t t = s; t > 1; t >>= 1) --l;
        if (l < 0 || (int64_t(1) << (L0 - l)) != s) fail(FR_EINTERNAL, "mesh_refine: cell edge is not a power of two");
        lev[size_t(c)] = int8_t(l);
        if (flags[c] && l == L0) grow = true;
    }
    const int L1 = L0 + (grow ? 1 : 0);
    if (L1 > 12) fail(FR_EINVAL, "mesh_refine: more than 12 levels");
    const int64_t f = grow ? 2 : 1;
    const int64_t S1 = int64_t(1) << L1;
    int64_t ext1[3] = {1, 1, 1};
    for (int k = 0; k < dim; ++k) ext1[k] = int64_t(old.desc.base[k]) * S1;
    for (int k = 0; k < dim; ++k)
        if (ext1[k] >= (int64_t(1) << 21)) fail(FR_EINVAL, "mesh_refine: more than 2^21 finest cells per axis");
    // split: every ancestor of an old leaf (the old tree) and every flagged leaf
    std::vector<KeySet> split(static_cast<size_t>(std::max(L1, 1)));
    for (int64_t c = 0; c < nc; ++c) {
        const int l = lev[size_t(c)];
        int64_t o[3] = {0, 0, 0};
        const int64_t a = old.cells[size_t(c) * nv];
        for (int k = 0; k < dim; ++k) o[k] = old.lattice[size_t(a) * dim + k] * f;
        if (flags[c]) split[size_t(l)].insert(pack(o));
        for (int j = l - 1; j >= 0; --j) {
            const int64_t sz = S1 >> j;
            int64_t po[3] = {0, 0, 0};
            for (int k = 0; k < dim; ++k) po[k] = (o[k] / sz) * sz;
            if (!split[size_t(j)].insert(pack(po))) break;
        }
    }
    RefineSeed seed;
    seed.L = L1;
    seed.split.resize(size_t(L1));
    for (int l = 0; l < L1; ++l) {
        seed.split[size_t(l)].reserve(split[size_t(l)].size());
        split[size_t(l)].for_each([&](uint64_t k) { seed.split[size_t(l)].push_back(k); });
    }
    HostMesh m = build_mesh(old.desc, &seed);
    if (m.levels != L1) fail(FR_EINTERNAL, "mesh_refine: level count");
    // locate every new node in an old cell: the old leaf of the finest level that contains it
    std::vector<std::vector<std::pair<uint64_t, int32_t>>> byl(static_cast<size_t>(L0) + 1);
    for (int64_t c = 0; c < nc; ++c) {
        int64_t o[3] = {0, 0, 0};
        const int64_t a = old.cells[size_t(c) * nv];
        for (int k = 0; k < dim; ++k) o[k] = old.lattice[size_t(a) * dim + k] * f;
        byl[size_t(lev[size_t(c)])].push_back({pack(o), int32_t(c)});
    }
    for (auto& v : byl) std::sort(v.begin(), v.end());
    loc_cell.assign(size_t(m.n_nodes), -1);
    loc_xi.assign(size_t(m.n_nodes) * dim, 0.0);
    parallel_ranges(m.n_nodes, [&](int64_t b, int64_t e, int) {
        for (int64_t n = b; n < e; ++n) {
            const int64_t* q = &m.lattice[size_t(n) * dim];
            for (int l = L0; l >= 0; --l) {
                const int64_t sz = S1 >> l;
                int64_t o[3] = {0, 0, 0};
                for (int k = 0; k < dim; ++k) o[k] = std::min((q[k] / sz) * sz, ext1[k] - sz);
                const auto& v = byl[size_t(l)];
                auto it = std::lower_bound(v.begin(), v.end(), std::make_pair(pack(o), int32_t(-1)));
                if (it == v.end() || it->first != pack(o)) continue;
                loc_cell[size_t(n)] = it->second;
                for (int k = 0; k < dim; ++k) loc_xi[size_t(n) * dim + k] = double(q[k] - o[k]) / double(sz);
                break;
            }
        }
    });
    for (int64_t n = 0; n < m.n_nodes; ++n)
        if (loc_cell[size_t(n)] < 0) fail(FR_EINTERNAL, "mesh_refine: a node of the refined mesh lies in no old cell");
    m.node_off = {0, m.n_nodes};
    m.cell_off = {0, m.n_cells};
    m.free_off = {0, m.n_free};
    m.inst_h_min = {m.h_min};
    return m;
}

void face_neighbors(const HostMesh& m, std::vector<int32_t>& ptr, std::vector<int32_t>& nbr) {
    const int dim = m.dim, nv = m.nv, nf = 2 * dim;
    const int64_t nc = m.n_cells;
    ptr.assign(size_t(nc) * nf + 1, 0);
    nbr.clear();
    // cells keyed by (instance, edge in lattice units, origin): the instances of a batch have
    // their own lattices
    std::vector<int32_t> inst(static_cast<size_t>(nc), 0);
    for (int i = 0; i < m.n_inst; ++i)
        for (int64_t c = m.cell_off.empty() ? 0 : m.cell_off[size_t(i)];
             c < (m.cell_off.empty() ? nc : m.cell_off[size_t(i) + 1]); ++c)
            inst[size_t(c)] = i;
    auto key = [&](int i, int64_t s, const int64_t* o) {
        int lg = 0;
        while ((int64_t(1) << lg) < s) ++lg;
        return std::make_pair((uint64_t(i) << 8) | uint64_t(lg), pack(o));
    };
    std::vector<std::pair<std::pair<uint64_t, uint64_t>, int32_t>> tab(static_cast<size_t>(nc));
    std::vector<int64_t> edge(static_cast<size_t>(nc));
    std::vector<std::array<int64_t, 3>> org(static_cast<size_t>(nc));
    std::vector<std::array<int64_t, 3>> iext(static_cast<size_t>(m.n_inst), {0, 0, 0});
    for (int64_t c = 0; c < nc; ++c) {
        const int64_t a = m.cells[size_t(c) * nv], b = m.cells[size_t(c) * nv + nv - 1];
        std::array<int64_t, 3> o{0, 0, 0};
        for (int k = 0; k < dim; ++k) o[k] = m.lattice[size_t(a) * dim + k];
        edge[size_t(c)] = m.lattice[size_t(b) * dim] - m.lattice[size_t(a) * dim];
        org[size_t(c)] = o;
        tab[size_t(c)] = {key(inst[size_t(c)], edge[size_t(c)], o.data()), int32_t(c)};
        for (int k = 0; k < dim; ++k)
            iext[size_t(inst[size_t(c)])][size_t(k)] =
                std::max(iext[size_t(inst[size_t(c)])][size_t(k)], o[k] + edge[size_t(c)]);
    }
    std::sort(tab.begin(), tab.end());
    auto find = [&](int i, int64_t s, const int64_t* o) -> int32_t {
        const auto k = key(i, s, o);
        auto it = std::lower_bound(tab.begin(), tab.end(), std::make_pair(k, int32_t(-1)));
        return (it != tab.end() && it->first == k) ? it->second : -1;
    };
    // cells in contiguous ranges, one per host thread; each range lists its neighbours in cell
    // order and the ranges are joined in order, so the table equals a serial sweep's
    std::vector<std::vector<int32_t>> part(16);
    std::vector<int32_t> cnt(size_t(nc) * nf, 0);
    parallel_ranges(nc, [&](int64_t cb, int64_t ce, int t) {
        std::vector<int32_t>& out = part[size_t(t)];
        for (int64_t c = cb; c < ce; ++c) {
            const int i = inst[size_t(c)];
            const int64_t s = edge[size_t(c)];
            const auto& o = org[size_t(c)];
            for (int j = 0; j < nf; ++j) {
                const int k = j / 2, side = j % 2;
                const int64_t q = side ? o[k] + s : o[k] - s;     // origin of a same-size neighbour
                if (side ? (o[k] + s >= iext[size_t(i)][size_t(k)]) : (o[k] == 0)) continue;
                const size_t before = out.size();
                int64_t on[3] = {o[0], o[1], o[2]};
                on[k] = q;
                int32_t n = find(i, s, on);
                if (n >= 0) {
                    out.push_back(n);
                } else {
                    // coarser: the cell of edge 2s that holds the same-size neighbour
                    int64_t oc[3] = {0, 0, 0};
                    for (int t = 0; t < dim; ++t) oc[t] = (on[t] / (2 * s)) * (2 * s);
                    n = find(i, 2 * s, oc);
                    if (n >= 0) {
                        out.push_back(n);
                    } else {
                        // finer: the 2^(dim-1) cells of edge s/2 along the face
                        const int64_t h = s / 2;
                        for (int sub = 0; sub < (1 << (dim - 1)); ++sub) {
                            int64_t of[3] = {on[0], on[1], on[2]};
                            of[k] = side ? q : q + h;
                            int b = 0;
                            for (int t = 0; t < dim; ++t) {
                                if (t == k) continue;
                                of[t] = o[t] + ((sub >> b) & 1) * h;
                                ++b;
                            }
                            const int32_t f = h >= 1 ? find(i, h, of) : -1;
                            if (f < 0) fail(FR_EINTERNAL, "kelly: face neighbour not found (mesh not 2:1 balanced?)");
                            out.push_back(f);
                        }
                    }
                }
                cnt[size_t(c) * nf + j] = int32_t(out.size() - before);
            }
        }
    });
    for (int64_t e = 0; e < nc * nf; ++e) ptr[size_t(e) + 1] = ptr[size_t(e)] + cnt[size_t(e)];
    nbr.reserve(size_t(ptr[size_t(nc) * nf]));
    for (auto& v : part) nbr.insert(nbr.end(), v.begin(), v.end());
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
    // node -> cells adjacency, filled by host threads with atomic counters: the order of a
    // node's list is arbitrary, and every row below sorts its entries by (cell, vertex), which
    // are unique, so the pattern does not depend on it
    std::vector<int32_t> nc_ptr(size_t(nn) + 1, 0);
    parallel_ranges(m.n_cells, [&](int64_t c0, int64_t c1, int) {
        for (int64_t c = c0; c < c1; ++c)
            for (int a = 0; a < nv; ++a)
                __atomic_fetch_add(&nc_ptr[size_t(m.cells[size_t(c) * nv + a]) + 1], 1, __ATOMIC_RELAXED);
    });
    for (int64_t n = 0; n < nn; ++n) nc_ptr[size_t(n) + 1] += nc_ptr[size_t(n)];
    const size_t n_inc = size_t(nc_ptr[size_t(nn)]);
    std::vector<int32_t> nc_cell(n_inc), nc_a(n_inc);
    {
        std::vector<int32_t> fill(nc_ptr.begin(), nc_ptr.end() - 1);
        parallel_ranges(m.n_cells, [&](int64_t c0, int64_t c1, int) {
            for (int64_t c = c0; c < c1; ++c)
                for (int a = 0; a < nv; ++a) {
                    const int32_t n = m.cells[size_t(c) * nv + a];
                    const int32_t pos = __atomic_fetch_add(&fill[size_t(n)], 1, __ATOMIC_RELAXED);
                    nc_cell[size_t(pos)] = int32_t(c);
                    nc_a[size_t(pos)] = a;
                }
        });
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
    // per row: assembly entries (cell, vertex, weight) ordered by (cell, vertex) and the
    // sorted unique node columns; rows are independent, so host threads take row ranges and
    // the pieces are concatenated in row order
    struct Ent { int32_t cell; uint8_t a; double w; };
    struct Part {
        std::vector<Ent> ents;
        std::vector<int32_t> n_ent, cols, n_col;
        int max_row = 0;
    };
    const int64_t hw = std::max<int64_t>(1, std::thread::hardware_concurrency());
    const int64_t T = std::max<int64_t>(1, std::min<int64_t>({hw, 16, nf / 4096 + 1}));
    std::vector<Part> parts(static_cast<size_t>(T));
    {
        std::vector<std::thread> th;
        std::vector<std::exception_ptr> err(static_cast<size_t>(T));
        for (int64_t t = 0; t < T; ++t)
            th.emplace_back([&, t]() {
                try {
                    Part& P = parts[size_t(t)];
                    const int64_t f0 = nf * t / T, f1 = nf * (t + 1) / T;
                    std::vector<Ent> tmp;
                    std::vector<int32_t> cand;
                    for (int64_t f = f0; f < f1; ++f) {
                        tmp.clear();
                        const int32_t node = m.node_of_free[size_t(f)];
                        for (int32_t j = nc_ptr[size_t(node)]; j < nc_ptr[size_t(node) + 1]; ++j)
                            tmp.push_back(Ent{nc_cell[size_t(j)], uint8_t(nc_a[size_t(j)]), 1.0});
                        if (m.n_hanging > 0)
                            for (int32_t j = dep_ptr[size_t(f)]; j < dep_ptr[size_t(f) + 1]; ++j) {
                                const int32_t h = dep_node[size_t(j)];
                                for (int32_t q = nc_ptr[size_t(h)]; q < nc_ptr[size_t(h) + 1]; ++q)
                                    tmp.push_back(Ent{nc_cell[size_t(q)], uint8_t(nc_a[size_t(q)]), dep_w[size_t(j)]});
                            }
                        std::sort(tmp.begin(), tmp.end(), [](const Ent& x, const Ent& y) {
                            return x.cell != y.cell ? x.cell < y.cell : x.a < y.a;
                        });
                        cand.clear();
                        for (const Ent& e : tmp) {
                            P.ents.push_back(e);
                            for (int b = 0; b < nv; ++b) {
                                const int32_t n = m.cells[size_t(e.cell) * nv + b];
                                for (int32_t q = m.con_ptr[size_t(n)]; q < m.con_ptr[size_t(n) + 1]; ++q)
                                    cand.push_back(m.con_master[size_t(q)]);
                            }
                        }
                        std::sort(cand.begin(), cand.end());
                        cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
                        if (cand.size() > 254) fail(FR_EINTERNAL, "pattern: more than 254 node neighbours in a row");
                        P.max_row = std::max(P.max_row, int(cand.size()));
                        P.n_ent.push_back(int32_t(tmp.size()));
                        P.n_col.push_back(int32_t(cand.size()));
                        P.cols.insert(P.cols.end(), cand.begin(), cand.end());
                    }
                } catch (...) {
                    err[size_t(t)] = std::current_exception();
                }
            });
        for (auto& x : th) x.join();
        for (auto& e : err)
            if (e) std::rethrow_exception(e);
    }
    // concatenate: entry pointers, row column lists (col_ptr / col_all)
    p.ent_ptr.assign(size_t(nf) + 1, 0);
    std::vector<int64_t> col_ptr(size_t(nf) + 1, 0);
    int max_row = 0;
    {
        int64_t f = 0;
        for (const Part& P : parts) {
            for (size_t r = 0; r < P.n_ent.size(); ++r, ++f) {
                p.ent_ptr[size_t(f) + 1] = p.ent_ptr[size_t(f)] + P.n_ent[r];
                col_ptr[size_t(f) + 1] = col_ptr[size_t(f)] + P.n_col[r];
            }
            max_row = std::max(max_row, P.max_row);
        }
    }
    p.max_row = max_row;
    const size_t n_ent = size_t(p.ent_ptr[size_t(nf)]);
    std::vector<Ent> ents(n_ent);
    std::vector<int32_t> col_all(static_cast<size_t>(col_ptr[static_cast<size_t>(nf)]));
    {
        // every part's pieces go to known offsets: one host thread per part
        std::vector<size_t> eo(parts.size() + 1, 0), co(parts.size() + 1, 0);
        for (size_t t = 0; t < parts.size(); ++t) {
            eo[t + 1] = eo[t] + parts[t].ents.size();
            co[t + 1] = co[t] + parts[t].cols.size();
        }
        std::vector<std::thread> th;
        for (size_t t = 0; t < parts.size(); ++t)
            th.emplace_back([&, t]() {
                std::copy(parts[t].ents.begin(), parts[t].ents.end(), ents.begin() + int64_t(eo[t]));
                std::copy(parts[t].cols.begin(), parts[t].cols.end(), col_all.begin() + int64_t(co[t]));
                parts[t] = Part();
            });
        for (auto& x : th) x.join();
    }
    p.ent_cell.resize(n_ent);
    p.ent_a.resize(n_ent);
    p.ent_w.resize(n_ent);
    p.ent_k.resize(n_ent * size_t(nv));
    parallel_ranges(nf, [&](int64_t f0, int64_t f1, int) {
        for (int64_t f = f0; f < f1; ++f) {
            const int32_t* cb = col_all.data() + col_ptr[size_t(f)];
            const int32_t* ce = col_all.data() + col_ptr[size_t(f) + 1];
            for (int32_t e = p.ent_ptr[size_t(f)]; e < p.ent_ptr[size_t(f) + 1]; ++e) {
                const Ent& en = ents[size_t(e)];
                p.ent_cell[size_t(e)] = en.cell;
                p.ent_a[size_t(e)] = en.a;
                p.ent_w[size_t(e)] = en.w;
                for (int b = 0; b < nv; ++b) {
                    const int32_t n = m.cells[size_t(en.cell) * nv + b];
                    const int32_t fb = m.free_of_node[size_t(n)];
                    uint8_t k = 255;
                    if (fb >= 0) k = uint8_t(std::lower_bound(cb, ce, fb) - cb);
                    p.ent_k[size_t(e) * nv + b] = k;
                }
            }
        }
    });
    if (m.n_hanging > 0) {
        // masters of hanging vertices: counted per row, then located in the row's columns
        p.hang_ptr.assign(size_t(nf) + 1, 0);
        parallel_ranges(nf, [&](int64_t f0, int64_t f1, int) {
            for (int64_t f = f0; f < f1; ++f) {
                int64_t c = 0;
                for (int32_t e = p.ent_ptr[size_t(f)]; e < p.ent_ptr[size_t(f) + 1]; ++e)
                    for (int b = 0; b < nv; ++b)
                        if (p.ent_k[size_t(e) * nv + b] == 255) {
                            const int32_t n = m.cells[size_t(p.ent_cell[size_t(e)]) * nv + b];
                            c += m.con_ptr[size_t(n) + 1] - m.con_ptr[size_t(n)];
                        }
                p.hang_ptr[size_t(f) + 1] = int32_t(c);
            }
        });
        int64_t tot = 0;
        for (int64_t f = 0; f < nf; ++f) {
            tot += p.hang_ptr[size_t(f) + 1];
            if (tot >= (int64_t(1) << 31)) fail(FR_EINTERNAL, "pattern: more than 2^31 hanging-column entries");
            p.hang_ptr[size_t(f) + 1] = int32_t(tot);
        }
        p.hang_k.resize(size_t(tot));
        parallel_ranges(nf, [&](int64_t f0, int64_t f1, int) {
            for (int64_t f = f0; f < f1; ++f) {
                const int32_t* cb = col_all.data() + col_ptr[size_t(f)];
                const int32_t* ce = col_all.data() + col_ptr[size_t(f) + 1];
                size_t o = size_t(p.hang_ptr[size_t(f)]);
                for (int32_t e = p.ent_ptr[size_t(f)]; e < p.ent_ptr[size_t(f) + 1]; ++e)
                    for (int b = 0; b < nv; ++b) {
                        if (p.ent_k[size_t(e) * nv + b] != 255) continue;
                        const int32_t n = m.cells[size_t(p.ent_cell[size_t(e)]) * nv + b];
                        for (int32_t j = m.con_ptr[size_t(n)]; j < m.con_ptr[size_t(n) + 1]; ++j) {
                            const int32_t g = m.con_master[size_t(j)];
                            const int32_t* it = std::lower_bound(cb, ce, g);
                            if (it == ce || *it != g) fail(FR_EINTERNAL, "pattern: hanging master missing from its row");
                            p.hang_k[o++] = uint8_t(it - cb);
                        }
                    }
            }
        });
    }
    // SELL-C layout (no row sorting: the node numbering already groups similar rows)
    p.n_slices = ceil_div(nf, C);
    p.slice_ptr.assign(size_t(p.n_slices) + 1, 0);
    p.row_len.resize(size_t(nf));
    int64_t off = 0;
    for (int64_t s = 0; s < p.n_slices; ++s) {
        int w = 0;
        for (int64_t r = s * C; r < std::min<int64_t>(nf, (s + 1) * C); ++r)
            w = std::max(w, int(col_ptr[size_t(r) + 1] - col_ptr[size_t(r)]));
        p.slice_ptr[size_t(s)] = int32_t(off);
        off += int64_t(w) * C;
        if (off >= (int64_t(1) << 31)) fail(FR_EINTERNAL, "pattern: more than 2^31 slots");
    }
    p.slice_ptr[size_t(p.n_slices)] = int32_t(off);
    p.n_slots = off;
    p.col.assign(size_t(off), 0);
    int64_t nnz = 0;
    for (int64_t r = 0; r < nf; ++r) {
        const int32_t* cf = col_all.data() + col_ptr[size_t(r)];
        const int len = int(col_ptr[size_t(r) + 1] - col_ptr[size_t(r)]);
        int64_t s = r / C, lane = r % C;
        int w = (p.slice_ptr[size_t(s) + 1] - p.slice_ptr[size_t(s)]) / C;
        p.row_len[size_t(r)] = int32_t(len);
        nnz += int64_t(len);
        for (int k = 0; k < w; ++k)
            p.col[size_t(p.slice_ptr[size_t(s)] + int64_t(k) * C + lane)] = k < len ? cf[k] : int32_t(r);
    }
    // slots of padded lanes past the last row point at row 0 (any valid column)
    p.nnz = nnz;
    return p;
}

}  // namespace fr
