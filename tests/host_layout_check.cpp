// host_layout_check.cpp -- CPU check of the library's host-only graph preparation
// (paper_1908_00210_amd/csrc/gdi_layout.cpp), built by tests/test_host_layout.py with
// the address and undefined-behaviour sanitizers. It runs the CSR validator on
// malformed inputs, and the colouring, relabelling and halo layout on generated graphs
// over grid sizes, tail starts and leader settings, and checks every invariant the
// sweep kernels rely on: each packed entry names the neighbour's bit in its owner's
// LDS image, windows and regions stay inside the image, chunks partition each class.
// Prints "OK <layouts checked>" and exits 0, or prints the first failure and exits 1.

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <set>
#include <string>
#include <vector>

#include "../include/gdi.h"
#include "../paper_1908_00210_amd/csrc/gdi_layout.h"

using namespace gdi_layout;

namespace {

struct Csr {
    int32_t n = 0;
    std::vector<int32_t> rp, col, w;
};

#define CHECK(cond, ...)                                 \
    do {                                                 \
        if (!(cond)) {                                   \
            std::printf("FAIL %s:%d: ", __FILE__, __LINE__); \
            std::printf(__VA_ARGS__);                    \
            std::printf("\n");                           \
            std::exit(1);                                \
        }                                                \
    } while (0)

Csr from_edges(int32_t n, const std::vector<std::pair<int32_t, int32_t>> &edges, const std::vector<int32_t> &wts)
{
    std::vector<std::vector<std::pair<int32_t, int32_t>>> rows((size_t)n);
    for (size_t e = 0; e < edges.size(); ++e) {
        rows[(size_t)edges[e].first].emplace_back(edges[e].second, wts[e]);
        rows[(size_t)edges[e].second].emplace_back(edges[e].first, wts[e]);
    }
    Csr g;
    g.n = n;
    g.rp.assign(1, 0);
    g.col.reserve(1);  // non-null arrays also for a graph without edges (NULL is rejected)
    g.w.reserve(1);
    for (auto &r : rows) {
        std::sort(r.begin(), r.end());
        for (auto &p : r) {
            g.col.push_back(p.first);
            g.w.push_back(p.second);
        }
        g.rp.push_back((int32_t)g.col.size());
    }
    return g;
}

// weights: 0 unit, 1 +-1, 2 up to the packed range, 3 one weight beyond it
std::vector<int32_t> weights(size_t m, int kind, std::mt19937 &rng)
{
    std::vector<int32_t> w(m, 1);
    for (size_t e = 0; e < m; ++e) {
        if (kind == 1) w[e] = (rng() & 1) ? 1 : -1;
        if (kind >= 2) w[e] = (int32_t)(rng() % 2047) - 1023;
    }
    if (kind == 3 && m) w[m / 2] = 5000;
    return w;
}

Csr er(int32_t n, double p, int kind, uint32_t seed)
{
    std::mt19937 rng(seed);
    std::uniform_real_distribution<double> U(0.0, 1.0);
    std::vector<std::pair<int32_t, int32_t>> e;
    for (int32_t i = 0; i < n; ++i)
        for (int32_t j = i + 1; j < n; ++j)
            if (U(rng) < p) e.emplace_back(i, j);
    return from_edges(n, e, weights(e.size(), kind, rng));
}

// points on a grid with neighbours within a radius, plus a few hubs with long rows
Csr local(int32_t side, int32_t radius, int32_t hubs, int kind, uint32_t seed)
{
    std::mt19937 rng(seed);
    const int32_t n = side * side;
    std::set<std::pair<int32_t, int32_t>> es;
    for (int32_t y = 0; y < side; ++y)
        for (int32_t x = 0; x < side; ++x)
            for (int32_t dy = 0; dy <= radius; ++dy)
                for (int32_t dx = -radius; dx <= radius; ++dx) {
                    if (dy == 0 && dx <= 0) continue;
                    const int32_t x2 = x + dx, y2 = y + dy;
                    if (x2 < 0 || x2 >= side || y2 >= side) continue;
                    if ((rng() % 3) == 0) es.emplace(y * side + x, y2 * side + x2);
                }
    for (int32_t h = 0; h < hubs; ++h) {
        const int32_t c = (int32_t)(rng() % (uint32_t)n);
        for (int32_t k = 0; k < 40; ++k) {
            const int32_t j = (int32_t)(rng() % (uint32_t)n);
            if (j != c) es.emplace(std::min(c, j), std::max(c, j));
        }
    }
    std::vector<std::pair<int32_t, int32_t>> e(es.begin(), es.end());
    return from_edges(n, e, weights(e.size(), kind, rng));
}

int32_t sext11(uint32_t e) { return (int32_t)(e << 16) >> 21; }

long check_layouts(const Csr &g, const char *name)
{
    int64_t mw = 0;
    int32_t md = 0;
    std::string err;
    CHECK(validate_csr(g.rp.data(), g.col.data(), g.w.data(), g.n, &mw, &md, &err) == GDI_OK, "%s: %s", name,
          err.c_str());
    std::vector<int32_t> colour((size_t)g.n);
    const int32_t C = colour_first_fit(g.rp.data(), g.col.data(), g.n, colour.data());
    for (int32_t i = 0; i < g.n; ++i) {
        std::vector<char> seen((size_t)C + 1, 0);
        for (int32_t k = g.rp[(size_t)i]; k < g.rp[(size_t)i + 1]; ++k) {
            const int32_t j = g.col[(size_t)k];
            CHECK(colour[(size_t)j] != colour[(size_t)i], "%s: neighbours %d %d share a colour", name, i, j);
            if (j < i) seen[(size_t)colour[(size_t)j]] = 1;
        }
        for (int32_t c = 0; c < colour[(size_t)i]; ++c)
            CHECK(seen[(size_t)c], "%s: node %d skips free colour %d", name, i, c);
    }
    Relabelled r;
    CHECK(relabel(g.rp.data(), g.col.data(), g.w.data(), g.n, colour.data(), C, &r, &err) == GDI_OK, "%s: relabel",
          name);
    CHECK((int32_t)r.orig.size() == r.n_pad && (int32_t)r.rp.size() == r.n_pad + 1, "%s: sizes", name);
    std::vector<int32_t> inv((size_t)g.n, -1);
    for (int32_t v = 0; v < r.n_pad; ++v) {
        const int32_t o = r.orig[(size_t)v];
        if (o < 0) {
            CHECK(r.cls[(size_t)v] == -1 && r.rp[(size_t)v + 1] == r.rp[(size_t)v], "%s: padding id %d", name, v);
            continue;
        }
        CHECK(inv[(size_t)o] == -1, "%s: original id %d twice", name, o);
        inv[(size_t)o] = v;
        CHECK(r.cls[(size_t)v] == colour[(size_t)o], "%s: class of %d", name, v);
    }
    for (int32_t c = 0; c < C; ++c) CHECK(r.cbeg[(size_t)c] % GDI_CLASS_ALIGN == 0, "%s: class start", name);
    for (int32_t v = 0; v < r.n_pad; ++v) {
        const int32_t o = r.orig[(size_t)v];
        if (o < 0) continue;
        CHECK(r.rp[(size_t)v + 1] - r.rp[(size_t)v] == g.rp[(size_t)o + 1] - g.rp[(size_t)o], "%s: row length", name);
        for (int32_t k = r.rp[(size_t)v]; k < r.rp[(size_t)v + 1]; ++k) {
            if (k > r.rp[(size_t)v]) CHECK(r.adj[(size_t)k - 1].x < r.adj[(size_t)k].x, "%s: row order", name);
            const int32_t j = r.orig[(size_t)r.adj[(size_t)k].x];
            const int32_t *b = g.col.data() + g.rp[(size_t)o], *e = g.col.data() + g.rp[(size_t)o + 1];
            const int32_t *f = std::lower_bound(b, e, j);
            CHECK(f != e && *f == j && g.w[(size_t)(f - g.col.data())] == r.adj[(size_t)k].y, "%s: entry", name);
        }
    }
    long checked = 0;
    // packed rows: built exactly for +-1 weights and n_pad < 32767; each row's chunks
    // decode to its entries followed by padding that names node n_pad
    {
        bool pm1 = true;
        for (const Edge &e : r.adj) pm1 = pm1 && (e.y == 1 || e.y == -1);
        PackedRows pr;
        const int rc = pack_rows8(r, &pr, &err);
        CHECK((rc == 0) == (pm1 && r.n_pad < 32767), "%s: pack_rows8 applicability", name);
        if (rc == 0) {
            CHECK(pr.prow.size() == (size_t)r.n_pad + 1 && pr.prow[0] == 0, "%s: prow size", name);
            CHECK(pr.pent.size() == (size_t)std::max<uint32_t>(pr.prow[(size_t)r.n_pad], 1) * GDI_P8_ENTRIES,
                  "%s: pent size", name);
            for (int32_t v = 0; v < r.n_pad; ++v) {
                const int32_t r0 = r.rp[(size_t)v], deg = r.rp[(size_t)v + 1] - r0;
                const uint32_t c0 = pr.prow[(size_t)v], c1 = pr.prow[(size_t)v + 1];
                CHECK(c1 - c0 == (uint32_t)((deg + GDI_P8_ENTRIES - 1) / GDI_P8_ENTRIES), "%s: chunks of %d", name, v);
                for (uint32_t q = 0; q < (c1 - c0) * GDI_P8_ENTRIES; ++q) {
                    const uint16_t x = pr.pent[(size_t)c0 * GDI_P8_ENTRIES + q];
                    if ((int32_t)q < deg) {
                        const Edge &a = r.adj[(size_t)r0 + q];
                        CHECK((x & 0x7FFF) == a.x && ((x >> 15) ? -1 : 1) == a.y, "%s: packed entry", name);
                    } else {
                        CHECK(x == (uint16_t)r.n_pad, "%s: padding entry", name);
                    }
                }
                ++checked;
            }
        }
    }
    const int budget = 160 * 1024 - 256;
    for (int32_t G : {8, 16, 64, 256}) {
        for (int32_t lead : {0, 8}) {
            if (lead && G < 16) continue;
            std::vector<int32_t> t0s = {C};
            if (C > 3) t0s.push_back(C - 1);
            if (C > 4) t0s.push_back(3);
            for (int32_t T0 : t0s) {
                HaloLayout L;
                CHECK(halo_layout(r, C, G, budget, T0, lead, &L, &err) == GDI_OK, "%s: halo_layout: %s", name,
                      err.c_str());
                if (L.status == -3) {
                    CHECK(std::any_of(r.adj.begin(), r.adj.end(), [](const Edge &e) {
                              return e.y < -GDI_HALO_WMAX - 1 || e.y > GDI_HALO_WMAX;
                          }), "%s: weights rejected without cause", name);
                    continue;
                }
                if (L.status == -2) continue;  // does not fit the budget: the library falls back
                ++checked;
                CHECK(gdi_halo_lds_bytes(L.lds_words, C, 0) <= budget && L.lds_words <= 65536, "%s: LDS budget", name);
                CHECK(L.adjL.size() == r.adj.size() + GDI_HALO_PF, "%s: adjL size", name);
                for (size_t k = r.adj.size(); k < L.adjL.size(); ++k) CHECK(L.adjL[k] == 0, "%s: zero tail", name);
                // chunks partition each grid class; interior bounds are multiples of 64
                for (int32_t c = 0; c < T0; ++c) {
                    std::vector<char> own((size_t)r.csz[(size_t)c], 0);
                    for (int32_t b = 0; b < G; ++b) {
                        const GdiHaloEntry &e = L.tab[(size_t)b * C + c];
                        if (b < lead) CHECK(e.node_hi == e.node_lo, "%s: leader holds nodes", name);
                        if (e.node_hi > e.node_lo) CHECK(e.node_lo % 64 == 0, "%s: chunk start", name);
                        for (int32_t v = e.node_lo; v < e.node_hi; ++v) {
                            const int32_t q = v - r.cbeg[(size_t)c];
                            CHECK(q >= 0 && q < r.csz[(size_t)c] && !own[(size_t)q], "%s: chunk overlap", name);
                            own[(size_t)q] = 1;
                        }
                    }
                    CHECK(std::all_of(own.begin(), own.end(), [](char x) { return x != 0; }), "%s: chunk gap", name);
                }
                // owner of every grid node
                std::vector<int32_t> owner((size_t)r.n_pad, -1);
                for (int32_t b = 0; b < G; ++b)
                    for (int32_t c = 0; c < T0; ++c)
                        for (int32_t v = L.tab[(size_t)b * C + c].node_lo; v < L.tab[(size_t)b * C + c].node_hi; ++v)
                            owner[(size_t)v] = b;
                // images: own words then foreign copies per class, inside [0, gather_off);
                // foreign lists ascending, foreign to the block, copied in the list region
                for (int32_t b = 0; b < G; ++b) {
                    int32_t end = 0;
                    for (int32_t c = 0; c < C; ++c) {
                        const GdiHaloEntry &e = L.tab[(size_t)b * C + c];
                        const int32_t nown = e.node_hi > e.node_lo ? ((e.node_hi + 31) >> 5) - (e.node_lo >> 5) : 0;
                        CHECK(e.own_off >= end && e.for_off >= e.own_off + nown && e.for_len >= 0, "%s: image order", name);
                        end = e.for_off + e.for_len;
                        CHECK(end <= L.gather_off, "%s: image outside", name);
                        CHECK(e.list_off >= L.list_off && e.list_off + e.for_len <= L.list_off + L.flist_len,
                              "%s: list outside", name);
                        const int32_t *lst = L.flist.data() + (size_t)b * L.flist_len + (e.list_off - L.list_off);
                        for (int32_t i = 0; i < e.for_len; ++i) {
                            const int32_t wd = lst[i];
                            CHECK(wd >= 0 && wd * 32 < r.n_pad && (i == 0 || lst[i - 1] < wd), "%s: list order", name);
                            const int32_t j0 = wd * 32;
                            bool any_c = false, any_own = false;
                            for (int32_t j = j0; j < j0 + 32; ++j) {
                                any_c |= r.cls[(size_t)j] == c;
                                any_own |= owner[(size_t)j] == b;
                            }
                            CHECK(any_c && !any_own, "%s: foreign word %d of class %d", name, wd, c);
                        }
                    }
                }
                const int32_t tail_base = T0 < C ? r.cbeg[(size_t)T0] : r.n_pad;
                auto expect_lb = [&](int32_t b, int32_t j) {
                    const int32_t cj = r.cls[(size_t)j];
                    if (cj >= T0) return (L.tail_off + ((j - tail_base) >> 5)) * 32 + (j & 31);
                    const GdiHaloEntry &e = L.tab[(size_t)b * C + cj];
                    if (owner[(size_t)j] == b) return (e.own_off + (j >> 5) - (e.node_lo >> 5)) * 32 + (j & 31);
                    const int32_t *lst = L.flist.data() + (size_t)b * L.flist_len + (e.list_off - L.list_off);
                    const int32_t *f = std::lower_bound(lst, lst + e.for_len, j >> 5);
                    CHECK(f != lst + e.for_len && *f == (j >> 5), "%s: neighbour word not listed", name);
                    return (e.for_off + (int32_t)(f - lst)) * 32 + (j & 31);
                };
                for (int32_t v = 0; v < r.n_pad; ++v) {
                    const int32_t cv = r.cls[(size_t)v];
                    if (cv < 0 || cv >= T0) continue;
                    const int32_t b = owner[(size_t)v];
                    CHECK(b >= lead, "%s: node %d without owner", name, v);
                    const int32_t r0 = r.rp[(size_t)v], deg = r.rp[(size_t)v + 1] - r0;
                    const bool linked = L.ovf_len > 0 && deg > GDI_HALO_PF;
                    for (int32_t q = 0; q < deg; ++q) {
                        uint32_t e;
                        if (linked && q >= GDI_HALO_PF - 1) {
                            const int32_t pos = (int32_t)L.adjL[(size_t)r0 + GDI_HALO_PF - 1] - L.ovf_off;
                            CHECK(pos >= 0 && pos + deg - (GDI_HALO_PF - 1) <= L.ovf_len, "%s: overflow link", name);
                            e = L.ovf[(size_t)b * L.ovf_len + pos + (q - (GDI_HALO_PF - 1))];
                        } else {
                            e = L.adjL[(size_t)r0 + q];
                        }
                        const Edge &a = r.adj[(size_t)r0 + q];
                        CHECK(sext11(e) == a.y, "%s: packed weight", name);
                        const int32_t lb = (int32_t)(e >> 16) * 32 + (int32_t)(e & 31u);
                        CHECK(lb == expect_lb(b, a.x), "%s: packed bit of %d -> %d", name, v, a.x);
                        CHECK(lb < L.lds_words * 32, "%s: bit outside the image", name);
                    }
                }
                // the tail: rows in LDS, entries naming tail bits or gathered words
                CHECK((int32_t)L.tail_beg.size() == C - T0 + 1 && L.tail_rp.size() == L.tail_v.size() + 1, "%s: tail",
                      name);
                for (size_t i = 0; i < L.tail_v.size(); ++i) {
                    const int32_t v = L.tail_v[i];
                    CHECK(r.cls[(size_t)v] >= T0, "%s: tail node class", name);
                    const int32_t r0 = r.rp[(size_t)v];
                    CHECK(L.tail_rp[i + 1] - L.tail_rp[i] == r.rp[(size_t)v + 1] - r0, "%s: tail row", name);
                    for (int32_t q = 0; q < L.tail_rp[i + 1] - L.tail_rp[i]; ++q) {
                        const uint32_t e = L.tail_ent[(size_t)L.tail_rp[i] + q];
                        const Edge &a = r.adj[(size_t)r0 + q];
                        const int32_t j = a.x, lb = (int32_t)(e >> 16) * 32 + (int32_t)(e & 31u);
                        CHECK(sext11(e) == a.y && lb < L.trp_off * 32, "%s: tail entry", name);
                        if (r.cls[(size_t)j] >= T0) {
                            CHECK(lb == (L.tail_off + ((j - tail_base) >> 5)) * 32 + (j & 31), "%s: tail bit", name);
                        } else {
                            const int32_t gi = lb / 32 - L.gather_off;
                            const int32_t cj = r.cls[(size_t)j];
                            CHECK(gi >= L.gat_beg[(size_t)cj] && gi < L.gat_beg[(size_t)cj + 1] &&
                                      L.gat_words[(size_t)gi] == (j >> 5) && (lb & 31) == (j & 31),
                                  "%s: gathered bit", name);
                        }
                    }
                }
            }
        }
    }
    return checked;
}

void check_validator()
{
    // a triangle 0-1-2 with unit weights as the base case
    const std::vector<int32_t> rp0 = {0, 2, 4, 6}, col0 = {1, 2, 0, 2, 0, 1}, w0 = {1, 1, 1, 1, 1, 1};
    int64_t mw = 0;
    int32_t md = 0;
    std::string err;
    CHECK(validate_csr(rp0.data(), col0.data(), w0.data(), 3, &mw, &md, &err) == GDI_OK && mw == 2 && md == 2,
          "triangle");
    struct Bad {
        const char *what;
        std::vector<int32_t> rp, col, w;
        int32_t n;
        int code;
    };
    const std::vector<Bad> bad = {
        {"n < 2", {0, 0}, {}, {}, 1, GDI_EINVAL},
        {"row_ptr[0]", {1, 2, 4, 6}, col0, w0, 3, GDI_EINVAL},
        {"decreasing", {0, 3, 2, 6}, col0, w0, 3, GDI_EINVAL},
        {"column range", rp0, {1, 3, 0, 2, 0, 1}, w0, 3, GDI_EINVAL},
        {"negative column", rp0, {-1, 2, 0, 2, 0, 1}, w0, 3, GDI_EINVAL},
        {"self-loop", rp0, {0, 2, 0, 2, 0, 1}, w0, 3, GDI_EINVAL},
        {"unsorted", rp0, {2, 1, 0, 2, 0, 1}, w0, 3, GDI_EINVAL},
        {"duplicate", {0, 2, 3, 4}, {1, 1, 0, 0}, {1, 1, 1, 1}, 3, GDI_EINVAL},
        {"no mirror", {0, 2, 3, 4}, {1, 2, 0, 1}, {1, 1, 1, 1}, 3, GDI_EINVAL},
        {"mirror weight", rp0, col0, {1, 1, 2, 1, 1, 1}, 3, GDI_EINVAL},
        {"weight sum", {0, 2, 4, 6}, col0, {1 << 30, 1, 1 << 30, 1, 1, 1}, 3, GDI_ERANGE},
    };
    for (const Bad &b : bad) {
        const int rc = validate_csr(b.rp.data(), b.col.data(), b.w.data(), b.n, &mw, &md, &err);
        CHECK(rc == b.code, "validator case '%s' returned %d", b.what, rc);
        CHECK(!err.empty(), "validator case '%s' left no message", b.what);
    }
    CHECK(validate_csr(nullptr, col0.data(), w0.data(), 3, &mw, &md, &err) == GDI_EINVAL, "NULL row_ptr");
}

}  // namespace

int main()
{
    check_validator();
    long checked = 0;
    checked += check_layouts(er(300, 0.05, 0, 1), "er300 unit");
    checked += check_layouts(er(301, 0.08, 1, 2), "er301 pm1");
    checked += check_layouts(er(250, 0.06, 2, 3), "er250 wide weights");
    checked += check_layouts(er(200, 0.05, 3, 4), "er200 heavy weight");
    checked += check_layouts(local(60, 2, 6, 0, 5), "local60 hubs");
    checked += check_layouts(local(45, 1, 0, 1, 6), "local45 pm1");
    checked += check_layouts(local(90, 3, 12, 2, 7), "local90 hubs wide");
    checked += check_layouts(from_edges(2, {{0, 1}}, {1}), "single edge");
    checked += check_layouts(from_edges(5, {}, {}), "no edges");
    std::printf("OK %ld\n", checked);
    return 0;
}
