// gdi_layout.cpp -- host-only graph preparation (see gdi_layout.h). Plain C++17, no HIP.

#include "gdi_layout.h"

#include <algorithm>
#include <climits>
#include <cstdlib>
#include <cstring>
#include <utility>

#include "../../include/gdi.h"

int gdi_halo_lds_bytes(int32_t lds_words, int32_t C, int32_t thr_words)
{
    return lds_words * 4 + C * (int)sizeof(GdiHaloEntry) + C * 8 + thr_words * 4;
}

namespace gdi_layout {

static_assert(sizeof(Edge) == 8, "Edge must match the device's int2 entry");

namespace {

int fail(int code, std::string *err, const std::string &msg)
{
    if (err) *err = msg;
    return code;
}

}  // namespace

int validate_csr(const int32_t *rp, const int32_t *col, const int32_t *w, int32_t n, int64_t *max_wdeg,
                 int32_t *max_deg, std::string *err)
{
    if (!rp || !col || !w) return fail(GDI_EINVAL, err, "NULL CSR array");
    if (n < 2) return fail(GDI_EINVAL, err, "n must be >= 2");
    if (rp[0] != 0) return fail(GDI_EINVAL, err, "row_ptr[0] must be 0");
    for (int32_t i = 0; i < n; ++i)
        if (rp[i + 1] < rp[i]) return fail(GDI_EINVAL, err, "row_ptr is decreasing at row " + std::to_string(i));
    int64_t mw = 0;
    int32_t md = 0;
    for (int32_t i = 0; i < n; ++i) {
        int64_t s = 0;
        for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
            const int32_t j = col[k];
            if (j < 0 || j >= n) return fail(GDI_EINVAL, err, "column out of range in row " + std::to_string(i));
            if (j == i) return fail(GDI_EINVAL, err, "self-loop at node " + std::to_string(i));
            if (k > rp[i] && col[k - 1] >= j)
                return fail(GDI_EINVAL, err, "columns not strictly increasing (or duplicate) in row " + std::to_string(i));
            s += std::llabs((long long)w[k]);
        }
        if (s > (int64_t(1) << 30))
            return fail(GDI_ERANGE, err, "sum of |weights| exceeds 2^30 at node " + std::to_string(i));
        mw = std::max(mw, s);
        md = std::max(md, rp[i + 1] - rp[i]);
    }
    // symmetry: every (i, j, w) has its mirror (j, i, w); rows are sorted, so binary search
    for (int32_t i = 0; i < n; ++i) {
        for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
            const int32_t j = col[k];
            const int32_t *b = col + rp[j], *e = col + rp[j + 1];
            const int32_t *f = std::lower_bound(b, e, i);
            if (f == e || *f != i)
                return fail(GDI_EINVAL, err, "edge (" + std::to_string(i) + "," + std::to_string(j) + ") has no mirror");
            if (w[f - col] != w[k])
                return fail(GDI_EINVAL, err, "edge (" + std::to_string(i) + "," + std::to_string(j) +
                                                 ") has a different mirror weight");
        }
    }
    *max_wdeg = mw;
    *max_deg = md;
    return GDI_OK;
}

// used[c] == i marks colour c as taken by an already coloured neighbour of node i.
int32_t colour_first_fit(const int32_t *rp, const int32_t *col, int32_t n, int32_t *colour)
{
    std::vector<int32_t> used((size_t)n + 1, -1);
    int32_t ncol = 0;
    for (int32_t i = 0; i < n; ++i) {
        for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
            const int32_t j = col[k];
            if (j < i) used[(size_t)colour[j]] = i;
        }
        int32_t c = 0;
        while (used[(size_t)c] == i) ++c;
        colour[i] = c;
        ncol = std::max(ncol, c + 1);
    }
    return ncol;
}

int relabel(const int32_t *rp, const int32_t *col, const int32_t *w, int32_t n, const int32_t *colour, int32_t C,
            Relabelled *out, std::string *err)
{
    Relabelled &r = *out;
    std::vector<int32_t> cnt((size_t)C, 0);
    for (int32_t i = 0; i < n; ++i) cnt[(size_t)colour[i]]++;
    r.cbeg.assign((size_t)C, 0);
    r.csz = cnt;
    int64_t pos = 0;
    for (int32_t c = 0; c < C; ++c) {
        r.cbeg[(size_t)c] = (int32_t)pos;
        pos += cnt[(size_t)c];
        pos = (pos + GDI_CLASS_ALIGN - 1) / GDI_CLASS_ALIGN * GDI_CLASS_ALIGN;
    }
    if (pos > INT32_MAX - 1) return fail(GDI_ERANGE, err, "padded node count exceeds int32");
    r.n_pad = (int32_t)pos;
    std::vector<int32_t> inv((size_t)n);
    r.orig.assign((size_t)r.n_pad, -1);
    std::vector<int32_t> fillc((size_t)C, 0);
    for (int32_t i = 0; i < n; ++i) {
        const int32_t c = colour[i];
        const int32_t v = r.cbeg[(size_t)c] + fillc[(size_t)c]++;
        inv[(size_t)i] = v;
        r.orig[(size_t)v] = i;
    }
    r.rp.assign((size_t)r.n_pad + 1, 0);
    for (int32_t v = 0; v < r.n_pad; ++v) {
        const int32_t o = r.orig[(size_t)v];
        r.rp[(size_t)v + 1] = r.rp[(size_t)v] + (o >= 0 ? rp[o + 1] - rp[o] : 0);
    }
    r.adj.assign((size_t)rp[n], Edge{0, 0});
    std::vector<std::pair<int32_t, int32_t>> row;
    for (int32_t v = 0; v < r.n_pad; ++v) {
        const int32_t o = r.orig[(size_t)v];
        if (o < 0) continue;
        row.clear();
        for (int32_t k = rp[o]; k < rp[o + 1]; ++k) row.emplace_back(inv[(size_t)col[k]], w[k]);
        std::sort(row.begin(), row.end());
        const int64_t base = r.rp[(size_t)v];
        for (size_t q = 0; q < row.size(); ++q) r.adj[(size_t)base + q] = Edge{row[q].first, row[q].second};
    }
    r.cls.assign((size_t)r.n_pad, -1);
    for (int32_t c = 0; c < C; ++c)
        for (int32_t k = 0; k < r.csz[(size_t)c]; ++k) r.cls[(size_t)(r.cbeg[(size_t)c] + k)] = c;
    return GDI_OK;
}

int pack_rows8(const Relabelled &g, PackedRows *out, std::string *err)
{
    const int32_t np = g.n_pad;
    if (np >= 32767) {
        if (err) *err = "packed rows need n_pad < 32767";
        return -1;
    }
    for (const Edge &e : g.adj)
        if (e.y != 1 && e.y != -1) {
            if (err) *err = "packed rows need weights +-1";
            return -1;
        }
    PackedRows r;
    r.prow.assign((size_t)np + 1, 0);
    uint64_t chunks = 0;
    for (int32_t v = 0; v < np; ++v) {
        r.prow[(size_t)v] = (uint32_t)chunks;
        const int64_t len = (int64_t)g.rp[(size_t)v + 1] - g.rp[(size_t)v];
        chunks += (uint64_t)((len + GDI_P8_ENTRIES - 1) / GDI_P8_ENTRIES);
        if (chunks >= 0xFFFFFFFFull) {
            if (err) *err = "packed rows: too many chunks";
            return -1;
        }
    }
    r.prow[(size_t)np] = (uint32_t)chunks;
    r.pent.assign((size_t)std::max<uint64_t>(chunks, 1) * GDI_P8_ENTRIES, (uint16_t)np);
    for (int32_t v = 0; v < np; ++v) {
        size_t q = (size_t)r.prow[(size_t)v] * GDI_P8_ENTRIES;
        for (int32_t k = g.rp[(size_t)v]; k < g.rp[(size_t)v + 1]; ++k, ++q) {
            const Edge &e = g.adj[(size_t)k];
            r.pent[q] = (uint16_t)((uint32_t)e.x | (e.y < 0 ? 0x8000u : 0u));
        }
    }
    *out = std::move(r);
    return 0;
}

int halo_layout(const Relabelled &g, int32_t C, int32_t G, int lds_budget, int32_t T0, int32_t lead, HaloLayout *out,
                std::string *err)
{
    HaloLayout &L = *out;
    L = HaloLayout{};
    L.T0 = T0;
    L.unit_w = 1;
    for (const Edge &e : g.adj) {
        if (e.y < -GDI_HALO_WMAX - 1 || e.y > GDI_HALO_WMAX) {
            L.status = -3;  // weights beyond the packed entries' range
            return GDI_OK;
        }
        if (e.y != 1) L.unit_w = 0;
    }
    const int32_t Gw = G - lead;  // blocks holding nodes
    std::vector<int32_t> blk_of_q((size_t)Gw);
    for (int32_t b = lead; b < G; ++b) blk_of_q[(size_t)chunk_of_block(b, G, lead)] = b;
    // Chunk q of class c is [bnd(c, q), bnd(c, q + 1)) in class order, with bnd(c, q) =
    // 64 * round(q * csz / (64 Gw)): every chunk q covers the same fraction of its class,
    // and classes of a colouring in ascending id spread alike over the id order, so the
    // nodes a workgroup owns in different classes lie in the same part of the graph and
    // its foreign words stay few. Interior bounds are multiples of 64 (a packed
    // spin word never has two owners); chunks hold floor or ceil of csz / Gw rounded to 64.
    auto bnd = [&](int32_t c, int64_t q) -> int64_t {
        const int64_t sz = g.csz[(size_t)c];
        if (q >= Gw) return sz;
        const int64_t units = (sz + GDI_CLASS_ALIGN - 1) / GDI_CLASS_ALIGN;
        return std::min<int64_t>(sz, (q * units * 2 + Gw) / (2 * (int64_t)Gw) * GDI_CLASS_ALIGN);
    };
    const size_t GC = (size_t)G * (size_t)C;
    std::vector<GdiHaloEntry> &tab = L.tab;
    tab.assign(GC, GdiHaloEntry{});
    std::vector<int32_t> own((size_t)g.n_pad, -1);  // owner block of every node of a grid class
    for (int32_t b = 0; b < G; ++b) {
        const int32_t q = chunk_of_block(b, G, lead);
        for (int32_t c = 0; c < C; ++c) {
            GdiHaloEntry &e = tab[(size_t)b * C + c];
            std::memset(&e, 0, sizeof(e));
            if (c >= T0 || q < 0) continue;  // tail classes and dedicated leaders: no own chunks
            const int64_t lo = (int64_t)g.cbeg[(size_t)c] + bnd(c, q);
            const int64_t hi = (int64_t)g.cbeg[(size_t)c] + bnd(c, (int64_t)q + 1);
            e.node_lo = e.node_hi = (int32_t)lo;
            if (lo < hi) {
                e.node_hi = (int32_t)hi;
                for (int64_t v = lo; v < hi; ++v) own[(size_t)v] = b;
            }
        }
    }
    auto owner = [&](int32_t v) { return own[(size_t)v]; };
    // gather lists: the packed words of classes < T0 that tail nodes read; foreign
    // lists: per (workgroup, class), the packed words of that class its nodes read and
    // it does not own (an own chunk's words hold only its nodes and padding, since
    // interior chunk bounds are multiples of 64)
    std::vector<std::vector<int32_t>> gat((size_t)T0), fw(GC);
    for (int32_t v = 0; v < g.n_pad; ++v) {
        const int32_t cv = g.cls[(size_t)v];
        if (cv < 0) continue;
        for (int32_t k = g.rp[(size_t)v]; k < g.rp[(size_t)v + 1]; ++k) {
            const int32_t j = g.adj[(size_t)k].x;
            const int32_t cj = g.cls[(size_t)j];
            if (cj >= T0) continue;  // tail neighbours live in the tail region
            if (cv >= T0) {
                gat[(size_t)cj].push_back(j >> 5);
                continue;
            }
            const int32_t b = owner(v);
            if (owner(j) != b) fw[(size_t)b * C + cj].push_back(j >> 5);
        }
    }
    std::vector<int32_t> &gat_beg = L.gat_beg, &gat_words = L.gat_words;
    gat_beg.assign((size_t)T0 + 1, 0);
    for (int32_t c = 0; c < T0; ++c) {
        std::vector<int32_t> &W = gat[(size_t)c];
        std::sort(W.begin(), W.end());
        W.erase(std::unique(W.begin(), W.end()), W.end());
        gat_words.insert(gat_words.end(), W.begin(), W.end());
        gat_beg[(size_t)c + 1] = (int32_t)gat_words.size();
    }
    // image per workgroup: for each class its own chunk's words, then copies of its
    // foreign words; every workgroup's image is laid out from LDS word 0
    int32_t lds_words = 0, flist_max = 0;
    std::vector<int32_t> list_pos(GC, 0);  // position of each (b, c) list in the block's list
    for (int32_t b = 0; b < G; ++b) {
        int32_t off = 0, lpos = 0;
        for (int32_t c = 0; c < C; ++c) {
            const size_t i = (size_t)b * C + c;
            GdiHaloEntry &e = tab[i];
            std::vector<int32_t> &W = fw[i];
            std::sort(W.begin(), W.end());
            W.erase(std::unique(W.begin(), W.end()), W.end());
            e.own_off = off;
            off += e.node_hi > e.node_lo ? ((e.node_hi + 31) >> 5) - (e.node_lo >> 5) : 0;
            e.for_off = off;
            e.for_len = (int32_t)W.size();
            off += e.for_len;
            list_pos[i] = lpos;
            lpos += e.for_len;
        }
        lds_words = std::max(lds_words, off);
        flist_max = std::max(flist_max, lpos);
    }
    const int32_t tail_base = T0 < C ? g.cbeg[(size_t)T0] : g.n_pad;  // multiple of 64
    int32_t tail_n = 0, tail_nnz = 0;
    for (int32_t c = T0; c < C; ++c) {
        tail_n += g.csz[(size_t)c];
        for (int32_t v = g.cbeg[(size_t)c]; v < g.cbeg[(size_t)c] + g.csz[(size_t)c]; ++v)
            tail_nnz += g.rp[(size_t)v + 1] - g.rp[(size_t)v];
    }
    // LDS: images | gather words | tail spin bits | tail row offsets | tail entries |
    // foreign word ids | overflow entries
    const int32_t gather_off = lds_words;
    const int32_t tail_off = gather_off + (int32_t)gat_words.size();
    const int32_t trp_off = tail_off + (g.n_pad - tail_base) / 32;
    const int32_t tent_off = (trp_off + (T0 < C ? tail_n + 1 : 0) + 1) & ~1;  // 8-byte aligned
    lds_words = tent_off + 2 * tail_nnz;
    const int32_t list_off = lds_words;
    lds_words += flist_max;
    // (packed entries hold LDS word indices in 16 bits)
    if (gdi_halo_lds_bytes(lds_words, C, 0) > lds_budget || lds_words > 65536) {
        L.status = -2;
        return GDI_OK;
    }
    auto tail_lb = [&](int32_t j) { return (tail_off + ((j - tail_base) >> 5)) * 32 + (j & 31); };
    auto gather_lb = [&](int32_t j) {
        const int32_t c = g.cls[(size_t)j];
        const auto b0 = gat_words.begin() + gat_beg[(size_t)c], b1 = gat_words.begin() + gat_beg[(size_t)c + 1];
        const auto it = std::lower_bound(b0, b1, j >> 5);
        if (it == b1 || *it != (j >> 5)) return -1;  // rejected by the range check below
        return (gather_off + (int32_t)(it - gat_words.begin())) * 32 + (j & 31);
    };
    L.tail_beg.assign((size_t)(C - T0) + 1, 0);
    L.tail_rp.assign(1, 0);
    for (int32_t c = T0; c < C; ++c) {
        for (int32_t v = g.cbeg[(size_t)c]; v < g.cbeg[(size_t)c] + g.csz[(size_t)c]; ++v) {
            L.tail_v.push_back(v);
            for (int32_t k = g.rp[(size_t)v]; k < g.rp[(size_t)v + 1]; ++k) {
                const int32_t j = g.adj[(size_t)k].x;
                const int32_t lb = g.cls[(size_t)j] >= T0 ? tail_lb(j) : gather_lb(j);
                if (lb < 0 || lb >= trp_off * 32) return fail(GDI_EDEVICE, err, "internal error: tail index out of range");
                L.tail_ent.push_back(pack_entry(lb, g.adj[(size_t)k].y));
            }
            L.tail_rp.push_back((int32_t)L.tail_ent.size());
        }
        L.tail_beg[(size_t)(c - T0) + 1] = (int32_t)L.tail_v.size();
    }
    // after the last row: GDI_HALO_PF zero entries; the sweep reads GDI_HALO_PF entries
    // from any row start, so these keep it in bounds
    std::vector<uint32_t> &adjL = L.adjL;
    adjL.assign(g.adj.size() + GDI_HALO_PF, 0u);
    for (int32_t v = 0; v < g.n_pad; ++v) {
        const int32_t cv = g.cls[(size_t)v];
        if (cv < 0) continue;
        const int32_t b = cv < T0 ? owner(v) : -1;
        for (int32_t k = g.rp[(size_t)v]; k < g.rp[(size_t)v + 1]; ++k) {
            const int32_t j = g.adj[(size_t)k].x;
            const int32_t cj = g.cls[(size_t)j];
            int32_t lb;
            if (cj >= T0) {
                lb = tail_lb(j);
            } else if (cv >= T0) {
                lb = gather_lb(j);
            } else {
                const size_t i = (size_t)b * C + cj;
                const GdiHaloEntry &e = tab[i];
                if (owner(j) == b) {
                    lb = (e.own_off + (j >> 5) - (e.node_lo >> 5)) * 32 + (j & 31);
                } else {
                    const auto it = std::lower_bound(fw[i].begin(), fw[i].end(), j >> 5);
                    lb = (it == fw[i].end() || *it != (j >> 5)) ? -1
                                                                : (e.for_off + (int32_t)(it - fw[i].begin())) * 32 + (j & 31);
                }
            }
            // every index must land inside this workgroup's LDS image (checked here so
            // that a layout error surfaces as an error code, never as a device fault)
            if (lb < 0 || lb >= lds_words * 32) return fail(GDI_EDEVICE, err, "internal error: halo index out of range");
            adjL[(size_t)k] = pack_entry(lb, g.adj[(size_t)k].y);
        }
    }
    // Rows longer than GDI_HALO_PF keep their entries from GDI_HALO_PF - 1 on in an
    // overflow region at the end of the owner workgroup's LDS image, and the row's entry
    // GDI_HALO_PF - 1 then holds the LDS word where they start, so that no row needs a
    // second trip to memory. Only when every workgroup's region fits beside its image;
    // otherwise the sweep reads those entries from the packed CSR.
    std::vector<std::vector<uint32_t>> ovf((size_t)G);
    std::vector<std::pair<size_t, int32_t>> links;  // (entry index, position in the owner's region)
    for (int32_t v = 0; v < g.n_pad; ++v) {
        const int32_t cv = g.cls[(size_t)v];
        const int32_t r0 = g.rp[(size_t)v], r1 = g.rp[(size_t)v + 1];
        if (cv < 0 || cv >= T0 || r1 - r0 <= GDI_HALO_PF) continue;
        std::vector<uint32_t> &O = ovf[(size_t)owner(v)];
        links.emplace_back((size_t)r0 + GDI_HALO_PF - 1, (int32_t)O.size());
        O.insert(O.end(), adjL.begin() + r0 + GDI_HALO_PF - 1, adjL.begin() + r1);
    }
    int64_t ovf_max = 0;
    for (const auto &O : ovf) ovf_max = std::max<int64_t>(ovf_max, (int64_t)O.size());
    int32_t ovf_len = 0;
    const int32_t ovf_off = lds_words;
    if (ovf_max > 0 && ovf_max < INT32_MAX / 8 && gdi_halo_lds_bytes(lds_words + (int32_t)ovf_max, C, 0) <= lds_budget) {
        ovf_len = (int32_t)ovf_max;
        lds_words += ovf_len;
        for (const auto &l : links) adjL[l.first] = (uint32_t)(ovf_off + l.second);
    }
    L.flist_len = flist_max;
    L.flist.assign((size_t)G * (size_t)flist_max, 0);
    for (int32_t b = 0; b < G; ++b)
        for (int32_t c = 0; c < C; ++c) {
            const size_t i = (size_t)b * C + c;
            tab[i].list_off = list_off + list_pos[i];
            std::copy(fw[i].begin(), fw[i].end(), L.flist.begin() + (size_t)b * flist_max + list_pos[i]);
        }
    L.list_off = list_off;
    L.ovf.assign((size_t)G * (size_t)ovf_len, 0u);
    for (int32_t b = 0; b < G && ovf_len > 0; ++b)
        std::copy(ovf[(size_t)b].begin(), ovf[(size_t)b].end(), L.ovf.begin() + (size_t)b * ovf_len);
    L.lds_words = lds_words;
    L.gather_off = gather_off;
    L.tail_off = tail_off;
    L.trp_off = trp_off;
    L.tent_off = tent_off;
    L.ovf_off = ovf_off;
    L.ovf_len = ovf_len;
    return GDI_OK;
}

}  // namespace gdi_layout
