// gdi_host.cpp -- host side of the GDI annealer library (C ABI in include/gdi.h).
//
// Responsibilities: CSR validation (before any device call), first-fit greedy
// colouring in ascending node id, colour-major relabelling with 64-aligned class
// starts, FP64 -> uint32 Metropolis threshold tables, device buffers, launch
// selection (workgroup or grid scope) and result transfer. No exception crosses
// the C ABI.

#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/gdi.h"
#include "gdi_internal.h"
#include "gdi_tunecache.h"

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

int hip_fail(hipError_t e, const char *what)
{
    return fail(e == hipErrorOutOfMemory ? GDI_ENOMEM : GDI_EDEVICE,
                std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(expr, what)                                   \
    do {                                                      \
        hipError_t e_ = (expr);                               \
        if (e_ != hipSuccess) return hip_fail(e_, (what));    \
    } while (0)

// Fault injection for testing the GDI_ENOMEM paths: with the environment variable
// GDI_FAULT set to "alloc", every device allocation the library attempts fails as if
// the device were out of memory (read at each allocation).
inline bool alloc_fault()
{
    const char *f = std::getenv("GDI_FAULT");
    return f && std::strcmp(f, "alloc") == 0;
}

template <typename T>
struct DevBuf {
    T *p = nullptr;
    size_t n = 0;
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
    // grow-only allocation of at least count elements
    hipError_t reserve(size_t count)
    {
        if (count <= n && p) return hipSuccess;
        release();
        if (alloc_fault()) return hipErrorOutOfMemory;
        void *q = nullptr;
        hipError_t e = hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(T));
        if (e != hipSuccess) return e;
        p = static_cast<T *>(q);
        n = count;
        return hipSuccess;
    }
};

}  // namespace

struct gdi_graph {
    int32_t n = 0, n_pad = 0, C = 0;
    int64_t nnz = 0;
    int64_t max_abs_wdeg = 0;
    int32_t max_degree = 0;
    int32_t wkind = 0;                // 2: every weight +1; 1: every weight +-1; 0: general
    std::vector<int32_t> colour;      // original order
    gdi_layout::Relabelled rl;        // colour-major relabelling; new-id CSR kept for launch layouts

    // halo layout for one grid size (k_sweep_halo)
    int32_t halo_G = 0, halo_nwork = 0, halo_lead = 0;
    int32_t halo_lds_words = -1;      // -1: not built; -2: does not fit LDS; -3: weights too large
    int32_t halo_T0 = 0, halo_tail_n = 0, halo_gather_off = 0, halo_tail_off = 0;
    int32_t halo_tail_nnz = 0, halo_trp_off = 0, halo_tent_off = 0;
    DevBuf<uint32_t> d_adjL;
    DevBuf<int32_t> d_tail_v, d_tail_beg, d_gat_words, d_gat_beg, d_tail_rp;
    DevBuf<uint32_t> d_tail_ent;
    int32_t halo_ovf_off = 0, halo_ovf_len = 0, halo_unit_w = 0;
    int32_t halo_list_off = 0, halo_flist_len = 0;
    // epochs of the packed spin, member and group words: the next launch's base, and
    // whether the words hold only epochs below it (false after they are allocated)
    uint32_t halo_epoch = 0;
    bool halo_words_clean = false;
    DevBuf<uint32_t> d_ovf;
    DevBuf<int32_t> d_flist;
    DevBuf<GdiHaloEntry> d_tab;
    DevBuf<uint64_t> d_words, d_member, d_group;

    DevBuf<int32_t> d_rp, d_orig, d_cbeg, d_csz, d_P;
    // 16-bit copies of the relabelled CSR for the LDS-resident workgroup sweep (graphs with
    // n_pad <= 32768, nnz <= 65535 and +-1 weights; wgl_ok)
    bool wgl_ok = false;
    DevBuf<uint16_t> d_rp16, d_ent16;
    DevBuf<int2> d_adj;
    DevBuf<int8_t> d_spin, d_io;
    DevBuf<uint32_t> d_bits;          // bit-packed spins for the from-scratch cut's neighbour reads
    DevBuf<int64_t> d_state, d_red, d_trace;
    DevBuf<uint32_t> d_thr;
    DevBuf<uint64_t> d_bar;

    std::vector<double> thr_key;      // temperatures of the cached table
    int32_t thr_K = -1;
    int64_t thr_demax = -1;
    uint32_t thr_rule = 0;

    hipStream_t stream = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    gdi_tuning tune{};
    bool have_tune = false;

    // last run
    bool pending = false;
    int64_t last_cut0 = 0;
    gdi_result last{};
    bool last_valid = false;

    ~gdi_graph()
    {
        d_rp.release(); d_orig.release(); d_cbeg.release(); d_csz.release(); d_P.release();
        d_rp16.release(); d_ent16.release();
        d_adj.release(); d_spin.release(); d_io.release(); d_state.release(); d_red.release(); d_bits.release();
        d_trace.release(); d_thr.release(); d_bar.release();
        d_adjL.release(); d_tail_v.release(); d_tail_beg.release(); d_gat_words.release(); d_gat_beg.release();
        d_tail_rp.release(); d_tail_ent.release(); d_ovf.release(); d_flist.release();
        d_tab.release(); d_words.release(); d_member.release(); d_group.release();
        if (ev0) (void)hipEventDestroy(ev0);
        if (ev1) (void)hipEventDestroy(ev1);
    }
};

namespace {

// ------------------------------------------------------------------ validation
int validate_csr(const int32_t *rp, const int32_t *col, const int32_t *w, int32_t n, int64_t *max_wdeg,
                 int32_t *max_deg)
{
    std::string msg;
    const int rc = gdi_layout::validate_csr(rp, col, w, n, max_wdeg, max_deg, &msg);
    return rc ? fail(rc, msg) : GDI_OK;
}

uint32_t threshold_of(int64_t d, double T)
{
    const double v = std::floor(std::ldexp(std::exp(-(double)d / T), 32));
    if (v >= 4294967295.0) return 0xFFFFFFFFu;
    if (v <= 0.0) return 0u;
    return (uint32_t)v;
}

struct Choice {
    uint32_t scope, block, grid, lanes;
    bool spins_lds;
    bool csr_lds;  // workgroup scope with the whole graph in LDS (k_sweep_wgl)
};

int lanes_for_degree(double avg_deg)
{
    int L = 1;
    while (L < 32 && 2.0 * L < avg_deg) L *= 2;
    return L;
}

// Lanes per node of the workgroup-scope phase loop (plain, batched and cluster
// members): enough subgroups to take a class's nodes -- the average class, or a
// member's share of it -- in one round where the block allows (a phase is a chain of
// dependent loads, so nodes in flight matter more than lanes per row), and never more
// lanes than the mean degree asks for. Measured on MI355X with 1024-thread blocks:
// er2000 47.8 -> 25.2 us per sweep, torus100 28.1 -> 15.4, an 8000-node RGG 89 -> 44.
int lanes_for_wg(const gdi_graph *g, uint32_t nth, int32_t members)
{
    const int Ld = lanes_for_degree(g->n ? (double)g->nnz / g->n : 0.0);
    const double per_round = g->n ? (double)nth * (double)g->C * (double)members / (double)g->n : 64.0;
    int Lc = 1;
    while (Lc < 64 && 2.0 * Lc <= per_round) Lc *= 2;
    return std::min(Ld, Lc);
}

const int64_t kSpinLimit = int64_t(1) << 22;
const int32_t kWgMaxNodes = 65536;
// Automatic scope: one workgroup up to this many padded nodes, the halo grid sweep
// above (measured on MI355X, 300 sweeps: RGGs of mean degree 10 with 14-15 classes,
// workgroup / best halo grid: 3000 nodes 30.7 / 35.1 us per sweep, 5000 33.7 / 37.4,
// 8000 45.5 / 38.2, 12000 54.6 / 38.7, 20000 72.6 / 40.9). Graphs the halo sweep does
// not take (weights beyond its packed range, LDS) stay on one workgroup up to
// kWgMaxNodes padded nodes.
const int32_t kWgAutoNodes = 6144;

int build_halo(gdi_graph *g, int32_t G, int lds_budget, int32_t nwork, int32_t lead);

// one_wg: the automatic scope takes one workgroup whenever the graph has at most
// kWgMaxNodes padded nodes (the standard solver runs on one workgroup only)
int pick_launch(gdi_graph *g, Choice *ch, bool one_wg)
{
    const gdi_tuning t = g->have_tune ? g->tune : gdi_tuning{};
    const double avg = g->n ? (double)g->nnz / g->n : 0.0;
    ch->lanes = t.lanes_per_node ? t.lanes_per_node : (uint32_t)lanes_for_degree(avg);
    if (ch->lanes == 0 || ch->lanes > 64 || (ch->lanes & (ch->lanes - 1)))
        return fail(GDI_EINVAL, "lanes_per_node must be a power of two in [1, 64]");
    ch->block = t.block ? t.block : 1024u;
    if (ch->block < 64 || ch->block > GDI_MAX_BLOCK || ch->block % 64 || ch->block < ch->lanes)
        return fail(GDI_EINVAL, "block must be a multiple of 64 in [64, 1024]");
    ch->scope = t.scope ? t.scope
                        : (g->n_pad <= (one_wg ? kWgMaxNodes : kWgAutoNodes) ? GDI_SCOPE_WORKGROUP : GDI_SCOPE_GRID);
    if (ch->scope < GDI_SCOPE_WORKGROUP || ch->scope > GDI_SCOPE_GRID_FENCED)
        return fail(GDI_EINVAL, "unknown scope");
    ch->grid = 1;
    ch->spins_lds = false;
    ch->csr_lds = false;
    int dev = 0, lds_max = 0, cus = 0;
    HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
    HIP_TRY(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev), "hipDeviceGetAttribute");
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev), "hipDeviceGetAttribute");
    auto pick_wg = [&]() -> int {
        ch->scope = GDI_SCOPE_WORKGROUP;
        ch->grid = 1;
        if (!t.lanes_per_node) ch->lanes = (uint32_t)lanes_for_wg(g, ch->block, 1);
        // beside the dynamic part: the kernel's own LDS words and two threshold rows
        const int fixed = 64 + 2 * GDI_WG_THR_MAX * 4;
        ch->spins_lds = gdi_wg_lds_bytes(g->n_pad, g->C, 1) + fixed <= lds_max;
        if (gdi_wg_lds_bytes(g->n_pad, g->C, 0) + fixed > lds_max)
            return fail(GDI_ERANGE, "too many colour classes for one workgroup's LDS");
        // the whole graph in LDS when it fits (+-1 weights, 16-bit CSR)
        const bool wgl_fits = g->wgl_ok && gdi_wgl_lds_bytes(g->n_pad, g->C, (int32_t)g->nnz) + fixed <= lds_max;
        if (t.csr_lds > 0 && !wgl_fits)
            return fail(GDI_ERANGE, "the graph does not fit one workgroup's LDS as a 16-bit CSR "
                                    "(needs n_pad <= 32768, nnz <= 65535, weights +-1)");
        ch->csr_lds = wgl_fits && t.csr_lds >= 0;
        return GDI_OK;
    };
    if (ch->scope == GDI_SCOPE_WORKGROUP) return pick_wg();
    if (ch->scope == GDI_SCOPE_GRID) {
        // fence-free halo sweep: one node per thread, 1024-thread workgroups, grid a multiple of 8
        const uint32_t block = t.block ? t.block : 1024u;
        // automatic grid: about 1,500 nodes per workgroup, at most one workgroup per CU,
        // and at least 64 workgroups (fewer when that leaves under 128 nodes each)
        // (measured on RGGs: 128 and 256 workgroups are fastest at 2e5 and 1e6 nodes,
        // 64 from 1e4 to 6.4e4 nodes)
        const int64_t g_cap = (int64_t)std::min(cus, GDI_HALO_MAX_GRID) / 8 * 8;
        const int64_t g_small = std::min<int64_t>(64, g->n / 128 / 8 * 8);
        uint32_t G = t.grid ? t.grid
                            : (uint32_t)std::max<int64_t>(
                                  8, std::min<int64_t>(g_cap, std::max<int64_t>(g_small, g->n / 1536 / 8 * 8)));
        if (block < 256) return fail(GDI_EINVAL, "the grid sweep needs at least 256 threads per workgroup");
        if (G < 8 || G % 8 || G > GDI_HALO_MAX_GRID)
            return fail(GDI_EINVAL, "the grid sweep needs a grid that is a multiple of 8 in [8, 512]");
        const int32_t nwork = (int32_t)block - 64;  // worker threads: all but the barrier wave
        // the redundant tail (its gather words read a phase late) saves its classes'
        // grid barriers but every workgroup reads every gather word: on by default
        // (measured with the foreign-word layout: 108.3 -> 104.9 ms on a 1e6-node RGG at
        // 256 workgroups; 5-9 % faster on a 2e5-node RGG at 128); tail_max < 0 turns it off
        const int32_t tail_auto = nwork;
        const int32_t tail_cap = t.tail_max < 0 ? 0 : (t.tail_max == 0 ? tail_auto : std::min(t.tail_max, nwork));
        // dedicated group leaders: blocks 0..7 hold no nodes (automatic: on grids of 64 or
        // more workgroups; measured 105.9 -> 104.8 ms on the 1e6-node RGG at 256, and
        // chosen by the autotuner on 1e4..6.4e4-node RGGs at 32 and 64)
        const int32_t lead = t.leaders > 0 ? 8 : (t.leaders < 0 ? 0 : (G >= 64 ? 8 : 0));
        if (lead && G < 16) return fail(GDI_EINVAL, "dedicated leaders need a grid of at least 16 workgroups");
        int rc = build_halo(g, (int32_t)G, lds_max - 256, tail_cap, lead);
        if (rc) return rc;
        if (g->halo_lds_words >= 0) {
            int cap = 0;
            // without the threshold rows: they are staged in LDS only when they fit beside the image
            int e = gdi_halo_capacity((int)block, gdi_halo_lds_bytes(g->halo_lds_words, g->C, 0), &cap);
            if (e) return fail(GDI_EDEVICE, std::string("occupancy query: ") + gdi_hip_error_string(e));
            if ((int)G > cap)
                return fail(GDI_EDEVICE, "grid of " + std::to_string(G) + " workgroups cannot be co-resident (capacity " +
                                             std::to_string(cap) + ")");
            ch->grid = G;
            ch->block = block;
            ch->lanes = 1;
            return GDI_OK;
        }
        if (t.scope == GDI_SCOPE_GRID)
            return fail(GDI_ERANGE, g->halo_lds_words == -3
                                        ? "the grid scope packs weights into 11 bits: |w| must be <= 1023"
                                        : "the spin words this graph needs per workgroup do not fit its LDS");
        // the automatic choice falls back to one workgroup where the graph fits it, else
        // to the fenced grid sweep
        if (g->n_pad <= kWgMaxNodes) {
            const int rc_wg = pick_wg();
            if (rc_wg != GDI_ERANGE) return rc_wg;
        }
        ch->scope = GDI_SCOPE_GRID_FENCED;
    }
    int cap = 0;
    int e = gdi_grid_capacity((int)ch->block, (int)ch->lanes, &cap);
    if (e) return fail(GDI_EDEVICE, std::string("occupancy query: ") + gdi_hip_error_string(e));
    uint32_t want = t.grid ? t.grid : (uint32_t)std::min(cap, cus);
    if (want < 1 || (int)want > cap)
        return fail(GDI_EDEVICE, "grid of " + std::to_string(want) + " workgroups cannot be co-resident (capacity " +
                                     std::to_string(cap) + ")");
    ch->grid = want;
    return GDI_OK;
}

int check_device()
{
    int dev = 0;
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
    HIP_TRY(hipGetDeviceProperties(&prop, dev), "hipGetDeviceProperties");
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(GDI_EDEVICE, std::string("device is ") + prop.gcnArchName + ", library is built for gfx950");
    return GDI_OK;
}

int upload(gdi_graph *g, const int32_t *rp, const int32_t *col, const int32_t *w)
{
    std::string msg;
    if (int rc = gdi_layout::relabel(rp, col, w, g->n, g->colour.data(), g->C, &g->rl, &msg)) return fail(rc, msg);
    g->n_pad = g->rl.n_pad;
    const std::vector<int32_t> &nrp = g->rl.rp;
    const std::vector<gdi_layout::Edge> &adj = g->rl.adj;
    const int32_t n = g->n;
    HIP_TRY(g->d_rp.reserve(nrp.size()), "hipMalloc row_ptr");
    HIP_TRY(g->d_adj.reserve(adj.size()), "hipMalloc adjacency");
    HIP_TRY(g->d_orig.reserve(g->rl.orig.size()), "hipMalloc orig");
    HIP_TRY(g->d_cbeg.reserve((size_t)g->C), "hipMalloc classes");
    HIP_TRY(g->d_csz.reserve((size_t)g->C), "hipMalloc classes");
    HIP_TRY(g->d_P.reserve((size_t)g->C + 2), "hipMalloc P");
    HIP_TRY(g->d_spin.reserve((size_t)g->n_pad), "hipMalloc spins");
    HIP_TRY(g->d_bits.reserve((size_t)g->n_pad / 32 + 1), "hipMalloc spins");
    HIP_TRY(g->d_io.reserve((size_t)n), "hipMalloc io");
    HIP_TRY(g->d_state.reserve(8), "hipMalloc state");
    HIP_TRY(g->d_red.reserve(4), "hipMalloc state");
    HIP_TRY(hipMemcpy(g->d_rp.p, nrp.data(), nrp.size() * 4, hipMemcpyHostToDevice), "upload row_ptr");
    if (!adj.empty())
        HIP_TRY(hipMemcpy(g->d_adj.p, adj.data(), adj.size() * sizeof(gdi_layout::Edge), hipMemcpyHostToDevice),
                "upload adjacency");
    HIP_TRY(hipMemcpy(g->d_orig.p, g->rl.orig.data(), g->rl.orig.size() * 4, hipMemcpyHostToDevice), "upload orig");
    HIP_TRY(hipMemcpy(g->d_cbeg.p, g->rl.cbeg.data(), g->rl.cbeg.size() * 4, hipMemcpyHostToDevice), "upload classes");
    HIP_TRY(hipMemcpy(g->d_csz.p, g->rl.csz.data(), g->rl.csz.size() * 4, hipMemcpyHostToDevice), "upload classes");
    g->wkind = 2;
    for (size_t k = 0; k < adj.size() && g->wkind > 0; ++k)
        g->wkind = std::min(g->wkind, adj[k].y == 1 ? 2 : (adj[k].y == -1 ? 1 : 0));
    // the LDS-resident workgroup sweep's 16-bit CSR: column | (weight < 0) << 15
    g->wgl_ok = g->n_pad <= 32768 && g->nnz <= 65535 && g->wkind > 0;
    if (g->wgl_ok) {
        std::vector<uint16_t> rp16(nrp.size()), ent16(std::max<size_t>(adj.size(), 1), 0);
        for (size_t i = 0; i < nrp.size(); ++i) rp16[i] = (uint16_t)nrp[i];
        for (size_t k = 0; k < adj.size(); ++k) ent16[k] = (uint16_t)(adj[k].x | (adj[k].y < 0 ? 0x8000 : 0));
        HIP_TRY(g->d_rp16.reserve(rp16.size()), "hipMalloc 16-bit CSR");
        HIP_TRY(g->d_ent16.reserve(ent16.size()), "hipMalloc 16-bit CSR");
        HIP_TRY(hipMemcpy(g->d_rp16.p, rp16.data(), rp16.size() * 2, hipMemcpyHostToDevice), "upload 16-bit CSR");
        HIP_TRY(hipMemcpy(g->d_ent16.p, ent16.data(), ent16.size() * 2, hipMemcpyHostToDevice), "upload 16-bit CSR");
    }
    HIP_TRY(hipEventCreate(&g->ev0), "hipEventCreate");
    HIP_TRY(hipEventCreate(&g->ev1), "hipEventCreate");
    return GDI_OK;
}

// Halo layout with the tail starting at class T0 (T0 == C: none), uploaded.
int build_halo_for(gdi_graph *g, int32_t G, int lds_budget, int32_t T0, int32_t lead)
{
    gdi_layout::HaloLayout L;
    std::string msg;
    if (int rc = gdi_layout::halo_layout(g->rl, g->C, G, lds_budget, T0, lead, &L, &msg)) return fail(rc, msg);
    g->halo_unit_w = L.unit_w;
    if (L.status) {
        g->halo_lds_words = L.status;
        return GDI_OK;
    }
    HIP_TRY(g->d_flist.reserve(std::max<size_t>(L.flist.size(), 1)), "hipMalloc halo lists");
    if (!L.flist.empty())
        HIP_TRY(hipMemcpy(g->d_flist.p, L.flist.data(), L.flist.size() * 4, hipMemcpyHostToDevice), "upload halo lists");
    HIP_TRY(g->d_ovf.reserve(std::max<size_t>(L.ovf.size(), 1)), "hipMalloc halo overflow");
    if (!L.ovf.empty())
        HIP_TRY(hipMemcpy(g->d_ovf.p, L.ovf.data(), L.ovf.size() * 4, hipMemcpyHostToDevice), "upload halo overflow");
    HIP_TRY(g->d_adjL.reserve(L.adjL.size()), "hipMalloc halo CSR");
    HIP_TRY(g->d_tab.reserve(L.tab.size()), "hipMalloc halo table");
    HIP_TRY(g->d_words.reserve((size_t)g->n_pad / 32 + 1), "hipMalloc packed spins");
    HIP_TRY(g->d_member.reserve(8 * 64), "hipMalloc barrier");
    HIP_TRY(g->d_group.reserve(2 * 8 * GDI_HALO_GROUP_PAD), "hipMalloc barrier");
    if (!L.adjL.empty())
        HIP_TRY(hipMemcpy(g->d_adjL.p, L.adjL.data(), L.adjL.size() * 4, hipMemcpyHostToDevice), "upload halo CSR");
    HIP_TRY(hipMemcpy(g->d_tab.p, L.tab.data(), L.tab.size() * sizeof(GdiHaloEntry), hipMemcpyHostToDevice),
            "upload halo table");
    HIP_TRY(g->d_tail_v.reserve(std::max<size_t>(L.tail_v.size(), 1)), "hipMalloc halo tail");
    HIP_TRY(g->d_tail_beg.reserve(L.tail_beg.size()), "hipMalloc halo tail");
    HIP_TRY(g->d_gat_words.reserve(std::max<size_t>(L.gat_words.size(), 1)), "hipMalloc halo tail");
    HIP_TRY(g->d_gat_beg.reserve(L.gat_beg.size()), "hipMalloc halo tail");
    HIP_TRY(g->d_tail_rp.reserve(L.tail_rp.size()), "hipMalloc halo tail");
    HIP_TRY(g->d_tail_ent.reserve(std::max<size_t>(L.tail_ent.size(), 1)), "hipMalloc halo tail");
    HIP_TRY(hipMemcpy(g->d_tail_rp.p, L.tail_rp.data(), L.tail_rp.size() * 4, hipMemcpyHostToDevice), "upload halo tail");
    if (!L.tail_ent.empty())
        HIP_TRY(hipMemcpy(g->d_tail_ent.p, L.tail_ent.data(), L.tail_ent.size() * 4, hipMemcpyHostToDevice),
                "upload halo tail");
    if (!L.tail_v.empty())
        HIP_TRY(hipMemcpy(g->d_tail_v.p, L.tail_v.data(), L.tail_v.size() * 4, hipMemcpyHostToDevice), "upload halo tail");
    HIP_TRY(hipMemcpy(g->d_tail_beg.p, L.tail_beg.data(), L.tail_beg.size() * 4, hipMemcpyHostToDevice),
            "upload halo tail");
    if (!L.gat_words.empty())
        HIP_TRY(hipMemcpy(g->d_gat_words.p, L.gat_words.data(), L.gat_words.size() * 4, hipMemcpyHostToDevice),
                "upload halo tail");
    HIP_TRY(hipMemcpy(g->d_gat_beg.p, L.gat_beg.data(), L.gat_beg.size() * 4, hipMemcpyHostToDevice), "upload halo tail");
    g->halo_lds_words = L.lds_words;
    g->halo_T0 = T0;
    g->halo_tail_n = (int32_t)L.tail_v.size();
    g->halo_gather_off = L.gather_off;
    g->halo_tail_off = L.tail_off;
    g->halo_tail_nnz = (int32_t)L.tail_ent.size();
    g->halo_trp_off = L.trp_off;
    g->halo_tent_off = L.tent_off;
    g->halo_ovf_off = L.ovf_off;
    g->halo_ovf_len = L.ovf_len;
    g->halo_list_off = L.list_off;
    g->halo_flist_len = L.flist_len;
    g->halo_words_clean = false;
    return GDI_OK;
}

// Builds the halo layout for grid size G: own chunks, foreign words of the packed spin
// array per (workgroup, class), LDS offsets and the CSR with LDS bit indices.
// Classes T0..C-1 form the redundant tail when they hold at most nwork nodes.
int build_halo(gdi_graph *g, int32_t G, int lds_budget, int32_t nwork, int32_t lead)
{
    if (g->halo_G == G && g->halo_nwork == nwork && g->halo_lead == lead && g->halo_lds_words != -1) return GDI_OK;
    // a rebuild reallocates the layout's buffers: the old layout is invalid from here on,
    // also if the rebuild fails
    g->halo_G = 0;
    g->halo_lds_words = -1;
    const int32_t C = g->C;
    int32_t T0 = C;
    int64_t tail_n = 0;
    // at least three classes stay outside the tail: the gathered words of class c are
    // read in the phase of class c + 1 (those of the last grid class before the tail),
    // and are then republished only after a grid barrier that follows every
    // workgroup's read of them
    while (T0 > 3 && tail_n + g->rl.csz[(size_t)T0 - 1] <= nwork) tail_n += g->rl.csz[(size_t)--T0];
    for (;;) {
        int rc = build_halo_for(g, G, lds_budget, T0, lead);
        if (rc) return rc;
        if (g->halo_lds_words != -2 || T0 == C) break;
        ++T0;  // the tail's regions do not fit: a shorter tail
    }
    g->halo_G = G;
    g->halo_nwork = nwork;
    g->halo_lead = lead;
    return GDI_OK;
}

// Metropolis threshold table for a schedule: rows t < S, entries d = 0..K where K is
// the largest d <= de_max whose threshold is non-zero at some sweep.
// Schedule values: temperatures > 0 (Metropolis) or flip probabilities in [0, 1] (paper rule).
int check_schedule_values(const gdi_schedule *s)
{
    if (s->acceptance > GDI_ACCEPT_PAPER) return fail(GDI_EINVAL, "unknown acceptance rule");
    for (uint32_t t = 0; t < s->n_sweeps; ++t) {
        const double v = s->temps[t];
        if (s->acceptance == GDI_ACCEPT_PAPER ? !(v >= 0.0 && v <= 1.0) : !(v > 0.0))
            return fail(GDI_EINVAL, s->acceptance == GDI_ACCEPT_PAPER ? "flip probabilities must lie in [0, 1]"
                                                                     : "temperatures must be > 0");
    }
    return GDI_OK;
}

// Paper rule: one entry per sweep, min(2^32 - 1, floor(2^32 P_f)) (exact: P_f in [0, 1]
// scaled by a power of two, then truncated).
uint32_t flip_threshold_of(double pf)
{
    const double v = std::floor(std::ldexp(pf, 32));
    return v >= 4294967295.0 ? 0xFFFFFFFFu : (uint32_t)v;
}

int build_table(const double *temps, uint32_t S, int64_t de_max, int32_t *K_out, std::vector<uint32_t> &tab,
                uint32_t rule)
{
    if (rule == GDI_ACCEPT_PAPER) {
        tab.assign(S, 0u);
        for (uint32_t t = 0; t < S; ++t) tab[t] = flip_threshold_of(temps[t]);
        *K_out = 0;
        return GDI_OK;
    }
    int64_t K = 0;
    for (uint32_t t = 0; t < S; ++t) {
        const double T = temps[t];
        // thr(d) >= 1 iff 2^32 exp(-d/T) >= 1, i.e. d <= 32 ln2 T; probe around that bound exactly
        int64_t d = (int64_t)std::min<double>((double)de_max, std::floor(32.0 * 0.6931471805599453 * T) + 2.0);
        if (threshold_of(d, T) != 0) {
            while (d < de_max && threshold_of(d + 1, T) != 0) ++d;
        } else {
            while (d > K && threshold_of(d, T) == 0) --d;
        }
        K = std::max(K, d);
    }
    if (K > (int64_t)64 * 1024 * 1024 / std::max<uint32_t>(S, 1))
        return fail(GDI_ERANGE, "threshold table too large (temperatures too high for the graph size)");
    tab.assign((size_t)S * (size_t)(K + 1), 0u);
    for (uint32_t t = 0; t < S; ++t) {
        uint32_t *row = tab.data() + (size_t)t * (size_t)(K + 1);
        row[0] = 0xFFFFFFFFu;
        for (int64_t d = 1; d <= K; ++d) row[d] = threshold_of(d, temps[t]);
    }
    *K_out = (int32_t)K;
    return GDI_OK;
}

// Threshold table for the schedule, cached on the handle by temperature content.
int ensure_table(gdi_graph *g, const gdi_schedule *s, int64_t de_max)
{
    const uint32_t S = s->n_sweeps;
    if (g->thr_K >= 0 && g->thr_demax == de_max && g->thr_rule == s->acceptance && g->thr_key.size() == S &&
        std::memcmp(g->thr_key.data(), s->temps, S * sizeof(double)) == 0)
        return GDI_OK;
    std::vector<uint32_t> tab;
    int32_t K = 0;
    int rc = build_table(s->temps, S, de_max, &K, tab, s->acceptance);
    if (rc) return rc;
    // the cached table is gone once its buffer is reallocated: forget it first, so that a
    // failed allocation or upload never leaves a key that names a released buffer
    g->thr_K = -1;
    g->thr_key.clear();
    HIP_TRY(g->d_thr.reserve(tab.size()), "hipMalloc thresholds");
    HIP_TRY(hipMemcpyAsync(g->d_thr.p, tab.data(), tab.size() * 4, hipMemcpyHostToDevice, g->stream),
            "upload thresholds");
    HIP_TRY(hipStreamSynchronize(g->stream), "upload thresholds");
    g->thr_key.assign(s->temps, s->temps + S);
    g->thr_K = K;
    g->thr_demax = de_max;
    g->thr_rule = s->acceptance;
    return GDI_OK;
}

int finish_pending(gdi_graph *g)
{
    if (!g->pending) return GDI_OK;
    g->pending = false;
    HIP_TRY(hipStreamSynchronize(g->stream), "anneal");
    int64_t st[8], red[4];
    HIP_TRY(hipMemcpy(st, g->d_state.p, sizeof(st), hipMemcpyDeviceToHost), "read state");
    HIP_TRY(hipMemcpy(red, g->d_red.p, sizeof(red), hipMemcpyDeviceToHost), "read state");
    if (st[3] != 0) {
        g->last_valid = false;
        return fail(GDI_ETIMEOUT, "a device-side barrier wait expired; results are invalid");
    }
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, g->ev0, g->ev1), "hipEventElapsedTime");
    g->last.magnetization = st[0];
    g->last.cut_weighted = red[1] / 2 + st[1];
    g->last.sweep_ms = ms;
    g->last_cut0 = red[1] / 2;
    g->last_valid = true;
    return GDI_OK;
}

// One anneal in progress: the launch choice and the argument block shared by all
// of its sweep launches (a learned anneal launches sweep ranges repeatedly).
struct RunCtx {
    Choice ch;
    GdiSweepArgs a;
    int thr_in_lds;
    uint64_t bar_words;
    bool dense;        // the standard solver (GDI_FLAG_DENSE_BALANCE)
    bool racy;         // the asynchronous sweep (GDI_FLAG_RACY)
};

// Validates the schedule, builds the threshold table, writes the initial state
// (spins, M, per-class counts, cut) and fills the launch arguments.
int prepare_run(gdi_graph *g, const gdi_schedule *s, uint64_t seed, bool dev_out, RunCtx &r)
{
    if (!g) return fail(GDI_ESTATE, "NULL handle");
    if (!s) return fail(GDI_EINVAL, "NULL schedule");
    int rc = finish_pending(g);
    if (rc) return rc;
    const uint32_t S = s->n_sweeps;
    if (S < 1) return fail(GDI_EINVAL, "n_sweeps must be >= 1");
    if (!s->temps) return fail(GDI_EINVAL, "NULL temps");
    if (s->start_sweep > S) return fail(GDI_EINVAL, "start_sweep > n_sweeps");
    if (int rc0 = check_schedule_values(s)) return rc0;
    if (s->balance_mode > GDI_BAL_SNAPSHOT) return fail(GDI_EINVAL, "unknown balance_mode");
    if (s->flags & ~(GDI_FLAG_DENSE_BALANCE | GDI_FLAG_RACY)) return fail(GDI_EINVAL, "unknown schedule flags");
    if ((s->flags & GDI_FLAG_DENSE_BALANCE) && (s->flags & GDI_FLAG_RACY))
        return fail(GDI_EINVAL, "the dense-balance and asynchronous flags exclude each other");
    if ((s->flags & GDI_FLAG_RACY) && (s->trace_m || s->trace_cut))
        return fail(GDI_EINVAL, "the asynchronous sweep takes no traces");
    if (dev_out && (s->trace_m || s->trace_cut)) return fail(GDI_EINVAL, "traces need the host variant");
    const int64_t de_max = std::llabs((long long)s->B) * g->max_abs_wdeg + 4 * std::llabs((long long)s->A) * ((int64_t)g->n + 1);
    if (de_max >= (int64_t(1) << 31))
        return fail(GDI_ERANGE, "|B|*max_wdeg + 4|A|(n+1) must be < 2^31");
    const bool trace = s->trace_m || s->trace_cut;

    if ((rc = pick_launch(g, &r.ch, (s->flags & GDI_FLAG_DENSE_BALANCE) != 0))) return rc;
    r.dense = (s->flags & GDI_FLAG_DENSE_BALANCE) != 0;
    r.racy = (s->flags & GDI_FLAG_RACY) != 0;
    if (r.dense) {
        int dev = 0, lds_max = 0;
        HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
        HIP_TRY(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev), "hipDeviceGetAttribute");
        if (r.ch.scope != GDI_SCOPE_WORKGROUP || gdi_dense_lds_bytes(g->n_pad, g->C) + 64 > lds_max)
            return fail(GDI_ERANGE, "the standard solver runs graphs that fit one workgroup (workgroup scope, "
                                    "two spin copies in LDS)");
    }
    if ((rc = ensure_table(g, s, de_max))) return rc;
    const uint64_t phases = (uint64_t)(S - s->start_sweep) * (uint64_t)g->C;
    r.bar_words = 0;
    if (phases > (uint64_t(1) << 30)) return fail(GDI_ERANGE, "too many phases for one launch");
    if (r.ch.scope == GDI_SCOPE_GRID_FENCED && !r.racy) {
        if (phases > (uint64_t(1) << 22)) return fail(GDI_ERANGE, "too many phases for one launch");
        r.bar_words = phases * (GDI_BAR_GROUPS + 1) * GDI_BAR_PAD;
        HIP_TRY(g->d_bar.reserve(r.bar_words), "hipMalloc barrier");
    }
    if (r.racy) {
        // one device-wide barrier per sweep
        r.bar_words = (uint64_t)(S - s->start_sweep) * (GDI_BAR_GROUPS + 1) * GDI_BAR_PAD;
        HIP_TRY(g->d_bar.reserve(std::max<uint64_t>(r.bar_words, 1)), "hipMalloc barrier");
    }
    if (trace) HIP_TRY(g->d_trace.reserve(2 * (size_t)S), "hipMalloc trace");

    hipStream_t st = g->stream;
    if (s->init_spins) {
        HIP_TRY(hipMemcpyAsync(g->d_io.p, s->init_spins, (size_t)g->n, hipMemcpyHostToDevice, st), "upload spins");
        if ((rc = gdi_launch_gather_in(g->d_orig.p, g->d_io.p, g->n_pad, g->d_spin.p, st)))
            return fail(GDI_EDEVICE, gdi_hip_error_string(rc));
    } else {
        if ((rc = gdi_launch_init_spins(g->d_orig.p, nullptr, g->d_spin.p, g->n_pad, (uint32_t)seed,
                                        (uint32_t)(seed >> 32), s->replica, st)))
            return fail(GDI_EDEVICE, gdi_hip_error_string(rc));
    }
    rc = gdi_launch_fill_u64(reinterpret_cast<uint64_t *>(g->d_state.p), 8, st);
    if (!rc && trace) rc = gdi_launch_fill_u64(reinterpret_cast<uint64_t *>(g->d_trace.p), 2 * (int64_t)S, st);
    if (!rc) rc = gdi_launch_reduce(g->d_rp.p, g->d_adj.p, g->d_spin.p, g->n_pad, g->nnz, g->d_cbeg.p, g->d_csz.p,
                                    g->C, g->d_red.p, g->d_P.p, g->d_bits.p, st);
    // the sweep kernels read the initial M from state[0]
    if (!rc) {
        hipError_t e = hipMemcpyAsync(g->d_state.p, g->d_red.p, 8, hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return hip_fail(e, "state copy");
    }
    if (rc) return fail(GDI_EDEVICE, gdi_hip_error_string(rc));

    GdiSweepArgs &a = r.a;
    a = GdiSweepArgs{};
    a.rp = g->d_rp.p;
    a.adj = g->d_adj.p;
    a.orig = g->d_orig.p;
    a.spin = g->d_spin.p;
    a.cbeg = g->d_cbeg.p;
    a.csz = g->d_csz.p;
    a.thr = g->d_thr.p;
    a.state = g->d_state.p;
    a.P = g->d_P.p;
    a.trace_m = trace ? g->d_trace.p : nullptr;
    a.trace_dcut = trace ? g->d_trace.p + S : nullptr;
    a.n = g->n;
    a.n_pad = g->n_pad;
    a.C = g->C;
    a.K = g->thr_K;
    a.t0 = s->start_sweep;
    a.S = S;
    a.A4 = 4 * s->A;
    a.B = s->B;
    a.key0 = (uint32_t)seed;
    a.key1 = (uint32_t)(seed >> 32);
    a.replica = s->replica;
    a.snapshot = s->balance_mode == GDI_BAL_SNAPSHOT ? 1u : 0u;
    a.rule = s->acceptance;
    a.spin_limit = (g->have_tune && g->tune.spin_limit) ? (int64_t)g->tune.spin_limit : kSpinLimit;
    r.thr_in_lds = 0;
    if (r.ch.scope == GDI_SCOPE_GRID) {
        int lds_max = 0, dev = 0;
        HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
        HIP_TRY(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev), "hipDeviceGetAttribute");
        r.thr_in_lds = (g->thr_K <= GDI_HALO_THR_MAX &&
                        gdi_halo_lds_bytes(g->halo_lds_words, g->C, 2 * (g->thr_K + 1)) <= lds_max) ? 1 : 0;
    }
    g->last = gdi_result{};
    g->last.n_colours = (uint32_t)g->C;
    g->last.scope = r.ch.scope;
    g->last.grid = r.ch.grid;
    g->last.block = r.ch.block;
    g->last.lanes_per_node = r.ch.lanes;
    g->last.table_width = (uint32_t)g->thr_K;
    g->last_valid = false;
    return GDI_OK;
}

// Launches sweeps [t_from, t_to) continuing from the device state; mask (bit set =
// skip) and last_flip are optional.
// With gate set, the launch runs only if more than active_max nodes are active (the
// active-set kernel takes the other case).
// Sweeps t_from..t_to-1; the mask (if any) applies to sweeps before mask_end (0: all);
// a closed gate skips the launch, or with gate_t0 > 0 (grid scope only) starts it at
// sweep gate_t0.
int launch_range(gdi_graph *g, RunCtx &r, uint32_t t_from, uint32_t t_to, const uint32_t *mask, int32_t *last_flip,
                 const uint64_t *gate = nullptr, int32_t active_max = 0, uint32_t mask_end = 0, uint32_t gate_t0 = 0)
{
    hipStream_t st = g->stream;
    GdiSweepArgs a = r.a;
    a.t0 = t_from;
    a.S = t_to;
    a.mask = mask;
    a.last_flip = last_flip;
    a.skip_count = reinterpret_cast<const unsigned long long *>(gate);
    a.active_max = active_max;
    a.gate_small = 0;
    a.mask_end = mask_end ? mask_end : t_to;
    a.gate_t0 = gate_t0 ? gate_t0 : t_to;
    if ((mask_end && mask_end != t_to) || gate_t0) {
        if (r.ch.scope != GDI_SCOPE_GRID || r.racy || r.dense)
            return fail(GDI_EDEVICE, "internal: a partial mask or a late start needs the grid sweep");
    }
    int rc = 0;
    if (r.racy) {
        // Alg. 3 in one persistent launch; the magnetisation stays the one its atomic
        // adds tracked, the cut and the class counts are recounted from the spins
        int grid = 0;
        rc = gdi_async_capacity(1024, &grid);
        if (!rc && g->have_tune && g->tune.grid) {
            if ((int)g->tune.grid > grid) return fail(GDI_EDEVICE, "grid exceeds the co-resident capacity");
            grid = (int)g->tune.grid;
        }
        const uint64_t sweeps = t_to - t_from;
        a.bar_grp = g->d_bar.p;
        a.bar_glob = g->d_bar.p + sweeps * GDI_BAR_GROUPS * GDI_BAR_PAD;
        if (!rc) rc = gdi_launch_fill_u64(g->d_bar.p, (int64_t)(sweeps * (GDI_BAR_GROUPS + 1) * GDI_BAR_PAD), st);
        if (!rc && sweeps > 0) rc = gdi_launch_sweep_async(a, grid, 1024, st);
        if (!rc) rc = gdi_launch_reduce(g->d_rp.p, g->d_adj.p, g->d_spin.p, g->n_pad, g->nnz, g->d_cbeg.p, g->d_csz.p, g->C,
                                        g->d_red.p, g->d_P.p, g->d_bits.p, st);
        if (!rc) g->last.grid = (uint32_t)grid;
        if (!rc) g->last.block = 1024;
    } else if (r.dense) {
        rc = gdi_launch_sweep_dense(a, (int)r.ch.block, (int)r.ch.lanes, st);
    } else if (r.ch.scope == GDI_SCOPE_WORKGROUP) {
        rc = r.ch.csr_lds ? gdi_launch_sweep_wgl(a, g->d_rp16.p, g->d_ent16.p, (int32_t)g->nnz, (int)r.ch.block,
                                                 (int)r.ch.lanes, st)
                          : gdi_launch_sweep_wg(a, (int)r.ch.block, (int)r.ch.lanes, r.ch.spins_lds ? 1 : 0, st);
    } else if (r.ch.scope == GDI_SCOPE_GRID) {
        GdiHaloArgs ha{};
        ha.base = a;
        ha.adjL = g->d_adjL.p;
        ha.unit_w = (g->have_tune && g->tune.general_weights > 0) ? 0 : g->halo_unit_w;
        ha.tab = g->d_tab.p;
        ha.words = g->d_words.p;
        ha.member = g->d_member.p;
        ha.group = g->d_group.p;
        ha.lds_words = g->halo_lds_words;
        ha.T0 = g->halo_T0;
        ha.tail_n = g->halo_tail_n;
        ha.gather_off = g->halo_gather_off;
        ha.tail_off = g->halo_tail_off;
        ha.tail_v = g->d_tail_v.p;
        ha.tail_beg = g->d_tail_beg.p;
        ha.gat_words = g->d_gat_words.p;
        ha.gat_beg = g->d_gat_beg.p;
        ha.tail_nnz = g->halo_tail_nnz;
        ha.trp_off = g->halo_trp_off;
        ha.tent_off = g->halo_tent_off;
        ha.tail_rp = g->d_tail_rp.p;
        ha.tail_ent = g->d_tail_ent.p;
        ha.ovf_off = g->halo_ovf_off;
        ha.ovf_len = g->halo_ovf_len;
        ha.ovf = g->d_ovf.p;
        ha.list_off = g->halo_list_off;
        ha.flist_len = g->halo_flist_len;
        ha.flist = g->d_flist.p;
        ha.thr_in_lds = r.thr_in_lds;
        // epochs continue from launch to launch; the words are cleared only when they may
        // hold larger ones (new buffers) or the epochs would wrap
        const uint64_t span = (uint64_t)(t_to - t_from) * (uint64_t)std::max(g->halo_T0, 1) + 4;
        if (!g->halo_words_clean || (uint64_t)g->halo_epoch + span > 0x7FFFFFFFull) {
            rc = gdi_launch_fill_u64(g->d_words.p, (int64_t)g->n_pad / 32 + 1, st);
            if (!rc) rc = gdi_launch_fill_u64(g->d_member.p, 8 * 64, st);
            if (!rc) rc = gdi_launch_fill_u64(g->d_group.p, 2 * 8 * GDI_HALO_GROUP_PAD, st);
            g->halo_epoch = 0;
            g->halo_words_clean = rc == 0;
        }
        ha.epoch0 = g->halo_epoch;
        if (!rc) rc = gdi_launch_sweep_halo(ha, (int)r.ch.grid, (int)r.ch.block, st);
        g->halo_epoch += (uint32_t)span;  // also after a failed launch: its words stay below
    } else {
        const uint64_t phases = (uint64_t)(t_to - t_from) * (uint64_t)g->C;
        const uint64_t words = phases * (GDI_BAR_GROUPS + 1) * GDI_BAR_PAD;
        a.bar_grp = g->d_bar.p;
        a.bar_glob = g->d_bar.p + phases * GDI_BAR_GROUPS * GDI_BAR_PAD;
        rc = gdi_launch_fill_u64(g->d_bar.p, (int64_t)words, st);
        if (!rc) rc = gdi_launch_sweep_grid(a, (int)r.ch.grid, (int)r.ch.block, (int)r.ch.lanes, st);
    }
    if (rc) return fail(GDI_EDEVICE, std::string("sweep launch: ") + gdi_hip_error_string(rc));
    return GDI_OK;
}

int anneal_impl(gdi_graph *g, const gdi_schedule *s, uint64_t seed, int8_t *host_out, int8_t *dev_out)
{
    RunCtx r;
    int rc = prepare_run(g, s, seed, dev_out != nullptr, r);
    if (rc) return rc;
    hipStream_t st = g->stream;
    const uint32_t S = s->n_sweeps;
    HIP_TRY(hipEventRecord(g->ev0, st), "hipEventRecord");
    if ((rc = launch_range(g, r, s->start_sweep, S, nullptr, nullptr))) return rc;
    HIP_TRY(hipEventRecord(g->ev1, st), "hipEventRecord");

    int8_t *out_dev = dev_out ? dev_out : g->d_io.p;
    if ((rc = gdi_launch_scatter_out(g->d_orig.p, g->d_spin.p, g->n_pad, out_dev, st)))
        return fail(GDI_EDEVICE, gdi_hip_error_string(rc));
    g->pending = true;
    if (dev_out) return GDI_OK;

    if ((rc = finish_pending(g))) return rc;
    HIP_TRY(hipMemcpy(host_out, g->d_io.p, (size_t)g->n, hipMemcpyDeviceToHost), "download spins");
    if (s->trace_m || s->trace_cut) {
        std::vector<int64_t> tr(2 * (size_t)S);
        HIP_TRY(hipMemcpy(tr.data(), g->d_trace.p, tr.size() * 8, hipMemcpyDeviceToHost), "download trace");
        int64_t cut = g->last_cut0;
        for (uint32_t t = s->start_sweep; t < S; ++t) {
            cut += tr[S + t];
            if (s->trace_m) s->trace_m[t] = tr[t];
            if (s->trace_cut) s->trace_cut[t] = cut;
        }
    }
    return GDI_OK;
}

int cut_impl(gdi_graph *g, const int8_t *spins, bool dev, int64_t *cw, int64_t *ce, int64_t *m)
{
    if (!g) return fail(GDI_ESTATE, "NULL handle");
    if (!spins) return fail(GDI_EINVAL, "NULL spins");
    int rc = finish_pending(g);
    if (rc) return rc;
    hipStream_t st = g->stream;
    const int8_t *src = spins;
    if (!dev) {
        HIP_TRY(hipMemcpyAsync(g->d_io.p, spins, (size_t)g->n, hipMemcpyHostToDevice, st), "upload spins");
        src = g->d_io.p;
    }
    // a scratch copy so a pending anneal state is not disturbed
    DevBuf<int8_t> tmp;
    HIP_TRY(tmp.reserve((size_t)g->n_pad), "hipMalloc");
    DevBuf<int32_t> P;
    HIP_TRY(P.reserve((size_t)g->C + 2), "hipMalloc");
    DevBuf<int64_t> red;
    HIP_TRY(red.reserve(4), "hipMalloc");
    // the spins gathered into the annealer's order (one thread per id: a gather per
    // thread keeps the most loads in flight), then reduced
    rc = gdi_launch_gather_in(g->d_orig.p, src, g->n_pad, tmp.p, st);
    if (!rc)
        rc = gdi_launch_reduce(g->d_rp.p, g->d_adj.p, tmp.p, g->n_pad, g->nnz, g->d_cbeg.p, g->d_csz.p, g->C, red.p,
                               P.p, g->d_bits.p, st);
    if (rc) {
        tmp.release(); P.release(); red.release();
        return fail(GDI_EDEVICE, gdi_hip_error_string(rc));
    }
    int64_t h[4];
    hipError_t e = hipMemcpyAsync(h, red.p, sizeof(h), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    tmp.release(); P.release(); red.release();
    if (e != hipSuccess) return hip_fail(e, "gdi_cut");
    if (m) *m = h[0];
    if (cw) *cw = h[1] / 2;
    if (ce) *ce = h[2] / 2;
    return GDI_OK;
}

// ------------------------------------------------------------------ autotuner cache
// Launch choices the autotuners found, keyed by "<arch>/<CUs>cu|batch|..." or
// "<arch>/<CUs>cu|graph|..." (device, then problem shape). Held in memory and, when
// the environment variable GDI_TUNE_CACHE names a file, in that JSON file: read at the
// first lookup of the process, rewritten after every tuning run. The file is a hint:
// a missing, unreadable or malformed one leaves the in-memory cache as it is.
std::mutex g_tune_mu;
gdi_tunecache::Table g_tune_table;
bool g_tune_env_read = false;

const char *tune_env_path()
{
    const char *p = std::getenv("GDI_TUNE_CACHE");
    return (p && *p) ? p : nullptr;
}

void tune_env_read_locked()
{
    if (g_tune_env_read) return;
    g_tune_env_read = true;
    const char *p = tune_env_path();
    std::string text, err;
    if (p && gdi_tunecache::read_file(p, &text)) (void)gdi_tunecache::parse(text, &g_tune_table, &err);
}

gdi_tunecache::Fields tuning_fields(const gdi_tuning &t, double ms)
{
    gdi_tunecache::Fields f;
    f["scope"] = t.scope;
    f["block"] = t.block;
    f["grid"] = t.grid;
    f["lanes_per_node"] = t.lanes_per_node;
    f["tail_max"] = t.tail_max;
    f["leaders"] = t.leaders;
    f["general_weights"] = t.general_weights;
    f["csr_lds"] = t.csr_lds;
    f["batch_members"] = t.batch_members;
    f["ms"] = ms;
    return f;
}

// false when a field is missing, not an integer or out of its range
bool fields_tuning(const gdi_tunecache::Fields &f, gdi_tuning *t, double *ms)
{
    auto get = [&](const char *k, double lo, double hi, double *v) {
        auto it = f.find(k);
        if (it == f.end() || !(it->second >= lo && it->second <= hi) || it->second != std::floor(it->second))
            return false;
        *v = it->second;
        return true;
    };
    double v[9];
    if (!get("scope", 0, GDI_SCOPE_GRID_FENCED, &v[0]) || !get("block", 0, GDI_MAX_BLOCK, &v[1]) ||
        !get("grid", 0, 1 << 20, &v[2]) || !get("lanes_per_node", 0, 64, &v[3]) ||
        !get("tail_max", -1, 1 << 20, &v[4]) || !get("leaders", -1, 1, &v[5]) ||
        !get("general_weights", -1, 1, &v[6]) || !get("csr_lds", -1, 1, &v[7]) ||
        !get("batch_members", -1, GDI_BATCH_MAX_MEMBERS, &v[8]))
        return false;
    gdi_tuning r{};
    r.scope = (uint32_t)v[0];
    r.block = (uint32_t)v[1];
    r.grid = (uint32_t)v[2];
    r.lanes_per_node = (uint32_t)v[3];
    r.tail_max = (int32_t)v[4];
    r.leaders = (int32_t)v[5];
    r.general_weights = (int32_t)v[6];
    r.csr_lds = (int32_t)v[7];
    r.batch_members = (int32_t)v[8];
    *t = r;
    auto it = f.find("ms");
    *ms = it != f.end() ? it->second : 0.0;
    return true;
}

bool tune_lookup(const std::string &key, gdi_tuning *t, double *ms)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_env_read_locked();
    auto it = g_tune_table.find(key);
    return it != g_tune_table.end() && fields_tuning(it->second, t, ms);
}

void tune_store(const std::string &key, const gdi_tuning &t, double ms)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_env_read_locked();
    g_tune_table[key] = tuning_fields(t, ms);
    if (const char *p = tune_env_path()) (void)gdi_tunecache::write_file(p, gdi_tunecache::dump(g_tune_table));
}

// "<arch>/<CUs>cu" of the current device ("" if it cannot be queried)
std::string device_tag()
{
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "";
    std::string arch = prop.gcnArchName;
    const size_t colon = arch.find(':');
    if (colon != std::string::npos) arch.resize(colon);
    return arch + "/" + std::to_string(prop.multiProcessorCount) + "cu";
}

std::string graph_key(const gdi_graph *g)
{
    return device_tag() + "|graph|n=" + std::to_string(g->n) + "|nnz=" + std::to_string(g->nnz) +
           "|C=" + std::to_string(g->C) + "|maxdeg=" + std::to_string(g->max_degree) +
           "|w=" + (g->wkind == 2 ? "unit" : g->wkind == 1 ? "pm1" : "general");
}

// ------------------------------------------------------------------ batched form
std::string batch_key(const gdi_instance *inst, uint32_t n_inst)
{
    int64_t sn = 0, snnz = 0;
    int32_t mx = 0, mc = 0;
    for (uint32_t i = 0; i < n_inst; ++i) {
        sn += inst[i].graph->n;
        snnz += inst[i].graph->nnz;
        mx = std::max(mx, inst[i].graph->n_pad);
        mc = std::max(mc, inst[i].graph->C);
    }
    return device_tag() + "|batch|inst=" + std::to_string(n_inst) + "|n=" + std::to_string(sn) +
           "|nnz=" + std::to_string(snnz) + "|maxnpad=" + std::to_string(mx) + "|maxC=" + std::to_string(mc);
}

// Single-graph autotuner: coordinate descent over the launch choices that apply to the
// graph -- the workgroup sweep (graphs of at most 65536 padded nodes) with the CSR in
// LDS or global memory, the halo grid sweep on 8 .. 256 workgroups -- then lanes per
// node and block size (workgroup sweep) or the redundant tail and dedicated leaders
// (grid sweep). Each candidate is timed as the best device time of two runs over the
// first probe sweeps of the schedule; a candidate that does not fit is skipped.
int autotune_graph(gdi_graph *g, const gdi_schedule *s, uint64_t seed, uint32_t probe, gdi_tuning *best,
                   double *best_ms)
{
    if (!g) return fail(GDI_ESTATE, "NULL handle");
    if (!s || !s->temps || s->n_sweeps < 1) return fail(GDI_EINVAL, "bad schedule");
    if (s->flags) return fail(GDI_EINVAL, "the autotuner times the deterministic sweep (schedule flags 0)");
    gdi_schedule ps = *s;
    ps.n_sweeps = std::max<uint32_t>(1, std::min(probe ? probe : std::max<uint32_t>(1, s->n_sweeps / 50), s->n_sweeps));
    ps.start_sweep = 0;
    ps.init_spins = nullptr;
    ps.trace_m = nullptr;
    ps.trace_cut = nullptr;
    std::vector<int8_t> out((size_t)g->n);
    const gdi_tuning saved = g->tune;
    const bool saved_have = g->have_tune;
    int last_err = GDI_OK;
    auto timed = [&](const gdi_tuning &t, double *ms) -> int {
        g->tune = t;
        g->have_tune = true;
        double a = 1e300;
        for (int k = 0; k < 2; ++k) {
            const int r = anneal_impl(g, &ps, seed, out.data(), nullptr);
            if (r) return r;
            a = std::min(a, g->last.sweep_ms);
        }
        *ms = a;
        return GDI_OK;
    };
    gdi_tuning cur{};
    double cur_ms = 1e300;
    bool any = false;
    // a candidate that does not fit (range, launch shape) is skipped; anything else stops
    auto consider = [&](const gdi_tuning &t) -> int {
        double ms = 0;
        const int r = timed(t, &ms);
        if (r == GDI_ERANGE || r == GDI_EDEVICE || r == GDI_EINVAL) {
            last_err = r;
            return GDI_OK;
        }
        if (r) return r;
        if (!any || ms < cur_ms) {
            cur_ms = ms;
            cur = t;
            any = true;
        }
        return GDI_OK;
    };
    int rc = GDI_OK;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        rc = fail(GDI_EDEVICE, "device query");
    if (!rc && g->n_pad <= kWgMaxNodes) {
        gdi_tuning t{};
        t.scope = GDI_SCOPE_WORKGROUP;
        if (!rc) rc = consider(t);
        if (!rc && g->wgl_ok) {
            t.csr_lds = -1;
            rc = consider(t);
        }
    }
    const int32_t g_cap = std::min(cus, GDI_HALO_MAX_GRID) / 8 * 8;
    for (int32_t G = 8; !rc && G <= g_cap; G *= 2) {
        if (G > 8 && (int64_t)G * 256 > g->n) break;  // fewer than 256 nodes per workgroup
        gdi_tuning t{};
        t.scope = GDI_SCOPE_GRID;
        t.grid = (uint32_t)G;
        rc = consider(t);
    }
    if (!rc && any && cur.scope == GDI_SCOPE_WORKGROUP) {
        const gdi_tuning base = cur;
        for (uint32_t l : {1u, 2u, 4u, 8u, 16u, 32u}) {
            gdi_tuning t = base;
            t.lanes_per_node = l;
            if ((rc = consider(t))) break;
        }
        const gdi_tuning base2 = cur;
        for (uint32_t b : {256u, 512u}) {
            if (rc) break;
            gdi_tuning t = base2;
            t.block = b;
            if (t.lanes_per_node > b) continue;
            rc = consider(t);
        }
    } else if (!rc && any && cur.scope == GDI_SCOPE_GRID) {
        gdi_tuning t = cur;
        t.tail_max = -1;
        rc = consider(t);
        if (!rc && cur.grid >= 16) {
            // the other leader arrangement than the automatic one for this grid
            t = cur;
            t.leaders = cur.grid >= 64 ? -1 : 1;
            rc = consider(t);
        }
    }
    if (!rc && !any) rc = last_err ? last_err : fail(GDI_EDEVICE, "no launch candidate ran");
    if (rc) {
        g->tune = saved;
        g->have_tune = saved_have;
        return rc;
    }
    g->tune = cur;
    g->have_tune = true;
    *best = cur;
    if (best_ms) *best_ms = cur_ms;
    tune_store(graph_key(g), cur, cur_ms);
    return GDI_OK;
}

int check_batch(const gdi_instance *inst, uint32_t n_inst, const gdi_schedule *s)
{
    if (!inst || n_inst == 0) return fail(GDI_EINVAL, "empty batch");
    if (!s || !s->temps || s->n_sweeps < 1) return fail(GDI_EINVAL, "bad schedule");
    if (s->start_sweep != 0 || s->init_spins || s->trace_m || s->trace_cut)
        return fail(GDI_EINVAL, "batched anneals start fresh and take no traces");
    if (s->balance_mode > GDI_BAL_SNAPSHOT) return fail(GDI_EINVAL, "unknown balance_mode");
    if (int rc0 = check_schedule_values(s)) return rc0;
    if (s->flags) return fail(GDI_EINVAL, "the batched form takes no schedule flags");
    for (uint32_t i = 0; i < n_inst; ++i)
        if (!inst[i].graph) return fail(GDI_EINVAL, "NULL graph in batch");
    return GDI_OK;
}

// One batched launch. probe_S > 0 runs only the first probe_S sweeps and writes no
// outputs (autotuning); otherwise results go to inst[].
int run_batch(gdi_instance *inst, uint32_t n_inst, const gdi_schedule *s, uint64_t seed, const gdi_tuning &tn,
              bool dev_out, uint32_t probe_S, double *kernel_ms)
{
    int rc = check_batch(inst, n_inst, s);
    if (rc) return rc;
    for (uint32_t i = 0; i < n_inst; ++i)
        if ((rc = finish_pending(inst[i].graph))) return rc;
    const uint32_t S = probe_S ? std::min(probe_S, s->n_sweeps) : s->n_sweeps;
    int64_t de_max = 0;
    int32_t lds = 0;
    for (uint32_t i = 0; i < n_inst; ++i) {
        const gdi_graph *g = inst[i].graph;
        de_max = std::max<int64_t>(de_max, std::llabs((long long)s->B) * g->max_abs_wdeg +
                                               4 * std::llabs((long long)s->A) * ((int64_t)g->n + 1));
        lds = std::max(lds, gdi_batch_lds_bytes(g->n_pad, g->C));
    }
    if (de_max >= (int64_t(1) << 31)) return fail(GDI_ERANGE, "|B|*max_wdeg + 4|A|(n+1) must be < 2^31");
    int dev = 0, lds_max = 0, cus = 0;
    HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
    HIP_TRY(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev), "hipDeviceGetAttribute");
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev), "hipDeviceGetAttribute");
    if (lds + 64 + 2 * GDI_WG_THR_MAX * 4 > lds_max) return fail(GDI_ERANGE, "an instance does not fit one workgroup's LDS");
    const uint32_t block = tn.block ? tn.block : 512u;
    if (block < 64 || block > GDI_MAX_BLOCK || block % 64) return fail(GDI_EINVAL, "block must be a multiple of 64 in [64, 1024]");
    if (tn.lanes_per_node && (tn.lanes_per_node > 64 || (tn.lanes_per_node & (tn.lanes_per_node - 1))))
        return fail(GDI_EINVAL, "lanes_per_node must be a power of two in [1, 64]");
    int per_cu = 0;
    int e = gdi_batch_occupancy((int)block, lds, &per_cu);
    if (e || per_cu < 1) return fail(GDI_EDEVICE, "batched sweep cannot be launched with this block size");
    // workgroups of the launch (clamped to the number of tickets below)
    uint32_t grid = std::max<uint32_t>(1, tn.grid ? tn.grid : (uint32_t)(cus * per_cu));

    std::vector<uint32_t> tab;
    int32_t K = 0;
    if ((rc = build_table(s->temps, S, de_max, &K, tab, s->acceptance))) return rc;

    // Clusters: an instance whose work (n + nnz) exceeds twice the per-workgroup share of
    // the batch runs on k workgroups (k about its work over the share, at most
    // GDI_BATCH_MAX_MEMBERS or tuning.batch_members; graphs with at least two colour
    // classes). All cluster members are dealt first, so that the launch's first pops
    // start every member of every cluster at once (the launch is then cooperative).
    std::vector<int32_t> mem(n_inst, 1);
    {
        // Clusters need a co-resident launch: at most 16 waves per CU (the shape every
        // cooperative launch of this library runs with; a larger occupancy figure was
        // refused by the cooperative launch or not co-resident), and the grid within it.
        const uint32_t coop_cap = (uint32_t)cus * (uint32_t)std::max(1, std::min(per_cu, (int)(GDI_MAX_BLOCK / block)));
        const bool coresident = grid <= coop_cap || !tn.grid;
        const uint32_t cgrid = std::min(grid, coop_cap);  // the grid if clusters form
        const int32_t cap = !coresident ? 1
                            : tn.batch_members > 0 ? std::min<int32_t>(tn.batch_members, GDI_BATCH_MAX_MEMBERS)
                                                   : (tn.batch_members < 0 ? 1 : GDI_BATCH_MAX_MEMBERS);
        double total = 0;
        for (uint32_t i = 0; i < n_inst; ++i) total += (double)(inst[i].graph->nnz + inst[i].graph->n);
        const double share = total / cgrid;
        int64_t sum = 0;
        for (uint32_t i = 0; i < n_inst; ++i) {
            const gdi_graph *g = inst[i].graph;
            const double w = (double)(g->nnz + g->n);
            if (cap > 1 && g->C >= 2 && w > 2.0 * share)
                mem[i] = (int32_t)std::min<double>(cap, std::ceil(w / share));
            sum += mem[i] > 1 ? mem[i] : 0;
        }
        // all members must start together: shrink the largest clusters until they fit the grid
        while (sum > (int64_t)cgrid) {
            uint32_t big = 0;
            for (uint32_t i = 1; i < n_inst; ++i)
                if (mem[i] > mem[big]) big = i;
            if (mem[big] <= 1) break;
            --mem[big];
            sum -= mem[big] == 1 ? 2 : 1;
        }
        if (sum > 0) grid = cgrid;
    }
    // tickets: cluster members first (largest work per member first), then the other
    // instances longest first
    std::vector<uint32_t> order(n_inst);
    for (uint32_t i = 0; i < n_inst; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](uint32_t x, uint32_t y) {
        const bool cx = mem[x] > 1, cy = mem[y] > 1;
        if (cx != cy) return cx;
        const double wx = (double)(inst[x].graph->nnz + inst[x].graph->n) / mem[x];
        const double wy = (double)(inst[y].graph->nnz + inst[y].graph->n) / mem[y];
        return wx > wy;
    });
    size_t n_tickets = 0, sync_words = 0;
    std::vector<size_t> sync_off(n_inst, 0);
    for (uint32_t i = 0; i < n_inst; ++i) {
        n_tickets += (size_t)mem[i];
        if (mem[i] > 1) {
            sync_off[i] = sync_words;
            sync_words += (size_t)inst[i].graph->n_pad / 32 + 1 + 32;
        }
    }
    const bool clusters = sync_words > 0;
    grid = std::max<uint32_t>(1, std::min<uint32_t>(grid, (uint32_t)n_tickets));
    DevBuf<GdiBatchInstance> d_inst;
    DevBuf<uint64_t> d_queue;
    DevBuf<int64_t> d_res;
    DevBuf<int8_t> d_out;
    DevBuf<uint32_t> d_thr;
    DevBuf<uint64_t> d_sync;
    struct Release {
        DevBuf<GdiBatchInstance> &a; DevBuf<uint64_t> &b; DevBuf<int64_t> &c; DevBuf<int8_t> &d; DevBuf<uint32_t> &e;
        DevBuf<uint64_t> &f;
        ~Release() { a.release(); b.release(); c.release(); d.release(); e.release(); f.release(); }
    } rel{d_inst, d_queue, d_res, d_out, d_thr, d_sync};
    std::vector<size_t> out_off(n_inst, 0);
    size_t out_total = 0;
    if (!probe_S && !dev_out)
        for (uint32_t i = 0; i < n_inst; ++i) {
            out_off[i] = out_total;
            if (inst[i].spins_out) out_total += (size_t)inst[i].graph->n;
        }
    HIP_TRY(d_inst.reserve(n_tickets), "hipMalloc batch");
    HIP_TRY(d_queue.reserve(2), "hipMalloc batch");  // [0] queue, [1] error flag
    HIP_TRY(d_res.reserve(2 * (size_t)n_inst), "hipMalloc batch");
    HIP_TRY(d_thr.reserve(tab.size()), "hipMalloc batch thresholds");
    if (clusters) HIP_TRY(d_sync.reserve(sync_words), "hipMalloc batch clusters");
    if (out_total) HIP_TRY(d_out.reserve(out_total), "hipMalloc batch outputs");
    std::vector<GdiBatchInstance> h_inst(n_tickets);
    size_t q = 0;
    for (uint32_t oi = 0; oi < n_inst; ++oi) {
        const uint32_t i = order[oi];
        const gdi_graph *g = inst[i].graph;
        for (int32_t rnk = 0; rnk < mem[i]; ++rnk, ++q) {
            GdiBatchInstance &b = h_inst[q];
            b.rp = g->d_rp.p;
            b.adj = g->d_adj.p;
            b.orig = g->d_orig.p;
            b.cbeg = g->d_cbeg.p;
            b.csz = g->d_csz.p;
            b.out = nullptr;
            if (!probe_S && inst[i].spins_out) b.out = dev_out ? inst[i].spins_out : d_out.p + out_off[i];
            b.result = d_res.p + 2 * (size_t)i;
            b.n = g->n;
            b.n_pad = g->n_pad;
            b.C = g->C;
            b.lanes = tn.lanes_per_node ? (int32_t)tn.lanes_per_node : lanes_for_wg(g, block, mem[i]);
            b.replica = inst[i].replica;
            b.wide = g->n && (double)g->nnz / g->n >= 4.0 * b.lanes ? 1u : 0u;
            b.sync = mem[i] > 1 ? d_sync.p + sync_off[i] : nullptr;
            b.members = mem[i];
            b.rank = rnk;
        }
    }
    hipStream_t st = inst[0].graph->stream;
    HIP_TRY(hipMemcpyAsync(d_inst.p, h_inst.data(), h_inst.size() * sizeof(GdiBatchInstance), hipMemcpyHostToDevice, st),
            "upload batch");
    HIP_TRY(hipMemcpyAsync(d_thr.p, tab.data(), tab.size() * 4, hipMemcpyHostToDevice, st), "upload thresholds");
    if ((e = gdi_launch_fill_u64(d_queue.p, 2, st))) return fail(GDI_EDEVICE, gdi_hip_error_string(e));
    if ((e = gdi_launch_fill_u64(reinterpret_cast<uint64_t *>(d_res.p), 2 * (int64_t)n_inst, st)))
        return fail(GDI_EDEVICE, gdi_hip_error_string(e));
    if (clusters && (e = gdi_launch_fill_u64(d_sync.p, (int64_t)sync_words, st)))
        return fail(GDI_EDEVICE, gdi_hip_error_string(e));
    GdiBatchArgs ba{};
    ba.inst = d_inst.p;
    ba.queue = reinterpret_cast<int32_t *>(d_queue.p);
    ba.thr = d_thr.p;
    ba.n_inst = (int32_t)n_tickets;
    ba.error = reinterpret_cast<int64_t *>(d_queue.p + 1);
    ba.spin_limit = kSpinLimit;
    ba.K = K;
    ba.S = S;
    ba.A4 = 4 * s->A;
    ba.B = s->B;
    ba.key0 = (uint32_t)seed;
    ba.key1 = (uint32_t)(seed >> 32);
    ba.snapshot = s->balance_mode == GDI_BAL_SNAPSHOT ? 1u : 0u;
    ba.rule = s->acceptance;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0), "hipEventCreate");
    HIP_TRY(hipEventCreate(&e1), "hipEventCreate");
    struct Ev {
        hipEvent_t &a, &b;
        ~Ev() { if (a) (void)hipEventDestroy(a); if (b) (void)hipEventDestroy(b); }
    } ev{e0, e1};
    HIP_TRY(hipEventRecord(e0, st), "hipEventRecord");
    if ((e = gdi_launch_sweep_batch(ba, (int)grid, (int)block, lds, clusters ? 1 : 0, st)))
        return fail(GDI_EDEVICE, std::string("batched sweep launch: ") + gdi_hip_error_string(e));
    HIP_TRY(hipEventRecord(e1, st), "hipEventRecord");
    HIP_TRY(hipStreamSynchronize(st), "batched sweep");
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
    if (kernel_ms) *kernel_ms = ms;
    int64_t err_flag = 0;
    HIP_TRY(hipMemcpy(&err_flag, d_queue.p + 1, 8, hipMemcpyDeviceToHost), "read batch error flag");
    if (err_flag) return fail(GDI_ETIMEOUT, "a cluster's device-side wait expired; results are invalid");
    if (probe_S) return GDI_OK;
    std::vector<int64_t> res(2 * (size_t)n_inst);
    HIP_TRY(hipMemcpy(res.data(), d_res.p, res.size() * 8, hipMemcpyDeviceToHost), "download batch results");
    for (uint32_t i = 0; i < n_inst; ++i) {
        inst[i].magnetization = res[2 * i];
        inst[i].cut_weighted = res[2 * i + 1];
    }
    if (out_total) {
        std::vector<int8_t> h(out_total);
        HIP_TRY(hipMemcpy(h.data(), d_out.p, out_total, hipMemcpyDeviceToHost), "download batch spins");
        for (uint32_t i = 0; i < n_inst; ++i)
            if (inst[i].spins_out) std::memcpy(inst[i].spins_out, h.data() + out_off[i], (size_t)inst[i].graph->n);
    }
    return GDI_OK;
}

int autotune_batch(gdi_instance *inst, uint32_t n_inst, const gdi_schedule *s, uint64_t seed, uint32_t probe,
                   gdi_tuning *best, double *best_ms)
{
    int rc = check_batch(inst, n_inst, s);
    if (rc) return rc;
    int dev = 0, cus = 0;
    HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev), "hipDeviceGetAttribute");
    probe = std::max<uint32_t>(1, std::min(probe, s->n_sweeps));
    gdi_tuning cur{};
    cur.block = 512;
    double cur_ms = 1e300;
    auto timed = [&](const gdi_tuning &t, double *ms) -> int {
        double a = 0, b = 0;
        int r = run_batch(inst, n_inst, s, seed, t, false, probe, &a);  // the first run also warms caches
        if (r) return r;
        r = run_batch(inst, n_inst, s, seed, t, false, probe, &b);
        if (r) return r;
        *ms = std::min(a, b);
        return GDI_OK;
    };
    // coordinate descent: block size, then lanes per node, then workgroups per CU
    const uint32_t blocks[] = {128, 256, 512, 1024};
    const uint32_t lanes[] = {0, 1, 2, 4, 8, 16, 32};
    for (uint32_t b : blocks) {
        gdi_tuning t = cur;
        t.block = b;
        double ms = 0;
        int r = timed(t, &ms);
        if (r == GDI_EDEVICE) continue;
        if (r) return r;
        if (ms < cur_ms) { cur_ms = ms; cur = t; }
    }
    for (uint32_t l : lanes) {
        gdi_tuning t = cur;
        t.lanes_per_node = l;
        if (l > t.block) continue;
        double ms = 0;
        int r = timed(t, &ms);
        if (r) return r;
        if (ms < cur_ms) { cur_ms = ms; cur = t; }
    }
    for (uint32_t per : {1u, 2u, 4u, 8u}) {
        gdi_tuning t = cur;
        t.grid = per * (uint32_t)cus;
        double ms = 0;
        int r = timed(t, &ms);
        if (r) return r;
        if (ms < cur_ms) { cur_ms = ms; cur = t; }
    }
    // cluster size of the large instances (none, or up to 2..16 workgroups), then the
    // grid once more: clusters run in a cooperative launch of at most 16 waves per CU
    for (int32_t m : {-1, 2, 4, 8, 16}) {
        gdi_tuning t = cur;
        t.batch_members = m;
        double ms = 0;
        int r = timed(t, &ms);
        if (r == GDI_EDEVICE) continue;
        if (r) return r;
        if (ms < cur_ms) { cur_ms = ms; cur = t; }
    }
    for (uint32_t g : {0u, (uint32_t)cus, 2u * (uint32_t)cus, 4u * (uint32_t)cus}) {
        gdi_tuning t = cur;
        if (g == t.grid) continue;
        t.grid = g;
        double ms = 0;
        int r = timed(t, &ms);
        if (r == GDI_EDEVICE) continue;
        if (r) return r;
        if (ms < cur_ms) { cur_ms = ms; cur = t; }
    }
    *best = cur;
    if (best_ms) *best_ms = cur_ms;
    tune_store(batch_key(inst, n_inst), cur, cur_ms);
    return GDI_OK;
}

int anneal_batch(gdi_instance *inst, uint32_t n_inst, const gdi_schedule *s, uint64_t seed, const gdi_tuning *tune,
                 double *kernel_ms, bool dev_out)
{
    int rc = check_batch(inst, n_inst, s);
    if (rc) return rc;
    gdi_tuning t{};
    if (tune) {
        t = *tune;
    } else {
        double cached_ms = 0;
        if (!tune_lookup(batch_key(inst, n_inst), &t, &cached_ms)) {
            double ms = 0;
            rc = autotune_batch(inst, n_inst, s, seed, std::max<uint32_t>(1, s->n_sweeps / 50), &t, &ms);
            if (rc) return rc;
        }
    }
    return run_batch(inst, n_inst, s, seed, t, dev_out, 0, kernel_ms);
}

// ------------------------------------------------------------------ learned proposal
// splitmix64: seeded stream for weight initialisation and minibatch shuffling.
uint64_t splitmix64(uint64_t &x)
{
    uint64_t z = (x += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

struct MlpDevice {
    DevBuf<float> master;
    DevBuf<GdiMlpDev> packed;
    ~MlpDevice() { master.release(); packed.release(); }
};

// Uploads FP32 master weights and packs the BF16 device copy on the stream.
int upload_mlp(const gdi_mlp_weights *w, MlpDevice &m, hipStream_t st)
{
    static_assert(sizeof(gdi_mlp_weights) == GDI_MLP_PARAMS * sizeof(float), "packed parameter layout");
    HIP_TRY(m.master.reserve(GDI_MLP_PARAMS), "hipMalloc network");
    HIP_TRY(m.packed.reserve(1), "hipMalloc network");
    HIP_TRY(hipMemcpyAsync(m.master.p, w, sizeof(gdi_mlp_weights), hipMemcpyHostToDevice, st), "upload network");
    int e = gdi_launch_mlp_pack(m.master.p, m.packed.p, st);
    if (e) return fail(GDI_EDEVICE, gdi_hip_error_string(e));
    return GDI_OK;
}

int learned_impl(gdi_graph *g, const gdi_schedule *s, uint64_t seed, const gdi_mlp_weights *w,
                 const gdi_learned_cfg *cfg, int8_t *spins_out, gdi_learned_result *res)
{
    if (!cfg || !spins_out) return fail(GDI_EINVAL, "NULL argument");
    if (cfg->k_full < 1) return fail(GDI_EINVAL, "k_full must be >= 1");
    if (cfg->skip_mode > GDI_SKIP_HEURISTIC) return fail(GDI_EINVAL, "unknown skip_mode");
    if (cfg->skip_mode == GDI_SKIP_MLP && (!w || !(cfg->skip_threshold > 0.0f && cfg->skip_threshold < 1.0f)))
        return fail(GDI_EINVAL, "the network proposal needs weights and a threshold in (0, 1)");
    if (cfg->skip_mode == GDI_SKIP_HEURISTIC && cfg->heuristic_k < 1) return fail(GDI_EINVAL, "heuristic_k must be >= 1");
    if (s && (s->trace_m || s->trace_cut)) return fail(GDI_EINVAL, "the learned anneal takes no traces");
    if (s && (s->acceptance != GDI_ACCEPT_METROPOLIS || s->flags))
        return fail(GDI_EINVAL, "the learned anneal takes temperatures (Metropolis acceptance) and no flags");
    RunCtx r;
    int rc = prepare_run(g, s, seed, false, r);
    if (rc) return rc;
    hipStream_t st = g->stream;
    const uint32_t S = s->n_sweeps, t_start = s->start_sweep, k = cfg->k_full;
    DevBuf<int32_t> lf;
    DevBuf<uint32_t> mask, part;
    DevBuf<uint64_t> skipped;
    DevBuf<GdiActiveRec> rec;
    MlpDevice net;
    struct Rel {
        DevBuf<int32_t> &a; DevBuf<uint32_t> &b, &c; DevBuf<uint64_t> &d; DevBuf<GdiActiveRec> &e;
        ~Rel() { a.release(); b.release(); c.release(); d.release(); e.release(); }
    } rel{lf, mask, part, skipped, rec};
    const int32_t kParts = 4096;  // workgroup counts of the proposal's mask kernel
    // masked sweeps with few active nodes: one workgroup over the active set, if every
    // spin fits its LDS as a bit
    int dev = 0, lds_max = 0;
    HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
    HIP_TRY(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev), "hipDeviceGetAttribute");
    int32_t amax = cfg->active_max;
    if (amax == 0) amax = r.ch.scope == GDI_SCOPE_WORKGROUP ? g->n : (int32_t)std::min<int64_t>(g->n, 4096LL * g->C);
    const bool use_active = cfg->skip_mode != GDI_SKIP_NONE && amax > 0 &&
                            gdi_active_lds_bytes(g->n_pad, g->C) + 512 <= lds_max;
    if (use_active) HIP_TRY(rec.reserve((size_t)g->n_pad), "hipMalloc learned");
    HIP_TRY(lf.reserve((size_t)g->n_pad), "hipMalloc learned");
    // n_pad is a multiple of 64: n_pad / 32 mask words, an even count, cleared as u64 pairs
    HIP_TRY(mask.reserve((size_t)g->n_pad / 32), "hipMalloc learned");
    HIP_TRY(skipped.reserve(2), "hipMalloc learned");  // [0] all skipped visits, [1] skipped nodes of a block
    int e = gdi_launch_fill_i32(lf.p, g->n_pad, (int32_t)t_start - 1, st);
    if (!e) e = gdi_launch_fill_u64(skipped.p, 2, st);
    if (!e) e = gdi_launch_fill_u64(reinterpret_cast<uint64_t *>(mask.p), (int64_t)g->n_pad / 64, st);
    if (e) return fail(GDI_EDEVICE, gdi_hip_error_string(e));
    float thr_logit = 0.0f;
    if (cfg->skip_mode != GDI_SKIP_NONE) HIP_TRY(part.reserve((size_t)kParts), "hipMalloc learned");
    if (cfg->skip_mode == GDI_SKIP_MLP) {
        if ((rc = upload_mlp(w, net, st))) return rc;
        thr_logit = std::log(cfg->skip_threshold / (1.0f - cfg->skip_threshold));
    }
    std::vector<uint32_t> hmask;
    const uint32_t b0 = std::min(S, std::max(t_start, cfg->learn_from));
    if (cfg->mask_trace)
        std::memset(cfg->mask_trace, 0, (size_t)((S - b0 + k - 1) / k) * (size_t)g->n);
    // On the grid sweep one launch runs a block's masked sweeps and the next block's full
    // sweep (one cooperative launch per block instead of two): the mask stops applying at
    // the block's end, and when the active-set kernel has run the masked sweeps the launch
    // starts at the full sweep.
    const bool merged = r.ch.scope == GDI_SCOPE_GRID;
    HIP_TRY(hipEventRecord(g->ev0, st), "hipEventRecord");
    if (b0 > t_start && (rc = launch_range(g, r, t_start, b0, nullptr, lf.p))) return rc;
    if (merged && b0 < S && (rc = launch_range(g, r, b0, b0 + 1, nullptr, lf.p))) return rc;
    for (uint32_t b = b0; b < S; b += k) {
        if (!merged && (rc = launch_range(g, r, b, b + 1, nullptr, lf.p))) return rc;
        if (b + 1 >= S) break;
        const uint32_t end = std::min<uint32_t>(b + k, S);
        // the sweeps this block's launch on the grid sweep runs: the masked ones, then the
        // next block's full sweep
        const uint32_t t_next = merged ? std::min<uint32_t>(end + 1, S) : end;
        const uint32_t *mp = cfg->skip_mode != GDI_SKIP_NONE ? mask.p : nullptr;
        if (cfg->skip_mode == GDI_SKIP_MLP) {
            // features, network and mask in one kernel, then the block's counts
            e = gdi_launch_mlp_mask(g->d_rp.p, g->d_adj.p, g->d_spin.p, lf.p, g->n_pad, g->d_state.p,
                                    (float)s->temps[b], (int32_t)b, s->A, s->B, g->d_orig.p, net.packed.p, thr_logit,
                                    mask.p, part.p, kParts, skipped.p, end - b - 1, skipped.p + 1, st);
        } else if (cfg->skip_mode == GDI_SKIP_HEURISTIC) {
            e = gdi_launch_mask_age(lf.p, g->d_orig.p, g->n_pad, (int32_t)b, (int32_t)cfg->heuristic_k, mask.p, part.p,
                                    kParts, skipped.p, end - b - 1, skipped.p + 1, st);
        }
        if (e) return fail(GDI_EDEVICE, gdi_hip_error_string(e));
        if (cfg->mask_trace) {
            const size_t words = (size_t)g->n_pad / 32;
            hmask.assign(words, 0u);
            if (mp) HIP_TRY(hipMemcpyAsync(hmask.data(), mask.p, words * 4, hipMemcpyDeviceToHost, st), "download mask");
            HIP_TRY(hipStreamSynchronize(st), "download mask");
            uint8_t *row = cfg->mask_trace + (size_t)((b - b0) / k) * (size_t)g->n;
            for (int32_t v = 0; v < g->n_pad; ++v) {
                const int32_t o = g->rl.orig[(size_t)v];
                if (o >= 0) row[o] = (uint8_t)((hmask[(size_t)v >> 5] >> (v & 31)) & 1u);
            }
        }
        if (mp && use_active) {
            GdiSweepArgs a = r.a;
            a.t0 = b + 1;
            a.S = end;
            a.mask = mp;
            a.last_flip = lf.p;
            a.skip_count = reinterpret_cast<const unsigned long long *>(skipped.p + 1);
            a.active_max = amax;
            a.gate_small = 1;
            a.mask_end = end;
            a.gate_t0 = end;
            if ((e = gdi_launch_sweep_active(a, rec.p, st))) return fail(GDI_EDEVICE, gdi_hip_error_string(e));
            if ((rc = launch_range(g, r, b + 1, t_next, mp, lf.p, skipped.p + 1, amax, merged ? end : 0,
                                   merged ? end : 0)))
                return rc;
        } else if ((rc = launch_range(g, r, b + 1, t_next, mp, lf.p, nullptr, 0, merged && mp ? end : 0))) {
            return rc;
        }
    }
    HIP_TRY(hipEventRecord(g->ev1, st), "hipEventRecord");
    if ((rc = gdi_launch_scatter_out(g->d_orig.p, g->d_spin.p, g->n_pad, g->d_io.p, st)))
        return fail(GDI_EDEVICE, gdi_hip_error_string(rc));
    g->pending = true;
    if ((rc = finish_pending(g))) return rc;
    HIP_TRY(hipMemcpy(spins_out, g->d_io.p, (size_t)g->n, hipMemcpyDeviceToHost), "download spins");
    uint64_t nskip = 0;
    HIP_TRY(hipMemcpy(&nskip, skipped.p, 8, hipMemcpyDeviceToHost), "download counts");
    if (res) {
        res->magnetization = g->last.magnetization;
        res->cut_weighted = g->last.cut_weighted;
        res->total_ms = g->last.sweep_ms;
        res->node_skips = nskip;
        res->node_visits = (uint64_t)g->n * (uint64_t)(S - t_start) - nskip;
    }
    return GDI_OK;
}

int traces_impl(gdi_graph *g, const gdi_schedule *s, uint64_t seed, uint32_t every, uint32_t k_label, void *d_x,
                uint8_t *d_y, uint32_t max_snapshots, uint32_t *n_snapshots)
{
    if (!d_x || !d_y || !n_snapshots) return fail(GDI_EINVAL, "NULL argument");
    if (k_label < 1 || every <= k_label) return fail(GDI_EINVAL, "need every > k_label >= 1");
    if (s && (s->trace_m || s->trace_cut)) return fail(GDI_EINVAL, "no traces here");
    if (s && (s->acceptance != GDI_ACCEPT_METROPOLIS || s->flags))
        return fail(GDI_EINVAL, "trace features take temperatures (Metropolis acceptance) and no flags");
    RunCtx r;
    int rc = prepare_run(g, s, seed, false, r);
    if (rc) return rc;
    hipStream_t st = g->stream;
    DevBuf<int32_t> lf;
    HIP_TRY(lf.reserve((size_t)g->n_pad), "hipMalloc traces");
    int e = gdi_launch_fill_i32(lf.p, g->n_pad, (int32_t)s->start_sweep - 1, st);
    if (e) { lf.release(); return fail(GDI_EDEVICE, gdi_hip_error_string(e)); }
    uint32_t t_cur = s->start_sweep, count = 0;
    for (uint32_t ts = every - 1; ts + k_label < s->n_sweeps && count < max_snapshots; ts += every) {
        if (ts < s->start_sweep) continue;
        if ((rc = launch_range(g, r, t_cur, ts + 1, nullptr, lf.p))) { lf.release(); return rc; }
        e = gdi_launch_features(g->d_rp.p, g->d_adj.p, g->d_spin.p, lf.p, g->n_pad, g->d_state.p,
                                (float)s->temps[ts], (int32_t)ts, s->A, s->B, g->d_orig.p, d_x, 1,
                                (int64_t)count * g->n, st);
        if (e) { lf.release(); return fail(GDI_EDEVICE, gdi_hip_error_string(e)); }
        if ((rc = launch_range(g, r, ts + 1, ts + k_label + 1, nullptr, lf.p))) { lf.release(); return rc; }
        e = gdi_launch_labels(lf.p, g->d_orig.p, g->n_pad, (int32_t)ts, d_y, (int64_t)count * g->n, st);
        if (e) { lf.release(); return fail(GDI_EDEVICE, gdi_hip_error_string(e)); }
        t_cur = ts + k_label + 1;
        ++count;
    }
    hipError_t he = hipStreamSynchronize(st);
    lf.release();
    if (he != hipSuccess) return hip_fail(he, "trace collection");
    int64_t st8[8];
    HIP_TRY(hipMemcpy(st8, g->d_state.p, sizeof(st8), hipMemcpyDeviceToHost), "read state");
    if (st8[3] != 0) return fail(GDI_ETIMEOUT, "a device-side barrier wait expired; traces are invalid");
    *n_snapshots = count;
    return GDI_OK;
}

int train_impl(const void *d_x, const uint8_t *d_y, uint64_t n, gdi_mlp_weights *w, const gdi_train_cfg *cfg,
               float *epoch_loss, hipStream_t st)
{
    if (!d_x || !d_y || !w || !cfg || n == 0) return fail(GDI_EINVAL, "bad argument");
    if (cfg->batch < 16 || n > (uint64_t)INT32_MAX) return fail(GDI_EINVAL, "batch must be >= 16, n < 2^31");
    MlpDevice net;
    DevBuf<float> grad, mo, ve, loss, part;
    DevBuf<int32_t> perm;
    struct Rel {
        DevBuf<float> &a, &b, &c, &d, &f; DevBuf<int32_t> &e;
        ~Rel() { a.release(); b.release(); c.release(); d.release(); f.release(); e.release(); }
    } rel{grad, mo, ve, loss, part, perm};
    int rc = upload_mlp(w, net, st);
    if (rc) return rc;
    HIP_TRY(grad.reserve(GDI_MLP_PARAMS + 1), "hipMalloc training");
    HIP_TRY(part.reserve((size_t)gdi_mlp_grad_part_floats((int32_t)std::min<uint64_t>(cfg->batch, n))),
            "hipMalloc training");
    HIP_TRY(mo.reserve(GDI_MLP_PARAMS + 1), "hipMalloc training");
    HIP_TRY(ve.reserve(GDI_MLP_PARAMS + 1), "hipMalloc training");
    HIP_TRY(loss.reserve(2), "hipMalloc training");
    HIP_TRY(perm.reserve((size_t)n), "hipMalloc training");
    HIP_TRY(hipMemsetAsync(mo.p, 0, (GDI_MLP_PARAMS + 1) * 4, st), "zero Adam state");
    HIP_TRY(hipMemsetAsync(ve.p, 0, (GDI_MLP_PARAMS + 1) * 4, st), "zero Adam state");
    std::vector<int32_t> hp((size_t)n);
    uint64_t rng = cfg->seed;
    uint64_t step = 0;
    for (uint32_t ep = 0; ep < cfg->epochs; ++ep) {
        for (uint64_t i = 0; i < n; ++i) hp[i] = (int32_t)i;
        for (uint64_t i = n - 1; i > 0; --i) std::swap(hp[i], hp[splitmix64(rng) % (i + 1)]);
        HIP_TRY(hipMemcpyAsync(perm.p, hp.data(), n * 4, hipMemcpyHostToDevice, st), "upload minibatch order");
        HIP_TRY(hipMemsetAsync(loss.p, 0, 8, st), "zero loss");
        for (uint64_t off = 0; off < n; off += cfg->batch) {
            const int32_t cnt = (int32_t)std::min<uint64_t>(cfg->batch, n - off);
            ++step;
            // the gradient is written whole, the loss added
            int e = gdi_launch_mlp_grad(d_x, d_y, perm.p + off, cnt, net.packed.p, 1.0f / (float)cnt, part.p, grad.p,
                                        loss.p, st);
            const float bc1 = 1.0f - std::pow(cfg->beta1, (float)step), bc2 = 1.0f - std::pow(cfg->beta2, (float)step);
            if (!e) e = gdi_launch_adam(net.master.p, grad.p, mo.p, ve.p, GDI_MLP_PARAMS, cfg->lr, cfg->beta1, cfg->beta2,
                                        cfg->eps, bc1, bc2, st);
            if (!e) e = gdi_launch_mlp_pack(net.master.p, net.packed.p, st);
            if (e) return fail(GDI_EDEVICE, gdi_hip_error_string(e));
        }
        float l = 0.0f;
        HIP_TRY(hipMemcpyAsync(&l, loss.p, 4, hipMemcpyDeviceToHost, st), "download loss");
        HIP_TRY(hipStreamSynchronize(st), "training");
        if (epoch_loss) epoch_loss[ep] = l / (float)n;
    }
    HIP_TRY(hipMemcpyAsync(w, net.master.p, sizeof(gdi_mlp_weights), hipMemcpyDeviceToHost, st), "download network");
    HIP_TRY(hipStreamSynchronize(st), "training");
    return GDI_OK;
}

}  // namespace

// ====================================================================== C ABI
extern "C" {

int gdi_version(void) { return 100; }

const char *gdi_last_error(void) { return g_err.c_str(); }

int gdi_colour_csr(const int32_t *row_ptr, const int32_t *col_idx, int32_t n, int32_t *colour_out)
{
    if (!row_ptr || !col_idx || !colour_out) return fail(GDI_EINVAL, "NULL argument");
    if (n < 1) return fail(GDI_EINVAL, "n must be >= 1");
    try {
        return gdi_layout::colour_first_fit(row_ptr, col_idx, n, colour_out);
    } catch (const std::bad_alloc &) {
        return fail(GDI_ENOMEM, "out of host memory");
    }
}

int gdi_threshold_table(const double *temps, uint32_t n_sweeps, int32_t width, uint32_t *out)
{
    if (!temps || !out || width < 0) return fail(GDI_EINVAL, "bad argument");
    for (uint32_t t = 0; t < n_sweeps; ++t) {
        if (!(temps[t] > 0.0)) return fail(GDI_EINVAL, "temperatures must be > 0");
        uint32_t *row = out + (size_t)t * (size_t)(width + 1);
        row[0] = 0xFFFFFFFFu;
        for (int32_t d = 1; d <= width; ++d) row[d] = threshold_of(d, temps[t]);
    }
    return GDI_OK;
}

int gdi_philox4x32_10(uint64_t seed, const uint32_t ctr[4], uint32_t out[4])
{
    if (!ctr || !out) return fail(GDI_EINVAL, "NULL argument");
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    for (int r = 0; r < 10; ++r) {
        const uint64_t a = (uint64_t)0xD2511F53u * x0;
        const uint64_t b = (uint64_t)0xCD9E8D57u * x2;
        const uint32_t y0 = (uint32_t)(b >> 32) ^ x1 ^ k0;
        const uint32_t y2 = (uint32_t)(a >> 32) ^ x3 ^ k1;
        x0 = y0;
        x1 = (uint32_t)b;
        x2 = y2;
        x3 = (uint32_t)a;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
    return GDI_OK;
}

int gdi_create(const int32_t *row_ptr, const int32_t *col_idx, const int32_t *weights, int32_t n,
               gdi_graph **out)
{
    if (!out) return fail(GDI_EINVAL, "NULL out");
    *out = nullptr;
    gdi_graph *g = nullptr;
    try {
        int64_t mw = 0;
        int32_t md = 0;
        int rc = validate_csr(row_ptr, col_idx, weights, n, &mw, &md);
        if (rc) return rc;
        g = new gdi_graph();
        g->n = n;
        g->nnz = row_ptr[n];
        g->max_abs_wdeg = mw;
        g->max_degree = md;
        g->colour.assign((size_t)n, 0);
        g->C = gdi_layout::colour_first_fit(row_ptr, col_idx, n, g->colour.data());
        if ((rc = check_device())) { delete g; return rc; }
        // set-up of the allocation-free entry point on this device: the address of its
        // fixed scratch array (looked up once per device)
        void *scratch = nullptr;
        if (int e = gdi_scratch_ptr(&scratch)) {
            delete g;
            return fail(GDI_EDEVICE, std::string("scratch address: ") + gdi_hip_error_string(e));
        }
        if ((rc = upload(g, row_ptr, col_idx, weights))) { delete g; return rc; }
    } catch (const std::bad_alloc &) {
        delete g;
        return fail(GDI_ENOMEM, "out of host memory");
    }
    *out = g;
    return GDI_OK;
}

void gdi_destroy(gdi_graph *g)
{
    if (!g) return;
    if (g->pending) (void)hipStreamSynchronize(g->stream);
    delete g;
}

int gdi_set_stream(gdi_graph *g, void *hip_stream)
{
    if (!g) return fail(GDI_ESTATE, "NULL handle");
    int rc = finish_pending(g);
    if (rc) return rc;
    g->stream = (hipStream_t)hip_stream;
    return GDI_OK;
}

int gdi_set_tuning(gdi_graph *g, const gdi_tuning *tune)
{
    if (!g) return fail(GDI_ESTATE, "NULL handle");
    if (tune) {
        g->tune = *tune;
        g->have_tune = true;
    } else {
        g->have_tune = false;
    }
    return GDI_OK;
}

int gdi_anneal(gdi_graph *g, const gdi_schedule *s, uint64_t seed, int8_t *spins_out)
{
    if (!spins_out) return fail(GDI_EINVAL, "NULL spins_out");
    try {
        return anneal_impl(g, s, seed, spins_out, nullptr);
    } catch (const std::bad_alloc &) {
        return fail(GDI_ENOMEM, "out of host memory");
    }
}

int gdi_anneal_dev(gdi_graph *g, const gdi_schedule *s, uint64_t seed, int8_t *d_spins_out)
{
    if (!d_spins_out) return fail(GDI_EINVAL, "NULL d_spins_out");
    try {
        return anneal_impl(g, s, seed, nullptr, d_spins_out);
    } catch (const std::bad_alloc &) {
        return fail(GDI_ENOMEM, "out of host memory");
    }
}

int gdi_last_result(gdi_graph *g, gdi_result *out)
{
    if (!g) return fail(GDI_ESTATE, "NULL handle");
    if (!out) return fail(GDI_EINVAL, "NULL out");
    int rc = finish_pending(g);
    if (rc) return rc;
    if (!g->last_valid) return fail(GDI_ESTATE, "no completed anneal on this handle");
    *out = g->last;
    return GDI_OK;
}

int gdi_cut(gdi_graph *g, const int8_t *spins, int64_t *cut_weighted, int64_t *cut_edges,
            int64_t *magnetization)
{
    try {
        return cut_impl(g, spins, false, cut_weighted, cut_edges, magnetization);
    } catch (const std::bad_alloc &) {
        return fail(GDI_ENOMEM, "out of host memory");
    }
}

int gdi_cut_dev(gdi_graph *g, const int8_t *d_spins, int64_t *cut_weighted, int64_t *cut_edges,
                int64_t *magnetization)
{
    try {
        return cut_impl(g, d_spins, true, cut_weighted, cut_edges, magnetization);
    } catch (const std::bad_alloc &) {
        return fail(GDI_ENOMEM, "out of host memory");
    }
}

int gdi_cut_dev_noalloc(gdi_graph *g, const int8_t *d_spins, int64_t *d_out)
{
    if (!g) return fail(GDI_ESTATE, "NULL handle");
    if (!d_spins || !d_out) return fail(GDI_EINVAL, "NULL device pointer");
    if ((int64_t)g->n_pad > GDI_NOALLOC_MAX_NODES)
        return fail(GDI_ERANGE, "graph too large for the fixed scratch array (n + 64 * colours must be <= " +
                                    std::to_string(GDI_NOALLOC_MAX_NODES) + ")");
    if (g->C > GDI_NOALLOC_MAX_C)
        return fail(GDI_ERANGE, "more than " + std::to_string(GDI_NOALLOC_MAX_C) + " colour classes");
    void *base = nullptr;
    if (int e = gdi_scratch_ptr(&base)) return fail(GDI_EDEVICE, std::string("scratch address: ") + gdi_hip_error_string(e));
    int64_t *red = static_cast<int64_t *>(base);
    int32_t *P = reinterpret_cast<int32_t *>(static_cast<unsigned char *>(base) + 256);
    int8_t *sp = reinterpret_cast<int8_t *>(static_cast<unsigned char *>(base) + GDI_NOALLOC_SPIN_OFF);
    uint32_t *bits = reinterpret_cast<uint32_t *>(static_cast<unsigned char *>(base) + GDI_NOALLOC_SPIN_OFF +
                                                  (((size_t)g->n_pad + 255) & ~(size_t)255));
    hipStream_t st = g->stream;
    // the accumulators and counts keep the last call's values: the reduction's first
    // kernel clears them (a kernel, not a memset)
    int rc = gdi_launch_gather_in(g->d_orig.p, d_spins, g->n_pad, sp, st);
    if (!rc) rc = gdi_launch_reduce(g->d_rp.p, g->d_adj.p, sp, g->n_pad, g->nnz, g->d_cbeg.p, g->d_csz.p, g->C, red, P, bits, st);
    if (!rc) rc = gdi_launch_cut_finish(red, d_out, st);
    if (rc) return fail(GDI_EDEVICE, gdi_hip_error_string(rc));
    return GDI_OK;
}

int gdi_anneal_batch(gdi_instance *inst, uint32_t n_inst, const gdi_schedule *s, uint64_t seed,
                     const gdi_tuning *tune, double *kernel_ms)
{
    try {
        return anneal_batch(inst, n_inst, s, seed, tune, kernel_ms, false);
    } catch (const std::bad_alloc &) {
        return fail(GDI_ENOMEM, "out of host memory");
    }
}

int gdi_anneal_batch_dev(gdi_instance *inst, uint32_t n_inst, const gdi_schedule *s, uint64_t seed,
                         const gdi_tuning *tune, double *kernel_ms)
{
    try {
        return anneal_batch(inst, n_inst, s, seed, tune, kernel_ms, true);
    } catch (const std::bad_alloc &) {
        return fail(GDI_ENOMEM, "out of host memory");
    }
}

int gdi_autotune_batch(gdi_instance *inst, uint32_t n_inst, const gdi_schedule *s, uint64_t seed,
                       uint32_t probe_sweeps, gdi_tuning *best, double *best_ms)
{
    if (!best) return fail(GDI_EINVAL, "NULL best");
    try {
        return autotune_batch(inst, n_inst, s, seed, probe_sweeps, best, best_ms);
    } catch (const std::bad_alloc &) {
        return fail(GDI_ENOMEM, "out of host memory");
    }
}

int gdi_autotune(gdi_graph *g, const gdi_schedule *s, uint64_t seed, uint32_t probe_sweeps, int use_cache,
                 gdi_tuning *best, double *best_ms)
{
    if (!best) return fail(GDI_EINVAL, "NULL best");
    if (!g) return fail(GDI_ESTATE, "NULL handle");
    try {
        if (use_cache) {
            gdi_tuning t{};
            double ms = 0;
            if (tune_lookup(graph_key(g), &t, &ms)) {
                g->tune = t;
                g->have_tune = true;
                *best = t;
                if (best_ms) *best_ms = ms;
                return GDI_OK;
            }
        }
        return autotune_graph(g, s, seed, probe_sweeps, best, best_ms);
    } catch (const std::bad_alloc &) {
        return fail(GDI_ENOMEM, "out of host memory");
    }
}

int gdi_tune_cache_load(const char *path)
{
    if (!path) return fail(GDI_EINVAL, "NULL path");
    try {
        std::string text, err;
        if (!gdi_tunecache::read_file(path, &text)) return fail(GDI_EINVAL, std::string("cannot read ") + path);
        std::lock_guard<std::mutex> lk(g_tune_mu);
        tune_env_read_locked();
        if (gdi_tunecache::parse(text, &g_tune_table, &err)) return fail(GDI_EINVAL, std::string(path) + ": " + err);
        return GDI_OK;
    } catch (const std::bad_alloc &) {
        return fail(GDI_ENOMEM, "out of host memory");
    }
}

int gdi_tune_cache_save(const char *path)
{
    if (!path) return fail(GDI_EINVAL, "NULL path");
    try {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        tune_env_read_locked();
        if (!gdi_tunecache::write_file(path, gdi_tunecache::dump(g_tune_table)))
            return fail(GDI_EINVAL, std::string("cannot write ") + path);
        return GDI_OK;
    } catch (const std::bad_alloc &) {
        return fail(GDI_ENOMEM, "out of host memory");
    }
}

int gdi_tune_cache_clear(void)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_env_read = true;  // a cleared cache is not refilled from GDI_TUNE_CACHE
    g_tune_table.clear();
    return GDI_OK;
}

int gdi_tune_cache_size(void)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_env_read_locked();
    return (int)std::min<size_t>(g_tune_table.size(), 0x7FFFFFFF);
}

int gdi_anneal_learned(gdi_graph *g, const gdi_schedule *s, uint64_t seed, const gdi_mlp_weights *w,
                       const gdi_learned_cfg *cfg, int8_t *spins_out, gdi_learned_result *res)
{
    try {
        return learned_impl(g, s, seed, w, cfg, spins_out, res);
    } catch (const std::bad_alloc &) {
        return fail(GDI_ENOMEM, "out of host memory");
    }
}

int gdi_collect_traces(gdi_graph *g, const gdi_schedule *s, uint64_t seed, uint32_t every, uint32_t k_label,
                       void *d_x, uint8_t *d_y, uint32_t max_snapshots, uint32_t *n_snapshots)
{
    try {
        return traces_impl(g, s, seed, every, k_label, d_x, d_y, max_snapshots, n_snapshots);
    } catch (const std::bad_alloc &) {
        return fail(GDI_ENOMEM, "out of host memory");
    }
}

int gdi_mlp_init(gdi_mlp_weights *w, uint64_t seed)
{
    if (!w) return fail(GDI_EINVAL, "NULL weights");
    uint64_t x = seed;
    auto uni = [&](float a) { return (float)((double)(splitmix64(x) >> 11) * 0x1.0p-53 * 2.0 - 1.0) * a; };
    for (int h = 0; h < 64; ++h)
        for (int f = 0; f < 6; ++f) w->w1[h][f] = uni(std::sqrt(6.0f / 6.0f));
    for (int h = 0; h < 64; ++h)
        for (int k = 0; k < 64; ++k) w->w2[h][k] = uni(std::sqrt(6.0f / 64.0f));
    for (int h = 0; h < 64; ++h) {
        w->b1[h] = 0.0f;
        w->b2[h] = 0.0f;
        w->w3[h] = uni(std::sqrt(3.0f / 64.0f));
    }
    w->b3 = 0.0f;
    return GDI_OK;
}

int gdi_mlp_train(const void *d_x, const uint8_t *d_y, uint64_t n, gdi_mlp_weights *w, const gdi_train_cfg *cfg,
                  float *epoch_loss, void *hip_stream)
{
    try {
        return train_impl(d_x, d_y, n, w, cfg, epoch_loss, (hipStream_t)hip_stream);
    } catch (const std::bad_alloc &) {
        return fail(GDI_ENOMEM, "out of host memory");
    }
}

int gdi_mlp_forward(const gdi_mlp_weights *w, const void *d_x, uint32_t n, float *d_logits, void *hip_stream)
{
    if (!w || !d_x || !d_logits || n == 0) return fail(GDI_EINVAL, "bad argument");
    hipStream_t st = (hipStream_t)hip_stream;
    MlpDevice net;
    int rc = upload_mlp(w, net, st);
    if (rc) return rc;
    int e = gdi_launch_mlp_infer(d_x, (int32_t)n, net.packed.p, 0.0f, nullptr, d_logits, st);
    if (e) return fail(GDI_EDEVICE, gdi_hip_error_string(e));
    HIP_TRY(hipStreamSynchronize(st), "network forward");
    return GDI_OK;
}

int gdi_mlp_gradient(const gdi_mlp_weights *w, const void *d_x, const uint8_t *d_y, uint32_t n,
                     gdi_mlp_weights *grad, float *loss, void *hip_stream)
{
    if (!w || !d_x || !d_y || !grad || n == 0) return fail(GDI_EINVAL, "bad argument");
    hipStream_t st = (hipStream_t)hip_stream;
    if (n > (uint32_t)INT32_MAX) return fail(GDI_EINVAL, "n must be < 2^31");
    MlpDevice net;
    DevBuf<float> gbuf, part;
    struct Rel {
        DevBuf<float> &a, &b;
        ~Rel() { a.release(); b.release(); }
    } rel{gbuf, part};
    int rc = upload_mlp(w, net, st);
    if (rc) return rc;
    HIP_TRY(gbuf.reserve(GDI_MLP_PARAMS + 2), "hipMalloc gradient");
    HIP_TRY(part.reserve((size_t)gdi_mlp_grad_part_floats((int32_t)n)), "hipMalloc gradient");
    HIP_TRY(hipMemsetAsync(gbuf.p, 0, (GDI_MLP_PARAMS + 2) * 4, st), "zero gradient");
    int e = gdi_launch_mlp_grad(d_x, d_y, nullptr, (int32_t)n, net.packed.p, 1.0f / (float)n, part.p, gbuf.p,
                                gbuf.p + GDI_MLP_PARAMS + 1, st);
    if (e) return fail(GDI_EDEVICE, gdi_hip_error_string(e));
    std::vector<float> h(GDI_MLP_PARAMS + 2);
    hipError_t he = hipMemcpyAsync(h.data(), gbuf.p, h.size() * 4, hipMemcpyDeviceToHost, st);
    if (he == hipSuccess) he = hipStreamSynchronize(st);
    if (he != hipSuccess) return hip_fail(he, "network gradient");
    std::memcpy(grad, h.data(), sizeof(gdi_mlp_weights));
    if (loss) *loss = h[GDI_MLP_PARAMS + 1] / (float)n;
    return GDI_OK;
}

int gdi_get_info(const gdi_graph *g, gdi_graph_info *out)
{
    if (!g) return fail(GDI_ESTATE, "NULL handle");
    if (!out) return fail(GDI_EINVAL, "NULL out");
    out->n = g->n;
    out->n_colours = g->C;
    out->nnz = g->nnz;
    out->max_abs_wdeg = g->max_abs_wdeg;
    out->max_degree = g->max_degree;
    out->pad = 0;
    return GDI_OK;
}

int gdi_get_colouring(const gdi_graph *g, int32_t *colour_out, int32_t *class_size_out)
{
    if (!g) return fail(GDI_ESTATE, "NULL handle");
    if (colour_out) std::memcpy(colour_out, g->colour.data(), (size_t)g->n * 4);
    if (class_size_out) std::memcpy(class_size_out, g->rl.csz.data(), (size_t)g->C * 4);
    return GDI_OK;
}

}  // extern "C"
