// gdi_halo.hip -- the fence-free grid sweep (k_sweep_halo) of the GDI annealer for
// gfx950: every co-resident workgroup owns a chunk of every colour class, keeps the
// spin bits its nodes read in LDS, and hands spins and the per-phase change of the
// magnetisation to the others as epoch-tagged words (Sec. V Alg. 3 with colour phases).

#include <hip/hip_runtime.h>

#include <algorithm>

#include "gdi_internal.h"
#include "gdi_device.h"

// Optional per-phase timestamps for studying the grid sweep (off unless the
// library is compiled with -DGDI_PHASE_TIMING; the product build has none).
#ifdef GDI_PHASE_TIMING
__device__ unsigned long long *g_tbuf;
__device__ int g_tfirst;
__device__ int g_tphases;
#define GDI_TSTAMP(slot, cond)                                                                      \
    do {                                                                                          \
        if ((cond) && g_tbuf && (int)p >= g_tfirst && (int)p < g_tfirst + g_tphases)              \
            g_tbuf[((size_t)(p - g_tfirst) * gridDim.x + blockIdx.x) * 8 + (slot)] =              \
                __builtin_amdgcn_s_memrealtime();                                                 \
    } while (0)
#else
#define GDI_TSTAMP(slot, cond) \
    do {                       \
    } while (0)
#endif

namespace {

// ------------------------------------------------------------------ grid scope, fence-free
// Every value one workgroup hands to another travels in a self-describing 64-bit
// word (epoch << 32 | payload) written and read with agent-scope atomics, so no
// cache-wide release/acquire fence is needed: a reader that sees the epoch it
// waits for sees the payload of the same store.
//   * spins: after the phase of class c, each owner republishes every packed word
//     of its chunk with the phase's epoch; readers poll only their foreign words of
//     class c (the words of that class their nodes read and another workgroup owns)
//     and copy the bits into LDS;
//   * dM: each workgroup posts (epoch, dM) in its member word (the members of one
//     group are contiguous, so a leader polls two cache lines); the leader of each
//     group (workgroups b = x mod 8) sums its members' words and posts
//     (epoch, group sum) in the group word of the phase's parity; everyone sums
//     the 8 group words.
// A word can only be overwritten after every reader has consumed it: member and
// chunk words are rewritten at the earliest one full barrier later, group words
// alternate by phase parity. All waits are bounded by spin_limit.

__device__ __forceinline__ int32_t lds_spin(const uint32_t *bits, int32_t lb)
{
    return (int32_t)((bits[lb >> 5] >> (lb & 31)) & 1u) * 2 - 1;
}

// Spin bits (1 = +1) of packed word wd, read from the int8 spin array: 32 spins, two
// 16-byte loads; a byte is +1 when its low bit is set and its sign bit clear.
__device__ __forceinline__ uint32_t pack_spins(const int8_t *spin, int32_t wd)
{
    const uint4 *p = reinterpret_cast<const uint4 *>(spin + (size_t)wd * 32);
    const uint4 lo = p[0], hi = p[1];
    const uint32_t x[8] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
    uint32_t word = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const uint32_t y = x[i] & ~(x[i] >> 7) & 0x01010101u;
        word |= ((y | (y >> 7) | (y >> 14) | (y >> 21)) & 0xFu) << (4 * i);
    }
    return word;
}

// Polls foreign words first, first + stride, ... of one class until they carry
// `epoch`, copying their bits to LDS. Returns false when the bounded wait expires or
// another thread has aborted.
__device__ __forceinline__ bool poll_foreign(const GdiHaloArgs &h, const GdiHaloEntry &e, uint32_t *bits,
                                             uint32_t epoch, int first, int stride, int32_t *abort_sh)
{
    for (int32_t i = first; i < e.for_len; i += stride) {
        const uint64_t *src = h.words + (int32_t)bits[e.list_off + i];
        for (int64_t tries = 0;; ++tries) {
            const uint64_t w = ld_agent(src);
            if ((uint32_t)(w >> 32) >= epoch) {
                bits[e.for_off + i] = (uint32_t)w;
                break;
            }
            if (tries >= h.base.spin_limit || aborted(abort_sh)) return false;
            __builtin_amdgcn_s_sleep(1);
        }
    }
    return true;
}

// Per-node state carried across barriers. Everything of a node's update that
// does not depend on spins is loaded ahead: the row bounds and original id two
// phases ahead (RowAhead), the CSR entries and Philox words one phase ahead
// (NodePrefetch), so that no load issued while waiting depends on another.
struct RowAhead {
    int32_t r0, r1, id;
};

struct NodePrefetch {
    uint32_t r0t;              // row start (< 2^31) | low bit of Philox word x2 << 31 (paper rule's tie)
    int32_t deg;
    uint32_t x0, x1;
    uint32_t e[GDI_HALO_PF];  // packed entries (see ent_word / ent_bit / ent_w)
};

// Packed CSR entry of the halo sweep: the LDS word holding the neighbour's spin bit in
// bits 16..31, the weight as an 11-bit two's-complement number in bits 5..15, and the
// bit's position in that word in bits 0..4 (so a bit-field extract can take the entry
// itself as its offset operand).
__device__ __forceinline__ int32_t ent_word(uint32_t e) { return (int32_t)(e >> 16); }
__device__ __forceinline__ uint32_t ent_bit(uint32_t word, uint32_t e) { return (word >> (e & 31u)) & 1u; }
__device__ __forceinline__ int32_t ent_w(uint32_t e) { return (int32_t)(e << 16) >> 21; }

// Local field over the first `cnt` of GDI_HALO_PF loaded entries; the rest belong to
// later rows (or are the zero padding) and count for nothing. Every entry names a word
// inside every workgroup's LDS image, so all GDI_HALO_PF words are read, each before any
// is used (the reads overlap). With h = 2 * sum(w over +1 neighbours) - sum(w): for unit
// weights the first sum is a population count over a mask of neighbour bits.
__device__ __forceinline__ int32_t field_sum(const uint32_t *bits, const uint32_t (&e)[GDI_HALO_PF], int32_t cnt,
                                             bool unit)
{
    const int32_t c = cnt < GDI_HALO_PF ? cnt : GDI_HALO_PF;
    uint32_t wv[GDI_HALO_PF];
#pragma unroll
    for (int k = 0; k < GDI_HALO_PF; ++k) wv[k] = bits[ent_word(e[k])];
    if (unit) {
        uint32_t m = 0;
#pragma unroll
        for (int k = 0; k < GDI_HALO_PF; ++k) m |= ent_bit(wv[k], e[k]) << k;
        return 2 * __popc(m & ((1u << c) - 1u)) - c;
    }
    int32_t s = 0, W = 0;
#pragma unroll
    for (int k = 0; k < GDI_HALO_PF; ++k) {
        const int32_t w = k < c ? ent_w(e[k]) : 0;
        s += (int32_t)ent_bit(wv[k], e[k]) * w;
        W += w;
    }
    return 2 * s - W;
}

// GDI_HALO_PF consecutive packed entries from index k0, as 16-byte loads. Rows start at
// any entry, so the loads are only dword-aligned; the packed CSR carries GDI_HALO_PF zero
// entries after its last row, so the loads stay inside it for every k0 <= nnz.
typedef uint32_t gdi_u32x4 __attribute__((ext_vector_type(4)));
typedef gdi_u32x4 gdi_u32x4_a4 __attribute__((aligned(4)));
__device__ __forceinline__ void load_run(const uint32_t *adjL, int32_t k0, uint32_t (&e)[GDI_HALO_PF])
{
    const gdi_u32x4_a4 *src = reinterpret_cast<const gdi_u32x4_a4 *>(adjL + k0);
#pragma unroll
    for (int q = 0; q < GDI_HALO_PF / 4; ++q) {
        const gdi_u32x4 v = src[q];
        e[4 * q] = v.x;
        e[4 * q + 1] = v.y;
        e[4 * q + 2] = v.z;
        e[4 * q + 3] = v.w;
    }
}

// Local field over packed entries src[k0, k1) held in LDS (the tail's CSR, or a long
// row's overflow entries): eight entries are read before their spin words, and those
// before any is used, so the LDS latencies overlap. Past k1 the zero entry (bit 0,
// weight 0) adds nothing.
__device__ __forceinline__ int32_t lds_field(const uint32_t *bits, const uint32_t *src, int32_t k0, int32_t k1)
{
    int32_t hv = 0;
    for (int32_t k = k0; k < k1; k += 8) {
        uint32_t ee[8], wv[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) ee[j] = k + j < k1 ? src[k + j] : 0u;
#pragma unroll
        for (int j = 0; j < 8; ++j) wv[j] = bits[ent_word(ee[j])];
#pragma unroll
        for (int j = 0; j < 8; ++j) hv += ent_w(ee[j]) * ((int32_t)ent_bit(wv[j], ee[j]) * 2 - 1);
    }
    return hv;
}

// Local field of a row whose first GDI_HALO_PF entries are in registers. A longer row
// continues in the LDS overflow region at the word its entry GDI_HALO_PF - 1 names;
// without that region, the entries past GDI_HALO_PF are loaded GDI_HALO_PF at a time,
// every load of a batch issued before any is used (one memory round trip per batch).
template <bool UNIT>
__device__ __forceinline__ int32_t row_field(const GdiHaloArgs &h, const uint32_t *bits, const NodePrefetch &q)
{
    const bool linked = h.ovf_len > 0 && q.deg > GDI_HALO_PF;
    int32_t hv = field_sum(bits, q.e, linked ? GDI_HALO_PF - 1 : q.deg, UNIT);
    if (linked) {
        const int32_t k0 = (int32_t)q.e[GDI_HALO_PF - 1];
        return hv + lds_field(bits, bits, k0, k0 + q.deg - (GDI_HALO_PF - 1));
    }
    for (int32_t k0 = GDI_HALO_PF; k0 < q.deg; k0 += GDI_HALO_PF) {
        uint32_t ex[GDI_HALO_PF];
        load_run(h.adjL, (int32_t)(q.r0t & 0x7FFFFFFFu) + k0, ex);
        hv += field_sum(bits, ex, q.deg - k0, UNIT);
    }
    return hv;
}

__device__ __forceinline__ void load_row(const GdiSweepArgs &a, int32_t v, RowAhead &ra)
{
    ra.r0 = a.rp[v];
    ra.r1 = a.rp[v + 1];
    ra.id = a.orig[v];
}

__device__ __forceinline__ void load_entries(const GdiHaloArgs &h, const RowAhead &ra, uint32_t t,
                                             NodePrefetch &pf)
{
    const GdiSweepArgs &a = h.base;
    // The CSR loads go out first and the Philox words are drawn while they are in
    // flight. The id (loaded a phase ago) is pinned in a register before the loads are
    // issued, so the Philox rounds never wait on them (vector memory counters complete
    // in order, and a wait for a value loaded earlier would count the new loads too).
    uint32_t id = (uint32_t)ra.id;
    asm volatile("" : "+v"(id));
    pf.deg = ra.r1 - ra.r0;
    // every load is issued unconditionally, whatever the degree (field_sum drops the
    // entries past the row): a register that is zeroed and then conditionally loaded
    // makes the compiler wait for all earlier loads before zeroing it
    load_run(h.adjL, ra.r0, pf.e);
    const Words4 w = philox10(id, t, a.replica, 0u, a.key0, a.key1);
    pf.x0 = w.w0;
    pf.x1 = w.w1;
    pf.r0t = (uint32_t)ra.r0 | (w.w2 << 31);
}

// Metropolis decision with the node's Philox words already drawn. The threshold
// row is read from LDS when staged there (thr_l), else from global memory (thr_g).
__device__ __forceinline__ bool decide_words(const GdiSweepArgs &a, int32_t sigma, int32_t h,
                                             const PhaseView &pv, const uint32_t *thr_l, const uint32_t *thr_g,
                                             bool in_lds, uint32_t x0, uint32_t x1, uint32_t x2)
{
    int32_t m_seen;
    if (a.snapshot) {
        m_seen = pv.M0;
    } else {
        const bool gated = pv.D > 0 && sigma == pv.s &&
                           ((uint64_t)x1 * pv.O < ((uint64_t)(uint32_t)pv.D << 32));
        m_seen = gated ? pv.M0 : 0;
    }
    const int32_t dE = a.B * sigma * h + a.A4 * (1 - sigma * m_seen);
    if (a.rule) return paper_flip(dE, sigma, x0, x2, thr_at(thr_l, thr_g, in_lds, 0));
    if (dE <= 0) return true;
    if (dE > a.K) return false;
    return x0 < thr_at(thr_l, thr_g, in_lds, dE);
}

// Polls the tail's gather words of class c until they carry `epoch`, copying their
// bits into the gather region. Same bounded wait as poll_foreign.
__device__ __forceinline__ bool poll_gather(const GdiHaloArgs &h, int32_t c, uint32_t *bits, uint32_t epoch,
                                            int first, int stride, int32_t *abort_sh)
{
    const int32_t g1 = h.gat_beg[c + 1];
    for (int32_t i = h.gat_beg[c] + first; i < g1; i += stride) {
        const uint64_t *src = h.words + h.gat_words[i];
        for (int64_t tries = 0;; ++tries) {
            const uint64_t w = ld_agent(src);
            if ((uint32_t)(w >> 32) >= epoch) {
                bits[h.gather_off + i] = (uint32_t)w;
                break;
            }
            if (tries >= h.base.spin_limit || aborted(abort_sh)) return false;
            __builtin_amdgcn_s_sleep(1);
        }
    }
    return true;
}

// The polls after the phase of class c: the foreign words of class c (carrying
// `epoch`) and, with a tail, the gather words of class cg = c - 1 (carrying `epoch_g`,
// published a phase earlier, so they are there by now and no workgroup waits here for
// the slowest owner anywhere in the grid). A thread's first foreign word and first
// gather word (packed-word id gidx, loaded earlier, or -1) are loaded together, so
// their latencies overlap; further words, if any, use the loops above.
__device__ __forceinline__ bool poll_phase_words(const GdiHaloArgs &h, const GdiHaloEntry &e, int32_t cg, int32_t gidx,
                                                 uint32_t *bits, uint32_t epoch, uint32_t epoch_g, int tid, int nwork,
                                                 int32_t *abort_sh)
{
    const bool hw = tid < e.for_len, hg = gidx >= 0;
    const uint64_t *fsrc = h.words + (hw ? (int32_t)bits[e.list_off + tid] : 0);
    bool ok0 = !hw, ok1 = !hg;
    for (int64_t tries = 0;; ++tries) {
        const uint64_t w0 = ok0 ? 0 : ld_agent(fsrc);
        const uint64_t w1 = ok1 ? 0 : ld_agent(h.words + gidx);
        if (!ok0 && (uint32_t)(w0 >> 32) >= epoch) {
            bits[e.for_off + tid] = (uint32_t)w0;
            ok0 = true;
        }
        if (!ok1 && (uint32_t)(w1 >> 32) >= epoch_g) {
            bits[h.gather_off + h.gat_beg[cg] + tid] = (uint32_t)w1;
            ok1 = true;
        }
        if (ok0 && ok1) break;
        if (tries >= h.base.spin_limit || aborted(abort_sh)) return false;
        __builtin_amdgcn_s_sleep(1);
    }
    if (e.for_len > nwork && !poll_foreign(h, e, bits, epoch, tid + nwork, nwork, abort_sh)) return false;
    if (hg && h.gat_beg[cg + 1] - h.gat_beg[cg] > nwork) {
        for (int32_t i = h.gat_beg[cg] + tid + nwork; i < h.gat_beg[cg + 1]; i += nwork) {
            const uint64_t *src = h.words + h.gat_words[i];
            for (int64_t tries = 0;; ++tries) {
                const uint64_t w = ld_agent(src);
                if ((uint32_t)(w >> 32) >= epoch_g) {
                    bits[h.gather_off + i] = (uint32_t)w;
                    break;
                }
                if (tries >= h.base.spin_limit || aborted(abort_sh)) return false;
                __builtin_amdgcn_s_sleep(1);
            }
        }
    }
    return true;
}

// Copies of up to three global ranges into LDS as one index space, PRO_INFLIGHT loads
// per thread issued before any store, so the copies cost one memory round trip per
// PRO_INFLIGHT x nth words rather than one per range.
#define PRO_INFLIGHT 8
struct LdsCopy {
    uint32_t *dst;
    const uint32_t *src;
    int32_t n;
};
__device__ __forceinline__ void copy_ranges(const LdsCopy (&r)[3], int tid, int nth)
{
    const int32_t n01 = r[0].n + r[1].n, total = n01 + r[2].n;
    for (int32_t base = 0; base < total; base += PRO_INFLIGHT * nth) {
        uint32_t v[PRO_INFLIGHT];
#pragma unroll
        for (int u = 0; u < PRO_INFLIGHT; ++u) {
            const int32_t i = base + u * nth + tid;
            v[u] = 0u;
            if (i < r[0].n) v[u] = r[0].src[i];
            else if (i < n01) v[u] = r[1].src[i - r[0].n];
            else if (i < total) v[u] = r[2].src[i - n01];
        }
#pragma unroll
        for (int u = 0; u < PRO_INFLIGHT; ++u) {
            const int32_t i = base + u * nth + tid;
            if (i < r[0].n) r[0].dst[i] = v[u];
            else if (i < n01) r[1].dst[i - r[0].n] = v[u];
            else if (i < total) r[2].dst[i - n01] = v[u];
        }
    }
}

// Node of worker thread tid in the first pass of class s, or -1.
__device__ __forceinline__ int32_t step_node(const GdiHaloArgs &h, const GdiHaloEntry *tab, int32_t s, int tid)
{
    const int32_t v = tab[s].node_lo + tid;
    return v < tab[s].node_hi ? v : -1;
}

// UNIT: every weight is 1 (the local fields reduce to population counts)
template <bool UNIT>
__global__ void __launch_bounds__(GDI_MAX_BLOCK) k_sweep_halo(GdiHaloArgs h)
{
    const GdiSweepArgs &a = h.base;
    // sweeps t_begin..S-1 (t_begin is t0, or gate_t0 when the launch gate is closed)
    const uint32_t t_begin = launch_begin(a);
    if (t_begin >= a.S) return;
    extern __shared__ uint32_t lds[];
    uint32_t *bits = lds;                                                   // image, gather, tail, lists
    GdiHaloEntry *tab = reinterpret_cast<GdiHaloEntry *>(lds + h.lds_words); // C entries
    int32_t *Psh = reinterpret_cast<int32_t *>(tab + a.C);                  // C counts of +1
    int32_t *csz_sh = Psh + a.C;                                            // C class sizes
    uint32_t *thr_sh = reinterpret_cast<uint32_t *>(csz_sh + a.C);          // 2 x (K+1) thresholds
    __shared__ int32_t wg_acc;
    __shared__ int32_t total_sh;
    __shared__ int32_t abort_sh;
    __shared__ int32_t tacc[3];
    __shared__ uint32_t wdone;  // worker waves whose polls are done (running count)
    __shared__ int64_t dcut_sh;  // the workgroup's cut change, summed at the end

    const int tid = threadIdx.x, nth = blockDim.x;
    const int wave = tid >> 6, lane = tid & 63, nwaves = nth >> 6;
    const uint32_t G = gridDim.x, b = blockIdx.x;
    const uint32_t ngroups = G < 8u ? G : 8u;
    const uint32_t x = b % ngroups;
    const uint32_t gsz = G / ngroups + (x < G % ngroups ? 1u : 0u);
    const bool leader = b < ngroups;
    const int32_t K1 = a.K + 1;
    const bool thr_lds = h.thr_in_lds != 0;
    int32_t *abort_v = &abort_sh;
    // roles: the last wave is the barrier wave: as soon as a phase's nodes are done it
    // posts the workgroup's dM, collects its group's member words when this workgroup
    // leads the group, then reads the group words. All other waves ("workers") update
    // nodes, prefetch and poll their foreign words.
    const int nwork = (nwaves - 1) * 64;
    const bool worker = tid < nwork;
    const int32_t T0 = h.T0;
    const bool has_tail = T0 < a.C;
    const int32_t tail_base = has_tail ? a.cbeg[T0] : a.n_pad;  // a multiple of 64
    // this thread's tail node, its class and original id (-1: none)
    int32_t my_tail = -1, my_tc = -1, my_id = 0;
    if (has_tail && worker && tid < h.tail_n) {
        my_tail = h.tail_v[tid];
        my_id = a.orig[my_tail];
        for (int32_t k = 0; k < a.C - T0; ++k)
            if (tid >= h.tail_beg[k] && tid < h.tail_beg[k + 1]) my_tc = T0 + k;
    }

    for (int i = tid; i < a.C; i += nth) {
        tab[i] = h.tab[(size_t)b * a.C + i];
        Psh[i] = a.P[i];
        csz_sh[i] = a.csz[i];
    }
    if (thr_lds)
        for (int i = tid; i < K1; i += nth) thr_sh[(t_begin & 1u) * K1 + i] = a.thr[(size_t)t_begin * K1 + i];
    if (tid == 0) {
        wg_acc = 0;
        total_sh = 0;
        abort_sh = 0;
    }
    if (tid < 3) tacc[tid] = 0;
    if (tid == 0) {
        wdone = 0;
        dcut_sh = 0;
    }
    int32_t M = (int32_t)a.state[0];
    __syncthreads();

    // prologue: every own, foreign and gather word and the tail region straight from the
    // spin array, which no workgroup writes before its epilogue, so no workgroup waits for
    // another here (words published during the launch carry epochs >= epoch0 + 2, words
    // left by earlier launches smaller ones). The own and foreign words of classes
    // 0..T0-1 and the gather words form one index space (a word's id comes from the
    // chunk bounds, the foreign list in global memory, or the gather list), with up to
    // PRO_INFLIGHT words per thread in flight; the copies follow as one more space.
    {
        const int32_t *flist_b = h.flist + (size_t)b * h.flist_len;
        int32_t n_cls = 0;
        for (int32_t c = 0; c < T0; ++c) {
            const GdiHaloEntry e = tab[c];
            n_cls += (e.node_hi > e.node_lo ? ((e.node_hi + 31) >> 5) - (e.node_lo >> 5) : 0) + e.for_len;
        }
        const int32_t n_gat = has_tail ? h.gat_beg[T0] : 0, n_all = n_cls + n_gat;
        for (int32_t base = 0; base < n_all; base += PRO_INFLIGHT * nth) {
            int32_t wd[PRO_INFLIGHT], dst[PRO_INFLIGHT];
#pragma unroll
            for (int u = 0; u < PRO_INFLIGHT; ++u) {
                int32_t i = base + u * nth + tid;
                wd[u] = -1;
                dst[u] = 0;
                if (i < n_cls) {
                    int32_t c = 0;
                    for (;; ++c) {
                        const GdiHaloEntry e = tab[c];
                        const int32_t nown = e.node_hi > e.node_lo ? ((e.node_hi + 31) >> 5) - (e.node_lo >> 5) : 0;
                        if (i < nown) {
                            wd[u] = (e.node_lo >> 5) + i;
                            dst[u] = e.own_off + i;
                            break;
                        }
                        i -= nown;
                        if (i < e.for_len) {
                            wd[u] = flist_b[e.list_off - h.list_off + i];
                            dst[u] = e.for_off + i;
                            break;
                        }
                        i -= e.for_len;
                    }
                } else if (i < n_all) {
                    wd[u] = h.gat_words[i - n_cls];
                    dst[u] = h.gather_off + (i - n_cls);
                }
            }
            uint32_t word[PRO_INFLIGHT];
#pragma unroll
            for (int u = 0; u < PRO_INFLIGHT; ++u) word[u] = wd[u] >= 0 ? pack_spins(a.spin, wd[u]) : 0u;
#pragma unroll
            for (int u = 0; u < PRO_INFLIGHT; ++u)
                if (wd[u] >= 0) bits[dst[u]] = word[u];
        }
    }
    for (int32_t b0 = tail_base + wave * 64; b0 < a.n_pad; b0 += nwaves * 64) {
        const uint64_t m = __ballot(a.spin[b0 + lane] > 0);
        if (lane == 0) {
            bits[h.tail_off + ((b0 - tail_base) >> 5)] = (uint32_t)m;
            bits[h.tail_off + ((b0 - tail_base) >> 5) + 1] = (uint32_t)(m >> 32);
        }
    }
    // the foreign-word ids (polled from LDS in the sweep), the tail's CSR (row offsets,
    // then entries as LDS bit index and weight) and this workgroup's overflow entries
    int32_t *trp = reinterpret_cast<int32_t *>(bits + h.trp_off);
    uint32_t *tent = bits + h.tent_off;
    {
        const LdsCopy r0[3] = {
            {bits + h.list_off, reinterpret_cast<const uint32_t *>(h.flist + (size_t)b * h.flist_len), h.flist_len},
            {bits + h.ovf_off, h.ovf + (size_t)b * h.ovf_len, h.ovf_len},
            {reinterpret_cast<uint32_t *>(trp), reinterpret_cast<const uint32_t *>(h.tail_rp), has_tail ? h.tail_n + 1 : 0}};
        copy_ranges(r0, tid, nth);
        const LdsCopy r1[3] = {{tent, h.tail_ent, has_tail ? h.tail_nnz : 0}, {bits, nullptr, 0}, {bits, nullptr, 0}};
        copy_ranges(r1, tid, nth);
    }
    // pipeline fill: phase 0 entries, phase 1 rows
    NodePrefetch pf;
    RowAhead ra;
    {
        const uint32_t t1 = T0 > 1 ? t_begin : t_begin + 1u;
        const int32_t s1 = T0 > 1 ? 1 : 0;
        const int32_t v0 = step_node(h, tab, 0, tid);
        if (worker && v0 >= 0) {
            load_row(a, v0, ra);
            load_entries(h, ra, t_begin, pf);
        }
        const int32_t v1 = step_node(h, tab, s1, tid);
        if (worker && t1 < a.S && v1 >= 0) load_row(a, v1, ra);
    }
    __syncthreads();

    int64_t dcut = 0, dcut_total = 0;
    uint32_t p = 0, kk = 0;
    // local field of this thread's first-pass node of the coming phase, summed before
    // the phase's M is known (h_ready) or not
    int32_t h_pre = 0;
    bool h_ready = false;
    uint32_t wtarget = 0;
    // this thread's tail node in the current sweep: Philox words, drawn while the last
    // grid phase's dM travels
    uint32_t tx0 = 0, tx1 = 0;
    bool ttie = false;  // low bit of its word x2
    for (uint32_t t = t_begin; t < a.S; ++t) {
        const uint32_t *thr_l = thr_sh + (t & 1u) * K1;
        const uint32_t *thr_g = a.thr + (size_t)t * K1;
        for (int32_t c = 0; c < T0; ++c, ++p) {
            const GdiHaloEntry e = tab[c];
            const uint32_t epoch = h.epoch0 + p + 2u;
            int32_t dM = 0;
            GDI_TSTAMP(0, tid == 0);
            // this thread's first gather word of class c, loaded now so that the poll after
            // the phase does not wait for it
            const int32_t cg = c - 1;  // gather words are read one phase late
            int32_t gidx = -1;
            if (worker && has_tail && cg >= 0 && h.gat_beg[cg] + tid < h.gat_beg[cg + 1])
                gidx = h.gat_words[h.gat_beg[cg] + tid];
            if (worker) {
                const PhaseView pv = make_view(M, Psh[c], csz_sh[c], a.C, a.n);
                // wave-uniform trip count so that ballots see whole waves of 64 nodes;
                // the first pass uses the prefetched rows, later passes load their own
                // row bounds of this thread's node in the next pass, loaded at the end of
                // each pass (classes larger than the worker count take several passes)
                RowAhead rn;
                rn.r0 = rn.r1 = rn.id = 0;
                for (int32_t base = e.node_lo; base < e.node_hi; base += nwork) {
                    const int32_t v = base + tid;
                    const bool active = v < e.node_hi;
                    bool flip = false;
                    int32_t sigma_l = 0;
                    if (active && !masked_out(a, v, t)) {
                        NodePrefetch q;
                        if (base != e.node_lo) {
                            load_entries(h, rn, t, q);
                        } else {
                            q = pf;
                        }
                        const int32_t hv = base == e.node_lo && h_ready ? h_pre : row_field<UNIT>(h, bits, q);
                        const int32_t lb = (e.own_off + (v >> 5) - (e.node_lo >> 5)) * 32 + (v & 31);
                        const int32_t sigma = lds_spin(bits, lb);
                        flip = decide_words(a, sigma, hv, pv, thr_l, thr_g, thr_lds, q.x0, q.x1, q.r0t >> 31);
                        sigma_l = sigma;
                        if (flip) {
                            dcut += (int64_t)sigma * hv;
                            if (a.last_flip) a.last_flip[v] = (int32_t)t;
                        }
                    }
                    const uint64_t fm = __ballot(flip);
                    // flips of +1 spins lower M by 2, flips of -1 spins raise it by 2
                    const uint64_t fm_minus = __ballot(flip && sigma_l < 0);
                    dM += 2 * (__popcll(fm_minus) - __popcll(fm & ~fm_minus));
                    const int32_t v0 = base + (wave << 6);
                    if (lane == 0 && v0 < e.node_hi) {
                        // own chunk words covered by this wave: flip their bits, republish both
                        const int32_t wd = v0 >> 5;
                        const int32_t w_end = (e.node_hi + 31) >> 5;
                        uint32_t *lw = bits + e.own_off + wd - (e.node_lo >> 5);
                        lw[0] ^= (uint32_t)fm;
                        st_agent(h.words + wd, ((uint64_t)epoch << 32) | lw[0]);
                        if (wd + 1 < w_end) {
                            lw[1] ^= (uint32_t)(fm >> 32);
                            st_agent(h.words + wd + 1, ((uint64_t)epoch << 32) | lw[1]);
                        }
                    }
                    if (base + nwork < e.node_hi) load_row(a, min(v + nwork, e.node_hi - 1), rn);
                }
                if (lane == 0 && dM != 0) atomicAdd(&wg_acc, dM);
            }
            GDI_TSTAMP(1, tid == 0);
            __syncthreads();
            GDI_TSTAMP(2, tid == 0);
            uint64_t *gw = h.group + (size_t)((p & 1u) * 8u) * GDI_HALO_GROUP_PAD;
            bool good = true;
            if (worker) {
                // while the phase completes elsewhere: entries of the next phase (rows are
                // already here), rows of the phase after, next threshold row
                const bool last_s = c + 1 == T0;
                const uint32_t t1 = last_s ? t + 1u : t;
                const int32_t s1 = last_s ? 0 : c + 1;
                const bool last_s1 = s1 + 1 == T0;
                const uint32_t t2 = last_s1 ? t1 + 1u : t1;
                const int32_t s2 = last_s1 ? 0 : s1 + 1;
                // nodes the proposal skips need no entries
                const int32_t v1 = step_node(h, tab, s1, tid);
                const bool want1 = t1 < a.S && v1 >= 0 && !masked_out(a, v1, t1);
                if (t1 < a.S) {
                    if (c + 1 == T0 && thr_lds && t + 1u < a.S)
                        for (int i = tid; i < K1; i += nwork) thr_sh[((t + 1u) & 1u) * K1 + i] = a.thr[(size_t)(t + 1u) * K1 + i];
                    if (want1) load_entries(h, ra, t1, pf);
                }
                const int32_t v2 = step_node(h, tab, s2, tid);
                if (t2 < a.S && v2 >= 0) load_row(a, v2, ra);
                GDI_TSTAMP(6, tid == 0);
                good = poll_phase_words(h, e, cg, gidx, bits, epoch, epoch - 1u, tid, nwork, abort_v);
                GDI_TSTAMP(7, tid == 0);
                // Once every worker wave has polled, the image holds every spin the next
                // phase reads, so the next phase's local fields are summed now, while this
                // phase's dM is still travelling; only the decisions wait for the new M.
                // Each worker wave counts itself in whether or not its polls succeeded, so
                // this wait ends. Before the tail, the tail nodes' Philox words are drawn.
                h_ready = false;
                const bool pre_next = t1 < a.S && !(has_tail && last_s);
                if (has_tail && last_s && my_tail >= 0) {
                    const Words4 xw = philox10((uint32_t)my_id, t, a.replica, 0u, a.key0, a.key1);
                    tx0 = xw.w0;
                    tx1 = xw.w1;
                    ttie = (xw.w2 & 1u) != 0;
                }
                if (pre_next) {
                    if (lane == 0) __hip_atomic_fetch_add(&wdone, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
                    wtarget += (uint32_t)(nwork >> 6);
                    for (int64_t tries = 0;
                         (int32_t)(__hip_atomic_load(&wdone, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) - wtarget) < 0;
                         ++tries) {
                        if (tries >= a.spin_limit || aborted(abort_v)) {
                            good = false;
                            break;
                        }
                        __builtin_amdgcn_s_sleep(1);
                    }
                    if (good && want1) h_pre = row_field<UNIT>(h, bits, pf);
                    h_ready = true;
                }
            } else {
                // the barrier wave has no other memory traffic, so its store leaves at once
                const int32_t mine = wg_acc;
                if (lane == 0) {
                    st_agent(h.member + x * 64u + b / ngroups, ((uint64_t)epoch << 32) | (uint32_t)mine);
                    wg_acc = 0;
                }
                if (leader) {
                    // the leader's own member word is its group's first (b / ngroups == 0)
                    int32_t part = lane == 0 ? mine : 0;
                    if (lane > 0 && (uint32_t)lane < gsz)
                        good = poll_word(h.member + x * 64u + (uint32_t)lane, epoch, a.spin_limit, abort_v, &part);
                    if (!good) set_abort(abort_v);
                    part = wave_sum_i32(part);
                    if (lane == 0) st_agent(gw + (size_t)x * GDI_HALO_GROUP_PAD, ((uint64_t)epoch << 32) | (uint32_t)part);
                    GDI_TSTAMP(4, lane == 0);
                }
                int32_t part = 0;
                if (good && (uint32_t)lane < ngroups)
                    good = poll_word(gw + (size_t)lane * GDI_HALO_GROUP_PAD, epoch, a.spin_limit, abort_v, &part);
                part = wave_sum_i32(part);
                if (lane == 0) total_sh = part;
                GDI_TSTAMP(5, lane == 0);
            }
            if (!good) set_abort(abort_v);
            __syncthreads();
            GDI_TSTAMP(3, tid == 0);
            if (abort_sh) {
                if (tid == 0) __hip_atomic_store(&a.state[3], (int64_t)1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                return;
            }
            const int32_t tot = total_sh;
            M += tot;
            if (tid == 0 && a.C > 1) Psh[c] += tot / 2;
        }
        if (has_tail) {
            // the last grid class's gather words (its phase was p - 1): published before
            // that phase's barrier, so they are all there now
            if (worker && !poll_gather(h, T0 - 1, bits, h.epoch0 + p + 1u, tid, nwork, abort_v)) set_abort(abort_v);
            __syncthreads();
            if (abort_sh) {
                if (tid == 0) __hip_atomic_store(&a.state[3], (int64_t)1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                return;
            }
            // the tail, identically in every workgroup: one class after the other with
            // workgroup barriers only; dM through a rotating triple of LDS accumulators.
            // Its CSR is in LDS, so no global load is in flight across these barriers.
            for (int32_t tc = T0; tc < a.C; ++tc, ++kk) {
                int32_t dM = 0;
                if (worker && my_tc == tc && !masked_out(a, my_tail, t)) {
                    const PhaseView pv = make_view(M, Psh[tc], csz_sh[tc], a.C, a.n);
                    const int32_t v = my_tail;
                    const int32_t hv = lds_field(bits, tent, trp[tid], trp[tid + 1]);
                    const int32_t lb = (h.tail_off + ((v - tail_base) >> 5)) * 32 + (v & 31);
                    const int32_t sigma = lds_spin(bits, lb);
                    if (decide_words(a, sigma, hv, pv, thr_l, thr_g, thr_lds, tx0, tx1, ttie ? 1u : 0u)) {
                        // members of a class are never neighbours: concurrent readers of this
                        // word only look at bits that do not change in this class
                        atomicXor(&bits[lb >> 5], 1u << (lb & 31));
                        dM = -2 * sigma;
                        if (b == 0) {
                            dcut += (int64_t)sigma * hv;
                            if (a.last_flip) a.last_flip[v] = (int32_t)t;
                        }
                    }
                }
                dM = wave_sum_i32(dM);
                if (lane == 0 && dM != 0) atomicAdd(&tacc[kk % 3], dM);
                __syncthreads();
                const int32_t tot = tacc[kk % 3];
                M += tot;
                if (tid == 0) {
                    Psh[tc] += tot / 2;
                    tacc[(kk + 2) % 3] = 0;
                }
            }
        }
        if (a.trace_m) {
            if (b == 0 && tid == 0) a.trace_m[t] = M;
            const int64_t w = wave_sum_i64(dcut);
            if (lane == 0 && w != 0) atomicAdd((unsigned long long *)&a.trace_dcut[t], (unsigned long long)w);
            dcut_total += dcut;
            dcut = 0;
        }
    }
    dcut_total += dcut;
    __syncthreads();
    // epilogue: own spins back to the int8 array (the tail from workgroup 0)
    for (int32_t c = 0; c < T0; ++c) {
        const GdiHaloEntry e = tab[c];
        for (int32_t v = e.node_lo + tid; v < e.node_hi; v += nth) {
            const int32_t lb = (e.own_off + (v >> 5) - (e.node_lo >> 5)) * 32 + (v & 31);
            a.spin[v] = (int8_t)lds_spin(bits, lb);
        }
    }
    if (b == 0) {
        for (int32_t i = tid; i < h.tail_n; i += nth) {
            const int32_t v = h.tail_v[i];
            a.spin[v] = (int8_t)lds_spin(bits, (h.tail_off + ((v - tail_base) >> 5)) * 32 + (v & 31));
        }
        for (int i = tid; i < a.C; i += nth) a.P[i] = Psh[i];
        if (tid == 0) a.state[0] = M;
    }
    // one global atomic per workgroup: the device serialises atomics on one word
    const int64_t w = wave_sum_i64(dcut_total);
    if (lane == 0 && w != 0) atomicAdd((unsigned long long *)&dcut_sh, (unsigned long long)w);
    __syncthreads();
    if (tid == 0 && dcut_sh != 0) atomicAdd((unsigned long long *)&a.state[1], (unsigned long long)dcut_sh);
}

inline int status(hipError_t e) { return (int)e; }

}  // namespace

int gdi_halo_capacity(int block, int lds_bytes, int *max_grid)
{
    // the smaller capacity of the two instantiations (unit and general weights)
    const void *fs[2] = {(const void *)k_sweep_halo<false>, (const void *)k_sweep_halo<true>};
    int dev = 0, cus = 0, best = INT32_MAX;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    for (int i = 0; i < 2 && e == hipSuccess; ++i) {
        int per_cu = 0;
        e = hipFuncSetAttribute(fs[i], hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
        if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fs[i], block, lds_bytes);
        best = std::min(best, per_cu);
    }
    if (e != hipSuccess) return status(e);
    *max_grid = cus * best;
    return 0;
}

int gdi_launch_sweep_halo(const GdiHaloArgs &h, int grid, int block, void *stream)
{
    const void *f = h.unit_w ? (const void *)k_sweep_halo<true> : (const void *)k_sweep_halo<false>;
    const int lds = gdi_halo_lds_bytes(h.lds_words, h.base.C, h.thr_in_lds ? 2 * (h.base.K + 1) : 0);
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return status(e);
    GdiHaloArgs copy = h;
    void *args[] = {&copy};
    e = hipLaunchCooperativeKernel(f, dim3(grid), dim3(block), args, (unsigned)lds, (hipStream_t)stream);
    return status(e);
}

#ifdef GDI_PHASE_TIMING
extern "C" int gdi_timing_setup(unsigned long long *buf, int first, int phases)
{
    hipError_t e = hipMemcpyToSymbol(HIP_SYMBOL(g_tbuf), &buf, sizeof(buf));
    if (e == hipSuccess) e = hipMemcpyToSymbol(HIP_SYMBOL(g_tfirst), &first, sizeof(int));
    if (e == hipSuccess) e = hipMemcpyToSymbol(HIP_SYMBOL(g_tphases), &phases, sizeof(int));
    return (int)e;
}
#endif
