// gdi_kernels.hip -- gfx950 kernels of the GDI annealer (wave64, CDNA4).
//
// The hot path is one persistent launch per anneal: every sweep visits the
// colour classes in ascending colour; in each phase the nodes of one class
// read their CSR rows, gather neighbour spins, form the local field
// h_i = sum_j w_ij s_j, and make the Metropolis decision of Sec. V Alg. 3
// (balance term from the tracked magnetisation, eq. 5 / eq. 6 flip cost).
// The per-phase change of the magnetisation is reduced with wave reductions,
// an LDS accumulator and (grid scope) a two-level atomic barrier.
//
// Two scopes share the same per-node update:
//   k_sweep_wg   -- one workgroup owns the whole instance; phases are separated
//                   by s_barrier; spins live in LDS when they fit.
//   k_sweep_grid -- all co-resident workgroups (cooperative launch) split every
//                   class into 64-node-aligned chunks; phases are separated by a
//                   device-wide barrier that also sums the per-workgroup dM.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "gdi_internal.h"
#include "gdi_device.h"

namespace {


// One node of the current class: L lanes share its CSR row. All L lanes return
// the same decision; lane 0 of the subgroup performs the write.
// sp is an LDS or a global int8 pointer.
// Row bounds r0, r1 come from the caller (loaded ahead by the workgroup sweep); the
// original id is loaded before the row so that its latency overlaps the row's. U
// entries per lane and round: 8 for rows long against L, else 4 (skipped loads still
// cost their branch).
template <int L, int U = 4>
__device__ __forceinline__ bool node_decide(const GdiSweepArgs &a, const int8_t *sp, int32_t v, int32_t r0,
                                            int32_t r1, int lane, uint32_t t, const PhaseView &pv,
                                            const uint32_t *thr_row, const uint32_t *thr_l, int32_t *h_out,
                                            int32_t *sigma_out)
{
    const uint32_t o = (uint32_t)a.orig[v];
    int32_t h = 0;
    // up to U entries per lane and round, all loads of a round issued before any is
    // used; an entry past the row is not loaded and counts as (node 0, weight 0)
    for (int32_t k = r0 + lane; k < r1; k += U * L) {
        int2 e[U];
#pragma unroll
        for (int u = 0; u < U; ++u) e[u] = k + u * L < r1 ? a.adj[k + u * L] : make_int2(0, 0);
        int32_t sv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) sv[u] = sp[e[u].x];
#pragma unroll
        for (int u = 0; u < U; ++u) h += e[u].y * sv[u];
    }
    if (L > 1) h = group_sum<L>(h);
    const int32_t sigma = sp[v];
    *h_out = h;
    *sigma_out = sigma;
    return decide_id(a, o, t, sigma, h, pv, thr_row, thr_l);
}

// A subgroup's first node of a phase, fetched ahead of the phase: its row bounds and
// original id two phases before, the row's first GDI_AHEAD entries per lane one phase
// before. CSR rows do not depend on spins, so these loads run under the earlier
// phases' work and barriers, and the phase itself starts with LDS spin reads.
#define GDI_AHEAD 4
struct RowAhead {
    int32_t v;              // new id, -1 when the subgroup has no node in the phase
    int32_t r0, r1;
    uint32_t o;             // original id
    int2 e[GDI_AHEAD];      // entries r0 + lane + u * L (zero past the row)
};

// Bounds stage: node beg + j when j < hi.
__device__ __forceinline__ void ahead_bounds(const GdiSweepArgs &a, int32_t beg, int32_t j, int32_t hi, RowAhead &r)
{
    r.v = j < hi ? beg + j : -1;
    r.r0 = 0;
    r.r1 = 0;
    r.o = 0;
    if (r.v >= 0) {
        r.r0 = a.rp[r.v];
        r.r1 = a.rp[r.v + 1];
        r.o = (uint32_t)a.orig[r.v];
    }
}

// Entries stage (after the bounds have arrived).
template <int L>
__device__ __forceinline__ void ahead_entries(const GdiSweepArgs &a, int lane, RowAhead &r)
{
#pragma unroll
    for (int u = 0; u < GDI_AHEAD; ++u) {
        const int32_t k = r.r0 + lane + u * L;
        r.e[u] = k < r.r1 ? a.adj[k] : make_int2(0, 0);
    }
}

// node_decide for a node fetched ahead: the first GDI_AHEAD entries per lane come from
// registers, the rest of the row (if any) is read in rounds of U as usual.
template <int L, int U = 4>
__device__ __forceinline__ bool node_decide_ahead(const GdiSweepArgs &a, const int8_t *sp, const RowAhead &r, int lane,
                                                  uint32_t t, const PhaseView &pv, const uint32_t *thr_row,
                                                  const uint32_t *thr_l, int32_t *h_out, int32_t *sigma_out)
{
    int32_t h = 0;
    {
        int32_t sv[GDI_AHEAD];
#pragma unroll
        for (int u = 0; u < GDI_AHEAD; ++u) sv[u] = sp[r.e[u].x];
#pragma unroll
        for (int u = 0; u < GDI_AHEAD; ++u) h += r.e[u].y * sv[u];
    }
    for (int32_t k = r.r0 + lane + GDI_AHEAD * L; k < r.r1; k += U * L) {
        int2 e[U];
#pragma unroll
        for (int u = 0; u < U; ++u) e[u] = k + u * L < r.r1 ? a.adj[k + u * L] : make_int2(0, 0);
        int32_t sv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) sv[u] = sp[e[u].x];
#pragma unroll
        for (int u = 0; u < U; ++u) h += e[u].y * sv[u];
    }
    if (L > 1) h = group_sum<L>(h);
    const int32_t sigma = sp[r.v];
    *h_out = h;
    *sigma_out = sigma;
    return decide_id(a, r.o, t, sigma, h, pv, thr_row, thr_l);
}

// ------------------------------------------------------------------ workgroup scope
// All sweeps of one instance inside one workgroup: phases are separated by
// s_barrier, dM is summed in an LDS triple buffer (one barrier per phase).
// sp points to the instance's spins (LDS, or global for large instances),
// Psh to its per-class +1 counts in LDS, acc to three zeroed LDS words, thr_s to
// 2 x GDI_WG_THR_MAX LDS words for the current and the next threshold row.
template <int L, int U = 4>
__device__ __forceinline__ void wg_run_sweeps(const GdiSweepArgs &a, int8_t *sp, int32_t *Psh, int32_t *acc, uint32_t *thr_s,
                              int32_t &M, int64_t &dcut_total)
{
    const int tid = threadIdx.x;
    const int nth = blockDim.x;
    const int sub = tid / L, lane = tid % L, nsub = nth / L;
    int64_t dcut = 0;
    uint32_t p = 0;
    // the current and the next threshold row in LDS when they fit (staged during the
    // last phase of each sweep, whose barrier publishes them)
    const int32_t K1 = a.K + 1;
    const bool thr_lds = K1 <= GDI_WG_THR_MAX;
    if (thr_lds && a.t0 < a.S)
        for (int i = tid; i < K1; i += nth) thr_s[(a.t0 & 1u) * GDI_WG_THR_MAX + i] = a.thr[(size_t)a.t0 * K1 + i];
    __syncthreads();
    // the subgroup's first node of this phase (bounds and entries fetched) and of the
    // next phase (bounds fetched); phases run (t, 0..C-1) for t = t0..S-1
    RowAhead cur, b1;
    cur.v = b1.v = -1;
    cur.r0 = cur.r1 = b1.r0 = b1.r1 = 0;
    cur.o = b1.o = 0;
    if (a.t0 < a.S) {
        ahead_bounds(a, a.cbeg[0], sub, a.csz[0], cur);
        ahead_entries<L>(a, lane, cur);
        const bool wrap = a.C == 1;
        if (!wrap || a.t0 + 1u < a.S) ahead_bounds(a, a.cbeg[wrap ? 0 : 1], sub, a.csz[wrap ? 0 : 1], b1);
    }
    for (uint32_t t = a.t0; t < a.S; ++t) {
        const uint32_t *thr_row = a.thr + (size_t)t * (uint32_t)K1;
        const uint32_t *thr_l = thr_lds ? thr_s + (t & 1u) * GDI_WG_THR_MAX : nullptr;
        for (int32_t c = 0; c < a.C; ++c, ++p) {
            const int32_t beg = a.cbeg[c];
            const int32_t size = a.csz[c];
            const PhaseView pv = make_view(M, Psh[c], size, a.C, a.n);
            int32_t dM = 0;
            // each subgroup loads the next node's row bounds while it works on this one
            int32_t nr0 = 0, nr1 = 0;
            if (sub + nsub < size) {
                nr0 = a.rp[beg + sub + nsub];
                nr1 = a.rp[beg + sub + nsub + 1];
            }
            if (cur.v >= 0 && !(a.mask && ((a.mask[cur.v >> 5] >> (cur.v & 31)) & 1u))) {
                int32_t h, sigma;
                const bool flip = node_decide_ahead<L, U>(a, sp, cur, lane, t, pv, thr_row, thr_l, &h, &sigma);
                if (flip && lane == 0) {
                    sp[cur.v] = (int8_t)(-sigma);
                    dM -= 2 * sigma;
                    dcut += (int64_t)sigma * h;
                    if (a.last_flip) a.last_flip[cur.v] = (int32_t)t;
                }
            }
            for (int32_t j = sub + nsub; j < size; j += nsub) {
                const int32_t v = beg + j;
                const int32_t r0 = nr0, r1 = nr1;
                if (j + nsub < size) {
                    nr0 = a.rp[v + nsub];
                    nr1 = a.rp[v + nsub + 1];
                }
                if (a.mask && ((a.mask[v >> 5] >> (v & 31)) & 1u)) continue;  // skipped node
                int32_t h, sigma;
                const bool flip = node_decide<L, U>(a, sp, v, r0, r1, lane, t, pv, thr_row, thr_l, &h, &sigma);
                if (flip && lane == 0) {
                    sp[v] = (int8_t)(-sigma);
                    dM -= 2 * sigma;
                    dcut += (int64_t)sigma * h;
                    if (a.last_flip) a.last_flip[v] = (int32_t)t;
                }
            }
            if (c + 1 == a.C && thr_lds && t + 1u < a.S)
                for (int i = tid; i < K1; i += nth)
                    thr_s[((t + 1u) & 1u) * GDI_WG_THR_MAX + i] = a.thr[(size_t)(t + 1u) * K1 + i];
            // after this phase's loads: the next phase's entries and the bounds of the phase
            // after it (issued last, so that no wait of this phase's work covers them)
            ahead_entries<L>(a, lane, b1);
            cur = b1;
            {
                int32_t c2 = c + 2;
                uint32_t t2 = t;
                while (c2 >= a.C) {
                    c2 -= a.C;
                    ++t2;
                }
                b1.v = -1;
                b1.r0 = b1.r1 = 0;
                b1.o = 0;
                if (t2 < a.S) ahead_bounds(a, a.cbeg[c2], sub, a.csz[c2], b1);
            }
            dM = wave_sum_i32(dM);
            if ((tid & 63) == 0 && dM != 0) atomicAdd(&acc[p % 3], dM);
            __syncthreads();
            const int32_t tot = acc[p % 3];
            M += tot;
            if (tid == 0) {
                if (a.C > 1) Psh[c] += tot / 2;
                acc[(p + 2) % 3] = 0;
            }
        }
        if (a.trace_m) {
            if (tid == 0) a.trace_m[t] = M;
            const int64_t w = wave_sum_i64(dcut);
            if ((tid & 63) == 0 && w != 0) atomicAdd((unsigned long long *)&a.trace_dcut[t], (unsigned long long)w);
            dcut_total += dcut;
            dcut = 0;
        }
    }
    dcut_total += dcut;
}

template <int L, bool SPIN_LDS>
__global__ void __launch_bounds__(GDI_MAX_BLOCK) k_sweep_wg(GdiSweepArgs a)
{
    if (!gate_open(a)) return;
    extern __shared__ int32_t dyn[];
    __shared__ int32_t acc[3];
    __shared__ uint32_t thr_s[2 * GDI_WG_THR_MAX];
    int32_t *Psh = dyn;
    const int c_round = (a.C + 3) & ~3;
    int8_t *sp = SPIN_LDS ? reinterpret_cast<int8_t *>(dyn + c_round) : a.spin;

    const int tid = threadIdx.x;
    const int nth = blockDim.x;
    for (int i = tid; i < a.C; i += nth) Psh[i] = a.P[i];
    if (SPIN_LDS)
        for (int i = tid; i < a.n_pad; i += nth) sp[i] = a.spin[i];
    if (tid < 3) acc[tid] = 0;
    int32_t M = (int32_t)a.state[0];
    __syncthreads();

    int64_t dcut_total = 0;
    wg_run_sweeps<L>(a, sp, Psh, acc, thr_s, M, dcut_total);

    __syncthreads();
    if (SPIN_LDS)
        for (int i = tid; i < a.n_pad; i += nth) a.spin[i] = sp[i];
    for (int i = tid; i < a.C; i += nth) a.P[i] = Psh[i];
    if (tid == 0) a.state[0] = M;
    const int64_t w = wave_sum_i64(dcut_total);
    if ((tid & 63) == 0 && w != 0) atomicAdd((unsigned long long *)&a.state[1], (unsigned long long)w);
}

// ------------------------------------------------------------------ workgroup scope, graph in LDS
// Small graphs with +-1 weights (n_pad <= 32768, nnz <= 65535): the whole instance
// lives in LDS for the launch -- spins (int8), original ids, row offsets and entries
// as 16-bit words (column | sign of the weight << 15) -- so a phase reads no global
// memory at all. Phases are separated by s_barrier as in k_sweep_wg.
__host__ __device__ __forceinline__ int32_t wgl_c_round(int32_t C) { return (C + 3) & ~3; }

template <int L>
__global__ void __launch_bounds__(GDI_MAX_BLOCK) k_sweep_wgl(GdiSweepArgs a, const uint16_t *rp16, const uint16_t *ent16,
                                                             int32_t nnz)
{
    if (!gate_open(a)) return;
    extern __shared__ int32_t dyn[];
    __shared__ int32_t acc[3];
    __shared__ uint32_t thr_s[2 * GDI_WG_THR_MAX];
    const int32_t c_round = wgl_c_round(a.C);
    int32_t *Psh = dyn;
    int32_t *orig_s = dyn + c_round;
    uint16_t *rp_s = reinterpret_cast<uint16_t *>(orig_s + a.n_pad);
    uint16_t *ent_s = rp_s + ((a.n_pad + 2) & ~1);
    int8_t *sp = reinterpret_cast<int8_t *>(ent_s + ((nnz + 1) & ~1));

    const int tid = threadIdx.x, nth = blockDim.x;
    const int sub = tid / L, lane = tid % L, nsub = nth / L;
    for (int i = tid; i < a.C; i += nth) Psh[i] = a.P[i];
    for (int i = tid; i < a.n_pad; i += nth) {
        orig_s[i] = a.orig[i];
        sp[i] = a.spin[i];
    }
    for (int i = tid; i <= a.n_pad; i += nth) rp_s[i] = rp16[i];
    for (int i = tid; i < nnz; i += nth) ent_s[i] = ent16[i];
    if (tid < 3) acc[tid] = 0;
    int32_t M = (int32_t)a.state[0];
    const int32_t K1 = a.K + 1;
    const bool thr_lds = K1 <= GDI_WG_THR_MAX;
    if (thr_lds && a.t0 < a.S)
        for (int i = tid; i < K1; i += nth) thr_s[(a.t0 & 1u) * GDI_WG_THR_MAX + i] = a.thr[(size_t)a.t0 * K1 + i];
    __syncthreads();

    int64_t dcut = 0, dcut_total = 0;
    uint32_t p = 0;
    for (uint32_t t = a.t0; t < a.S; ++t) {
        const uint32_t *thr_row = a.thr + (size_t)t * (uint32_t)K1;
        const uint32_t *thr_l = thr_lds ? thr_s + (t & 1u) * GDI_WG_THR_MAX : nullptr;
        for (int32_t c = 0; c < a.C; ++c, ++p) {
            const int32_t beg = a.cbeg[c];
            const int32_t size = a.csz[c];
            const PhaseView pv = make_view(M, Psh[c], size, a.C, a.n);
            int32_t dM = 0;
            for (int32_t j = sub; j < size; j += nsub) {
                const int32_t v = beg + j;
                if (a.mask && ((a.mask[v >> 5] >> (v & 31)) & 1u)) continue;  // skipped node
                const int32_t r0 = rp_s[v], r1 = rp_s[v + 1];
                const uint32_t o = (uint32_t)orig_s[v];
                int32_t h = 0;
                // four entries per lane and round, every LDS read of a round before any use
                for (int32_t k = r0 + lane; k < r1; k += 4 * L) {
                    uint32_t e[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) e[u] = k + u * L < r1 ? ent_s[k + u * L] : 0u;
                    int32_t sv[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) sv[u] = k + u * L < r1 ? sp[e[u] & 0x7FFFu] : 0;
#pragma unroll
                    for (int u = 0; u < 4; ++u) h += (e[u] & 0x8000u) ? -sv[u] : sv[u];
                }
                if (L > 1) h = group_sum<L>(h);
                const int32_t sigma = sp[v];
                const bool flip = decide_id(a, o, t, sigma, h, pv, thr_row, thr_l);
                if (flip && lane == 0) {
                    sp[v] = (int8_t)(-sigma);
                    dM -= 2 * sigma;
                    dcut += (int64_t)sigma * h;
                    if (a.last_flip) a.last_flip[v] = (int32_t)t;
                }
            }
            if (c + 1 == a.C && thr_lds && t + 1u < a.S)
                for (int i = tid; i < K1; i += nth)
                    thr_s[((t + 1u) & 1u) * GDI_WG_THR_MAX + i] = a.thr[(size_t)(t + 1u) * K1 + i];
            dM = wave_sum_i32(dM);
            if ((tid & 63) == 0 && dM != 0) atomicAdd(&acc[p % 3], dM);
            __syncthreads();
            const int32_t tot = acc[p % 3];
            M += tot;
            if (tid == 0) {
                if (a.C > 1) Psh[c] += tot / 2;
                acc[(p + 2) % 3] = 0;
            }
        }
        if (a.trace_m) {
            if (tid == 0) a.trace_m[t] = M;
            const int64_t w = wave_sum_i64(dcut);
            if ((tid & 63) == 0 && w != 0) atomicAdd((unsigned long long *)&a.trace_dcut[t], (unsigned long long)w);
            dcut_total += dcut;
            dcut = 0;
        }
    }
    dcut_total += dcut;
    __syncthreads();
    for (int i = tid; i < a.n_pad; i += nth) a.spin[i] = sp[i];
    for (int i = tid; i < a.C; i += nth) a.P[i] = Psh[i];
    if (tid == 0) a.state[0] = M;
    const int64_t w = wave_sum_i64(dcut_total);
    if ((tid & 63) == 0 && w != 0) atomicAdd((unsigned long long *)&a.state[1], (unsigned long long)w);
}

// Class of new id v: the last c with cbeg[c] <= v.
__device__ __forceinline__ int32_t class_of(const int32_t *cbeg, int32_t C, int32_t v)
{
    int32_t lo = 0, hi = C - 1;  // last c with cbeg[c] <= v
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (cbeg[mid] <= v) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// ------------------------------------------------------------------ active-set sweeps
// Bit i set iff byte i of q (sixteen int8 spins, +1 or -1) is positive: per 32-bit part,
// the bytes' inverted sign bits gathered into a nibble by one multiply (the partial
// products of the four bits meet in the top byte without carries).
__device__ __forceinline__ uint32_t plus_bits16(uint4 q)
{
    const uint32_t x[4] = {q.x, q.y, q.z, q.w};
    uint32_t r = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const uint32_t y = (~x[i] >> 7) & 0x01010101u;
        r |= ((y * 0x01020408u) >> 24) << (4 * i);
    }
    return r;
}

// Active ids of the 64-id chunk ch (first id v0) of a class ending at cend: real ids
// whose mask bit is clear.
__device__ __forceinline__ uint64_t active_chunk(const GdiSweepArgs &a, int32_t ch, int32_t v0, int32_t cend)
{
    const int32_t nv = min(64, max(0, cend - v0));
    const uint64_t valid = nv == 64 ? ~0ull : ((1ull << nv) - 1ull);
    const uint64_t m = a.mask ? reinterpret_cast<const uint64_t *>(a.mask)[ch] : 0ull;
    return valid & ~m;
}

// Masked sweeps of the learned proposal in one workgroup when few nodes are active:
// every spin of the graph is one bit in LDS (so neighbour reads never leave the CU),
// the active nodes (mask bit clear, real ids) are compacted at the start into
// records {new id, row, original id} in class order, and a class with no active node
// takes no phase at all -- nothing in it can change, so M and the class counts stay.
// The decisions are those of the full-graph kernels with the mask applied.
// Set-up in two passes over the graph: the spins become bits with 16-byte loads (32 ids
// per word, four words per thread in flight), and the compaction gives each thread a run
// of consecutive 64-id chunks (records in id order, which is class order), counts its
// active ids, takes its first record's position from one workgroup scan and writes its
// records; class starts are multiples of 64, so a chunk lies in one class. When thr_bytes
// (at LDS byte offset thr_off) hold the launch's threshold rows, they are copied there
// and every decision reads its threshold from LDS.
__global__ void __launch_bounds__(GDI_MAX_BLOCK) k_sweep_active(GdiSweepArgs a, GdiActiveRec *rec, int32_t thr_off,
                                                                int32_t thr_bytes)
{
    if (!gate_open(a)) return;
    extern __shared__ uint32_t lds[];
    const int32_t nw = a.n_pad >> 5;
    uint32_t *bits = lds;                                           // n_pad spin bits (1 = +1)
    int32_t *abeg = reinterpret_cast<int32_t *>(lds + nw);          // C + 1 record offsets
    int32_t *Psh = abeg + a.C + 1;                                  // C counts of +1
    int32_t *cb_s = Psh + a.C;                                      // C class starts, then n_pad
    int32_t *cs_s = cb_s + a.C + 1;                                 // C class sizes
    __shared__ int32_t acc[3];
    __shared__ int32_t wtot[GDI_MAX_BLOCK / 64];
    const int tid = threadIdx.x, nth = blockDim.x;
    const int lane = tid & 63, wave = tid >> 6, nwaves = nth >> 6;

    // spins -> bits (n_pad is a multiple of 64; the spin array is 16-byte aligned)
    const uint4 *sp4 = reinterpret_cast<const uint4 *>(a.spin);
    for (int32_t w0 = tid; w0 < nw; w0 += 4 * nth) {
        uint4 q[4][2] = {};
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int32_t wd = w0 + u * nth;
            if (wd < nw) {
                q[u][0] = sp4[2 * wd];
                q[u][1] = sp4[2 * wd + 1];
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int32_t wd = w0 + u * nth;
            if (wd < nw) bits[wd] = plus_bits16(q[u][0]) | (plus_bits16(q[u][1]) << 16);
        }
    }
    for (int i = tid; i < a.C; i += nth) {
        Psh[i] = a.P[i];
        cb_s[i] = a.cbeg[i];
        cs_s[i] = a.csz[i];
    }
    if (tid == 0) cb_s[a.C] = a.n_pad;
    // the threshold rows of sweeps t0 .. S - 1
    const int32_t K1 = a.K + 1;
    const int64_t thr_n = a.S > a.t0 ? (int64_t)(a.S - a.t0) * K1 : 0;
    const bool thr_staged = thr_n * 4 <= (int64_t)thr_bytes;
    uint32_t *thr_s = reinterpret_cast<uint32_t *>(reinterpret_cast<unsigned char *>(lds) + thr_off);
    if (thr_staged)
        for (int64_t i = tid; i < thr_n; i += nth) thr_s[i] = a.thr[(size_t)a.t0 * K1 + i];
    if (tid < 3) acc[tid] = 0;
    int32_t M = (int32_t)a.state[0];
    __syncthreads();

    // compaction: thread tid takes the chunks [ch0, ch1)
    const int32_t nch = a.n_pad >> 6;
    const int32_t per = (nch + nth - 1) / nth;
    const int32_t ch0 = min(nch, tid * per), ch1 = min(nch, ch0 + per);
    int32_t c0 = 0;  // class of chunk ch0: the last c with cb_s[c] <= its first id
    {
        int32_t lo = 0, hi = a.C - 1;
        const int32_t v0 = ch0 << 6;
        while (lo < hi) {
            const int32_t mid = (lo + hi + 1) >> 1;
            if (cb_s[mid] <= v0) lo = mid; else hi = mid - 1;
        }
        c0 = lo;
    }
    int32_t cnt = 0;
    for (int32_t ch = ch0, c = c0; ch < ch1; ++ch) {
        const int32_t v0 = ch << 6;
        while (cb_s[c + 1] <= v0) ++c;  // cb_s[C] = n_pad ends it
        cnt += __popcll(active_chunk(a, ch, v0, cb_s[c] + cs_s[c]));
    }
    int32_t incl = cnt;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int32_t y = __shfl_up(incl, off, 64);
        if (lane >= off) incl += y;
    }
    if (lane == 63) wtot[wave] = incl;
    __syncthreads();
    int32_t before = 0, total = 0;
    for (int w = 0; w < nwaves; ++w) {
        before += w < wave ? wtot[w] : 0;
        total += wtot[w];
    }
    int32_t pos = before + incl - cnt;
    for (int32_t ch = ch0, c = c0; ch < ch1; ++ch) {
        const int32_t v0 = ch << 6;
        while (cb_s[c + 1] <= v0) ++c;
        if (v0 == cb_s[c]) abeg[c] = pos;
        for (uint64_t x = active_chunk(a, ch, v0, cb_s[c] + cs_s[c]); x; x &= x - 1) {
            const int32_t v = v0 + __ffsll((unsigned long long)x) - 1;
            rec[pos++] = GdiActiveRec{v, a.rp[v], a.rp[v + 1], a.orig[v]};
        }
    }
    if (tid == 0) abeg[a.C] = total;
    __syncthreads();

    int64_t dcut = 0;
    uint32_t p = 0;
    for (uint32_t t = a.t0; t < a.S; ++t) {
        const uint32_t *thr_row = a.thr + (size_t)t * (uint32_t)(a.K + 1);
        const uint32_t *thr_l = thr_staged ? thr_s + (size_t)(t - a.t0) * K1 : nullptr;
        for (int32_t c = 0; c < a.C; ++c) {
            const int32_t jb = abeg[c], je = abeg[c + 1];
            if (jb == je) continue;
            const PhaseView pv = make_view(M, Psh[c], cs_s[c], a.C, a.n);
            int32_t dM = 0;
            // each thread loads its next record while it works on this one, and a row's
            // entries eight at a time, all loads of a round issued before any is used
            // (indices past the row are clamped to its last entry and count for nothing)
            GdiActiveRec rn{};
            if (jb + tid < je) rn = rec[jb + tid];
            for (int32_t j = jb + tid; j < je; j += nth) {
                const GdiActiveRec r = rn;
                if (j + nth < je) rn = rec[j + nth];
                int32_t h = 0;
                for (int32_t k0 = r.r0; k0 < r.r1; k0 += 8) {
                    int2 e[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) e[u] = a.adj[k0 + u < r.r1 ? k0 + u : r.r1 - 1];
#pragma unroll
                    for (int u = 0; u < 8; ++u)
                        if (k0 + u < r.r1) h += ((bits[e[u].x >> 5] >> (e[u].x & 31)) & 1u) ? e[u].y : -e[u].y;
                }
                const int32_t sigma = ((bits[r.v >> 5] >> (r.v & 31)) & 1u) ? 1 : -1;
                if (decide_id(a, (uint32_t)r.orig, t, sigma, h, pv, thr_row, thr_l)) {
                    // members of a class are never neighbours: other readers of this word
                    // only look at bits that do not change in this phase
                    atomicXor(&bits[r.v >> 5], 1u << (r.v & 31));
                    dM -= 2 * sigma;
                    dcut += (int64_t)sigma * h;
                    if (a.last_flip) a.last_flip[r.v] = (int32_t)t;
                }
            }
            dM = wave_sum_i32(dM);
            if (lane == 0 && dM != 0) atomicAdd(&acc[p % 3], dM);
            __syncthreads();
            const int32_t tot = acc[p % 3];
            M += tot;
            if (tid == 0) {
                if (a.C > 1) Psh[c] += tot / 2;
                acc[(p + 2) % 3] = 0;
            }
            ++p;
        }
    }
    __syncthreads();
    // only active nodes can have changed
    for (int32_t j = tid; j < abeg[a.C]; j += nth) {
        const int32_t v = rec[j].v;
        a.spin[v] = ((bits[v >> 5] >> (v & 31)) & 1u) ? (int8_t)1 : (int8_t)-1;
    }
    for (int i = tid; i < a.C; i += nth) a.P[i] = Psh[i];
    if (tid == 0) a.state[0] = M;
    const int64_t w = wave_sum_i64(dcut);
    if (lane == 0 && w != 0) atomicAdd((unsigned long long *)&a.state[1], (unsigned long long)w);
}

// ------------------------------------------------------------------ batched form, clusters
// A large instance of the batched form runs on a cluster of k workgroups ("members").
// Every member keeps the instance's whole spin vector in LDS and decides the nodes of
// its chunk of each class: chunk r of a class of `size` nodes is [bound(r), bound(r+1))
// in class order, with bound(r) = 64 round(r size / 64k), so a packed spin word has one
// owner. After its decisions a member publishes its chunk's spins as epoch-tagged words
// and its dM in a slot of the phase's parity, sums all k slots, and copies the other
// members' words of the class into its LDS: one memory round trip per phase. A word of
// class c is rewritten only in the next sweep's phase of c, and a slot two phases later,
// each after a total that needs every member's progress past its reads (C >= 2), so a
// reader never sees a value newer than the one it waits for. All waits are bounded.
__device__ __forceinline__ int32_t member_bound(int32_t size, int32_t r, int32_t k)
{
    if (r >= k) return size;
    const int64_t units = ((int64_t)size + 63) / 64;
    const int64_t b = ((int64_t)r * units * 2 + k) / (2 * (int64_t)k) * 64;
    return (int32_t)(b < size ? b : size);
}

template <int L, int U = 4>
__device__ __forceinline__ void cluster_run_sweeps(const GdiSweepArgs &a, const GdiBatchInstance &in, int8_t *sp, int32_t *Psh,
                                   int32_t *acc, uint32_t *thr_s, int32_t *tot_sh, int32_t *flag, int32_t &M,
                                   int64_t &dcut_total, int64_t limit)
{
    const int tid = threadIdx.x;
    const int nth = blockDim.x;
    const int sub = tid / L, lane = tid % L, nsub = nth / L;
    const int32_t k = in.members, r = in.rank;
    uint64_t *words = in.sync;
    uint64_t *slots = in.sync + (in.n_pad / 32 + 1);
    const int32_t K1 = a.K + 1;
    const bool thr_lds = K1 <= GDI_WG_THR_MAX;
    if (thr_lds && a.t0 < a.S)
        for (int i = tid; i < K1; i += nth) thr_s[(a.t0 & 1u) * GDI_WG_THR_MAX + i] = a.thr[(size_t)a.t0 * K1 + i];
    __syncthreads();
    int64_t dcut = 0;
    uint32_t p = 0;
    // this member's first node of a class for the subgroup, fetched ahead as in the
    // workgroup loop
    auto first_bounds = [&](int32_t cc, RowAhead &ra) {
        const int32_t sz = a.csz[cc];
        ahead_bounds(a, a.cbeg[cc], member_bound(sz, r, k) + sub, member_bound(sz, r + 1, k), ra);
    };
    RowAhead cur, b1;
    cur.v = b1.v = -1;
    cur.r0 = cur.r1 = b1.r0 = b1.r1 = 0;
    cur.o = b1.o = 0;
    if (a.t0 < a.S) {
        first_bounds(0, cur);
        ahead_entries<L>(a, lane, cur);
        if (a.C > 1 || a.t0 + 1u < a.S) first_bounds(a.C > 1 ? 1 : 0, b1);
    }
    for (uint32_t t = a.t0; t < a.S; ++t) {
        const uint32_t *thr_row = a.thr + (size_t)t * (uint32_t)K1;
        const uint32_t *thr_l = thr_lds ? thr_s + (t & 1u) * GDI_WG_THR_MAX : nullptr;
        for (int32_t c = 0; c < a.C; ++c, ++p) {
            const int32_t beg = a.cbeg[c];
            const int32_t size = a.csz[c];
            const int32_t lo = member_bound(size, r, k), hi = member_bound(size, r + 1, k);
            const PhaseView pv = make_view(M, Psh[c], size, a.C, a.n);
            int32_t dM = 0;
            int32_t nr0 = 0, nr1 = 0;
            if (lo + sub + nsub < hi) {
                nr0 = a.rp[beg + lo + sub + nsub];
                nr1 = a.rp[beg + lo + sub + nsub + 1];
            }
            if (cur.v >= 0) {
                int32_t h, sigma;
                const bool flip = node_decide_ahead<L, U>(a, sp, cur, lane, t, pv, thr_row, thr_l, &h, &sigma);
                if (flip && lane == 0) {
                    sp[cur.v] = (int8_t)(-sigma);
                    dM -= 2 * sigma;
                    dcut += (int64_t)sigma * h;
                }
            }
            for (int32_t j = lo + sub + nsub; j < hi; j += nsub) {
                const int32_t v = beg + j;
                const int32_t r0 = nr0, r1 = nr1;
                if (j + nsub < hi) {
                    nr0 = a.rp[v + nsub];
                    nr1 = a.rp[v + nsub + 1];
                }
                int32_t h, sigma;
                const bool flip = node_decide<L, U>(a, sp, v, r0, r1, lane, t, pv, thr_row, thr_l, &h, &sigma);
                if (flip && lane == 0) {
                    sp[v] = (int8_t)(-sigma);
                    dM -= 2 * sigma;
                    dcut += (int64_t)sigma * h;
                }
            }
            // the next sweep's threshold row, published by this phase's barriers
            if (c + 1 == a.C && thr_lds && t + 1u < a.S)
                for (int i = tid; i < K1; i += nth)
                    thr_s[((t + 1u) & 1u) * GDI_WG_THR_MAX + i] = a.thr[(size_t)(t + 1u) * K1 + i];
            // the next phase's entries, the bounds of the phase after it (issued after this
            // phase's loads; the exchange below hides them)
            ahead_entries<L>(a, lane, b1);
            cur = b1;
            {
                int32_t c2 = c + 2;
                uint32_t t2 = t;
                while (c2 >= a.C) {
                    c2 -= a.C;
                    ++t2;
                }
                b1.v = -1;
                b1.r0 = b1.r1 = 0;
                b1.o = 0;
                if (t2 < a.S) first_bounds(c2, b1);
            }
            dM = wave_sum_i32(dM);
            if ((tid & 63) == 0 && dM != 0) atomicAdd(&acc[p % 3], dM);
            __syncthreads();
            const uint32_t epoch = p + 1u;
            // this member's spins of class c (a byte is +1 when its low bit is set and its
            // sign bit clear; padding bytes are 0) and its dM
            const int32_t w0 = (beg + lo) >> 5, w1 = lo < hi ? (beg + hi + 31) >> 5 : w0;
            for (int32_t wd = w0 + tid; wd < w1; wd += nth) {
                const uint32_t *q = reinterpret_cast<const uint32_t *>(sp + (size_t)wd * 32);
                uint32_t bits = 0;
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const uint32_t x = q[i];
                    const uint32_t y = x & ~(x >> 7) & 0x01010101u;
                    bits |= ((y | (y >> 7) | (y >> 14) | (y >> 21)) & 0xFu) << (4 * i);
                }
                st_agent(words + wd, ((uint64_t)epoch << 32) | bits);
            }
            if (tid == 0) st_agent(slots + (p & 1u) * 16u + (uint32_t)r, ((uint64_t)epoch << 32) | (uint32_t)acc[p % 3]);
            if (tid < 64) {
                int32_t part = 0;
                bool ok = true;
                if (tid < k) ok = poll_word(slots + (p & 1u) * 16u + (uint32_t)tid, epoch, limit, flag, &part);
                if (!ok) set_abort(flag);
                part = wave_sum_i32(part);
                if (tid == 0) *tot_sh = part;
            }
            // the other members' spins of class c
            const int32_t cw0 = beg >> 5, cw1 = size > 0 ? (beg + size + 31) >> 5 : cw0;
            for (int32_t wd = cw0 + tid; wd < cw1; wd += nth) {
                if (wd >= w0 && wd < w1) continue;
                int32_t bits = 0;
                if (!poll_word(words + wd, epoch, limit, flag, &bits)) {
                    set_abort(flag);
                    break;
                }
                const int32_t id0 = wd * 32;
                for (int i = 0; i < 32; ++i) {
                    const int32_t id = id0 + i;
                    if (id >= beg + size) break;
                    if (id >= beg) sp[id] = (((uint32_t)bits >> i) & 1u) ? 1 : -1;
                }
            }
            __syncthreads();
            if (aborted(flag)) return;
            const int32_t tot = *tot_sh;
            M += tot;
            if (tid == 0) {
                if (a.C > 1) Psh[c] += tot / 2;
                acc[(p + 2) % 3] = 0;
            }
        }
    }
    dcut_total += dcut;
}

// ------------------------------------------------------------------ batched form
// One persistent launch over many independent instances (graph, replica): each
// workgroup takes the next instance from an atomic queue (the host orders the
// queue longest first), builds its initial state in LDS (Philox spins, M, per-class
// counts, cut), runs every sweep with the same per-phase code as k_sweep_wg, and
// writes spins (original order), M and the tracked cut. Workgroups never wait on
// each other, so the launch needs no co-residency and always drains.
__global__ void __launch_bounds__(GDI_MAX_BLOCK) k_sweep_batch(GdiBatchArgs ba)
{
    extern __shared__ int32_t dyn[];
    __shared__ int32_t acc[3];
    __shared__ uint32_t thr_s[2 * GDI_WG_THR_MAX];
    __shared__ int32_t next_idx;
    __shared__ int64_t red[2];
    __shared__ int32_t tot_sh, cflag;
    const int tid = threadIdx.x;
    const int nth = blockDim.x;
    for (;;) {
        if (tid == 0) next_idx = atomicAdd(ba.queue, 1);
        __syncthreads();
        const int32_t idx = next_idx;
        __syncthreads();
        if (idx >= ba.n_inst) return;
        const GdiBatchInstance in = ba.inst[idx];

        GdiSweepArgs a{};
        a.rp = in.rp;
        a.adj = in.adj;
        a.orig = in.orig;
        a.cbeg = in.cbeg;
        a.csz = in.csz;
        a.thr = ba.thr;
        a.n = in.n;
        a.n_pad = in.n_pad;
        a.C = in.C;
        a.K = ba.K;
        a.t0 = 0;
        a.S = ba.S;
        a.A4 = ba.A4;
        a.B = ba.B;
        a.key0 = ba.key0;
        a.key1 = ba.key1;
        a.replica = in.replica;
        a.snapshot = ba.snapshot;
        a.rule = ba.rule;

        int32_t *Psh = dyn;
        const int c_round = (in.C + 3) & ~3;
        int8_t *sp = reinterpret_cast<int8_t *>(dyn + c_round);

        // initial state: Philox spins (counter (id, 0, replica, 1))
        for (int32_t v = tid; v < in.n_pad; v += nth) {
            const int32_t o = in.orig[v];
            int8_t s0 = 0;
            if (o >= 0) s0 = (philox10((uint32_t)o, 0u, in.replica, 1u, ba.key0, ba.key1).w0 & 1u) ? 1 : -1;
            sp[v] = s0;
        }
        for (int i = tid; i < in.C; i += nth) Psh[i] = 0;
        if (tid < 3) acc[tid] = 0;
        if (tid < 2) red[tid] = 0;
        if (tid == 0) cflag = 0;
        __syncthreads();
        int64_t m = 0, cw = 0;
        for (int32_t v = tid; v < in.n_pad; v += nth) {
            const int32_t s0 = sp[v];
            if (s0 == 0) continue;
            m += s0;
            if (s0 > 0) atomicAdd(&Psh[class_of(in.cbeg, in.C, v)], 1);
            for (int32_t k = in.rp[v]; k < in.rp[v + 1]; ++k) {
                const int2 e = in.adj[k];
                if (sp[e.x] != s0) cw += e.y;
            }
        }
        m = wave_sum_i64(m);
        cw = wave_sum_i64(cw);
        if ((tid & 63) == 0) {
            if (m) atomicAdd((unsigned long long *)&red[0], (unsigned long long)m);
            if (cw) atomicAdd((unsigned long long *)&red[1], (unsigned long long)cw);
        }
        __syncthreads();
        int32_t M = (int32_t)red[0];
        const int64_t cut0 = red[1] / 2;

        int64_t dcut_total = 0;
        if (in.members > 1) {
            switch (in.lanes) {
            case 1: cluster_run_sweeps<1>(a, in, sp, Psh, acc, thr_s, &tot_sh, &cflag, M, dcut_total, ba.spin_limit); break;
            case 2: cluster_run_sweeps<2>(a, in, sp, Psh, acc, thr_s, &tot_sh, &cflag, M, dcut_total, ba.spin_limit); break;
            case 4: cluster_run_sweeps<4>(a, in, sp, Psh, acc, thr_s, &tot_sh, &cflag, M, dcut_total, ba.spin_limit); break;
            case 8: cluster_run_sweeps<8>(a, in, sp, Psh, acc, thr_s, &tot_sh, &cflag, M, dcut_total, ba.spin_limit); break;
            case 16: cluster_run_sweeps<16>(a, in, sp, Psh, acc, thr_s, &tot_sh, &cflag, M, dcut_total, ba.spin_limit); break;
            case 32: cluster_run_sweeps<32>(a, in, sp, Psh, acc, thr_s, &tot_sh, &cflag, M, dcut_total, ba.spin_limit); break;
            default: cluster_run_sweeps<64>(a, in, sp, Psh, acc, thr_s, &tot_sh, &cflag, M, dcut_total, ba.spin_limit); break;
            }
            if (aborted(&cflag)) {
                if (tid == 0) __hip_atomic_store(ba.error, (int64_t)1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __syncthreads();
                continue;  // results of this instance are invalid; the host reports the error
            }
        } else if (in.wide) {
            switch (in.lanes) {
            case 1: wg_run_sweeps<1, 8>(a, sp, Psh, acc, thr_s, M, dcut_total); break;
            case 2: wg_run_sweeps<2, 8>(a, sp, Psh, acc, thr_s, M, dcut_total); break;
            case 4: wg_run_sweeps<4, 8>(a, sp, Psh, acc, thr_s, M, dcut_total); break;
            case 8: wg_run_sweeps<8, 8>(a, sp, Psh, acc, thr_s, M, dcut_total); break;
            case 16: wg_run_sweeps<16, 8>(a, sp, Psh, acc, thr_s, M, dcut_total); break;
            case 32: wg_run_sweeps<32, 8>(a, sp, Psh, acc, thr_s, M, dcut_total); break;
            default: wg_run_sweeps<64, 8>(a, sp, Psh, acc, thr_s, M, dcut_total); break;
            }
        } else {
            switch (in.lanes) {
            case 1: wg_run_sweeps<1>(a, sp, Psh, acc, thr_s, M, dcut_total); break;
            case 2: wg_run_sweeps<2>(a, sp, Psh, acc, thr_s, M, dcut_total); break;
            case 4: wg_run_sweeps<4>(a, sp, Psh, acc, thr_s, M, dcut_total); break;
            case 8: wg_run_sweeps<8>(a, sp, Psh, acc, thr_s, M, dcut_total); break;
            case 16: wg_run_sweeps<16>(a, sp, Psh, acc, thr_s, M, dcut_total); break;
            case 32: wg_run_sweeps<32>(a, sp, Psh, acc, thr_s, M, dcut_total); break;
            default: wg_run_sweeps<64>(a, sp, Psh, acc, thr_s, M, dcut_total); break;
            }
        }
        __syncthreads();
        if (in.out && in.rank == 0)
            for (int32_t v = tid; v < in.n_pad; v += nth) {
                const int32_t o = in.orig[v];
                if (o >= 0) in.out[o] = sp[v];
            }
        if (tid < 2) red[tid] = 0;
        __syncthreads();
        const int64_t w = wave_sum_i64(dcut_total);
        if ((tid & 63) == 0 && w != 0) atomicAdd((unsigned long long *)&red[1], (unsigned long long)w);
        __syncthreads();
        // every member ends with the same M; the cut changes of all members add up
        // (the host zeroes the results before the launch)
        if (tid == 0) {
            if (in.rank == 0) in.result[0] = M;
            atomicAdd((unsigned long long *)&in.result[1], (unsigned long long)((in.rank == 0 ? cut0 : 0) + red[1]));
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------ grid scope
// Two-level barrier that also sums the per-workgroup dM of phase p.
// Level 1: workgroups of group x = blockIdx % 8 add (2^40 + dM) to their group
// word; the last arriver (count == group size) adds (2^40 + group sum) to the
// phase's global word. Everyone polls the global word until it holds all
// groups. Counts live above bit 40, sums below (|sum| < 2^39).
__device__ __forceinline__ bool grid_phase_sync(const GdiSweepArgs &a, uint32_t p, int32_t d,
                                                uint32_t x, uint32_t gsz, uint32_t ngroups,
                                                int32_t *tot)
{
    const uint64_t one = 1ull << 40, half = 1ull << 39;
    uint64_t *gw = a.bar_grp + ((size_t)p * GDI_BAR_GROUPS + x) * GDI_BAR_PAD;
    uint64_t *glw = a.bar_glob + (size_t)p * GDI_BAR_PAD;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    const uint64_t add = one + (uint64_t)(int64_t)d;
    const uint64_t now = __hip_atomic_fetch_add(gw, add, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + add;
    const uint64_t cnt = (now + half) >> 40;
    if (cnt == gsz) {
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
        const uint64_t gsum = now - (cnt << 40);
        __hip_atomic_fetch_add(glw, one + gsum, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    for (int64_t tries = 0;; ++tries) {
        const uint64_t v = __hip_atomic_load(glw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint64_t c2 = (v + half) >> 40;
        if (c2 >= ngroups) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            *tot = (int32_t)(int64_t)(v - (c2 << 40));
            return true;
        }
        if (tries >= a.spin_limit) return false;
        __builtin_amdgcn_s_sleep(1);
    }
}

template <int L>
__global__ void __launch_bounds__(GDI_MAX_BLOCK) k_sweep_grid(GdiSweepArgs a)
{
    if (!gate_open(a)) return;
    extern __shared__ int32_t Psh[];
    __shared__ int32_t wg_acc;
    __shared__ int32_t total;
    __shared__ int32_t abort_flag;

    const uint32_t G = gridDim.x, b = blockIdx.x;
    // XCD-aware chunk order: consecutive workgroup ids land on different XCDs,
    // so give each XCD (b % 8) a contiguous range of chunks.
    const uint32_t q = (G % 8u == 0u) ? (b % 8u) * (G / 8u) + b / 8u : b;
    const uint32_t ngroups = G < GDI_BAR_GROUPS ? G : GDI_BAR_GROUPS;
    const uint32_t x = b % ngroups;
    const uint32_t gsz = G / ngroups + (x < G % ngroups ? 1u : 0u);

    const int tid = threadIdx.x;
    const int nth = blockDim.x;
    for (int i = tid; i < a.C; i += nth) Psh[i] = a.P[i];
    if (tid == 0) {
        wg_acc = 0;
        abort_flag = 0;
    }
    int32_t M = (int32_t)a.state[0];
    __syncthreads();

    const int sub = tid / L, lane = tid % L, nsub = nth / L;
    int64_t dcut = 0, dcut_total = 0;
    uint32_t p = 0;
    for (uint32_t t = a.t0; t < a.S; ++t) {
        const uint32_t *thr_row = a.thr + (size_t)t * (uint32_t)(a.K + 1);
        for (int32_t c = 0; c < a.C; ++c, ++p) {
            const int32_t beg = a.cbeg[c];
            const int32_t size = a.csz[c];
            const PhaseView pv = make_view(M, Psh[c], size, a.C, a.n);
            int32_t chunk = (size + (int32_t)G - 1) / (int32_t)G;
            chunk = (chunk + GDI_CLASS_ALIGN - 1) & ~(GDI_CLASS_ALIGN - 1);
            const int32_t lo = (int32_t)q * chunk;
            const int32_t hi = min(size, lo + chunk);
            int32_t dM = 0;
            for (int32_t j = lo + sub; j < hi; j += nsub) {
                const int32_t v = beg + j;
                if (a.mask && ((a.mask[v >> 5] >> (v & 31)) & 1u)) continue;  // skipped node
                int32_t h, sigma;
                const bool flip = node_decide<L>(a, a.spin, v, a.rp[v], a.rp[v + 1], lane, t, pv, thr_row, nullptr, &h,
                                                 &sigma);
                if (flip && lane == 0) {
                    a.spin[v] = (int8_t)(-sigma);
                    dM -= 2 * sigma;
                    dcut += (int64_t)sigma * h;
                    if (a.last_flip) a.last_flip[v] = (int32_t)t;
                }
            }
            dM = wave_sum_i32(dM);
            if ((tid & 63) == 0 && dM != 0) atomicAdd(&wg_acc, dM);
            __syncthreads();
            if (tid == 0) {
                const int32_t d = wg_acc;
                wg_acc = 0;
                int32_t tot = 0;
                if (!grid_phase_sync(a, p, d, x, gsz, ngroups, &tot)) {
                    abort_flag = 1;
                    __hip_atomic_store(&a.state[3], (int64_t)1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
                total = tot;
            }
            __syncthreads();
            if (abort_flag) return;
            const int32_t tot = total;
            M += tot;
            if (tid == 0 && a.C > 1) Psh[c] += tot / 2;
        }
        if (a.trace_m) {
            if (b == 0 && tid == 0) a.trace_m[t] = M;
            const int64_t w = wave_sum_i64(dcut);
            if ((tid & 63) == 0 && w != 0) atomicAdd((unsigned long long *)&a.trace_dcut[t], (unsigned long long)w);
            dcut_total += dcut;
            dcut = 0;
        }
    }
    dcut_total += dcut;
    __syncthreads();
    if (b == 0) {
        for (int i = tid; i < a.C; i += nth) a.P[i] = Psh[i];
        if (tid == 0) a.state[0] = M;
    }
    const int64_t w = wave_sum_i64(dcut_total);
    if ((tid & 63) == 0 && w != 0) atomicAdd((unsigned long long *)&a.state[1], (unsigned long long)w);
}


// ------------------------------------------------------------------ fixed scratch
// Device memory of the allocation-free entry point (gdi_cut_dev_noalloc): one array per
// GPU for the life of the process. Layout: [0, 32) the reduction's four int64
// accumulators, [256, 256 + 4 (GDI_NOALLOC_MAX_C + 2)) the per-class counts, from
// GDI_NOALLOC_SPIN_OFF the relabelled spin copy (n_pad bytes). Host code never uses the
// name: it takes the address from gdi_scratch_ptr.
static __device__ __align__(256) unsigned char scratch[GDI_NOALLOC_SCRATCH_BYTES];

// Weighted cut, crossing count and M from the reduction's accumulators (doubled sums).
__global__ void k_cut_finish(const int64_t *red, int64_t *out3)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        out3[0] = red[1] / 2;
        out3[1] = red[2] / 2;
        out3[2] = red[0];
    }
}

// ------------------------------------------------------------------ helpers
__global__ void k_init_spins(const int32_t *orig, const int8_t *init_orig, int8_t *spin, int32_t n_pad,
                             uint32_t key0, uint32_t key1, uint32_t replica)
{
    const int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n_pad) return;
    const int32_t o = orig[v];
    int8_t s = 0;
    if (o >= 0) {
        if (init_orig) {
            s = init_orig[o] > 0 ? 1 : -1;
        } else {
            const Words4 r = philox10((uint32_t)o, 0u, replica, 1u, key0, key1);
            s = (r.w0 & 1u) ? 1 : -1;
        }
    }
    spin[v] = s;
}

__global__ void k_gather_in(const int32_t *orig, const int8_t *in_orig, int32_t n_pad, int8_t *spin)
{
    const int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n_pad) return;
    const int32_t o = orig[v];
    spin[v] = o >= 0 ? (in_orig[o] > 0 ? 1 : -1) : 0;
}

__global__ void k_scatter_out(const int32_t *orig, const int8_t *spin, int32_t n_pad, int8_t *out_orig)
{
    const int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n_pad) return;
    const int32_t o = orig[v];
    if (o >= 0) out_orig[o] = spin[v];
}

__global__ void k_fill_u64(uint64_t *p, int64_t count)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t st = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = i; k < count; k += st) p[k] = 0;
}

// From-scratch M, doubled weighted cut, doubled crossing count and per-class +1 counts.
// From-scratch M, doubled weighted cut, doubled crossing count and per-class +1
// counts. Grid-stride over 64-id chunks: a chunk (one wave) never straddles a class
// because class starts are 64-aligned, so each wave adds its +1 count to one class
// counter; the three sums are reduced per workgroup in LDS, one atomic each.
// Bit-packed copy of the spins for the neighbour reads of k_reduce: bit i of word w is
// set iff spin 32w + i is +1 (n_pad is a multiple of 64). The first threads also clear
// k_reduce's accumulators (zero64 64-bit words of z64, zero32 32-bit words of z32), so
// that no separate fill launches precede it.
__global__ void k_pack_spins(const int8_t *spin, int32_t words, uint32_t *bits, int64_t *z64, int32_t zero64,
                             int32_t *z32, int32_t zero32)
{
    const int32_t w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w < zero64) z64[w] = 0;
    if (w < zero32) z32[w] = 0;
    if (w >= words) return;
    const uint4 *p = reinterpret_cast<const uint4 *>(spin + (size_t)w * 32);
    const uint4 lo = p[0], hi = p[1];
    const uint32_t x[8] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
    uint32_t word = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) word |= (((int8_t)(x[i] >> (8 * j)) > 0) ? 1u : 0u) << (4 * i + j);
    bits[w] = word;
}

// From-scratch M, doubled weighted cut, doubled crossing count and per-class +1
// counts. L lanes share a row and read consecutive entries (U per lane in flight), and
// a wave takes 64 / L consecutive rows, so a wave's entry loads cover one contiguous
// stretch of the CSR; its rows lie in one 64-id chunk, hence in one class (classes
// start at multiples of 64). A node's own spin comes from the int8 array; its
// neighbours' from the bit-packed copy (an eighth of the cache lines for the random
// reads, which dominate the kernel's memory traffic).
template <int L, int U = 4>
__global__ void __launch_bounds__(1024) k_reduce(const int32_t *rp, const int2 *adj, const int8_t *spin,
                                                const uint32_t *bits, int32_t n_pad, const int32_t *cbeg,
                                                const int32_t *csz, int32_t C, int64_t *out3, int32_t *P)
{
    __shared__ int64_t red[3][16];
    // with few classes, class starts and this block's +1 counts live in LDS (one global
    // atomic per class and block instead of one per 64-id chunk)
    __shared__ int32_t cb_sh[256], pc_sh[256];
    const bool local = C <= 256;
    if (local)
        for (int i = threadIdx.x; i < C; i += blockDim.x) {
            cb_sh[i] = cbeg[i];
            pc_sh[i] = 0;
        }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int sub = lane / L, l = lane % L;
    constexpr int RPW = 64 / L;  // rows per wave and round
    int64_t m = 0, cw = 0, ce = 0;
    const int32_t waves = (int32_t)(gridDim.x * (blockDim.x >> 6));
    for (int32_t v0 = (int32_t)(blockIdx.x * (blockDim.x >> 6) + wave) * RPW; v0 < n_pad; v0 += waves * RPW) {
        const int32_t v = v0 + sub;  // n_pad is a multiple of 64, so v < n_pad
        const int32_t s = spin[v];
        if (l == 0) m += s;
        const int32_t r0 = rp[v], r1 = rp[v + 1];
        for (int32_t k = r0 + l; k < r1; k += U * L) {
            int2 e[U];
#pragma unroll
            for (int u = 0; u < U; ++u) e[u] = k + u * L < r1 ? adj[k + u * L] : make_int2(v, 0);
            uint32_t wj[U];
#pragma unroll
            for (int u = 0; u < U; ++u) wj[u] = bits[e[u].x >> 5];
            // a real neighbour's spin is never 0, so it differs from s iff its bit does
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (k + u * L < r1 && (int32_t)((wj[u] >> (e[u].x & 31)) & 1u) != (s > 0 ? 1 : 0)) {
                    cw += e[u].y;
                    ce += 1;
                }
        }
        const int32_t plus = __popcll(__ballot(l == 0 && s > 0));
        if (lane == 0 && plus) {
            int32_t lo = 0, hi = C - 1;  // class of the chunk: last c with cbeg[c] <= v0
            while (lo < hi) {
                const int32_t mid = (lo + hi + 1) >> 1;
                if ((local ? cb_sh[mid] : cbeg[mid]) <= v0) lo = mid; else hi = mid - 1;
            }
            // padding ids hold spin 0 and never count
            if (local) atomicAdd(&pc_sh[lo], plus);
            else atomicAdd(&P[lo], plus);
        }
    }
    m = wave_sum_i64(m);
    cw = wave_sum_i64(cw);
    ce = wave_sum_i64(ce);
    if (lane == 0) {
        red[0][wave] = m;
        red[1][wave] = cw;
        red[2][wave] = ce;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        int64_t t = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[threadIdx.x][w];
        if (t) atomicAdd((unsigned long long *)&out3[threadIdx.x], (unsigned long long)t);
    }
    if (local)
        for (int i = threadIdx.x; i < C; i += blockDim.x)
            if (pc_sh[i]) atomicAdd(&P[i], pc_sh[i]);
}

// ------------------------------------------------------------------ standard solver
// The standard annealer of Alg. 2: every node computes the balance term from the
// whole spin vector -- the sum of all n spins and the over-side count of its class --
// instead of reading the tracked magnetisation. The scans read an LDS snapshot of the
// phase-start spins, so the decisions equal those of the tracked sweep bit for bit;
// only the cost differs (n reads per decision, n^2 per sweep). One workgroup, spins
// and snapshot in LDS; the L lanes of a node split its scans.
template <int L>
__device__ __forceinline__ int32_t subgroup_sum(int32_t v)
{
    return L > 1 ? group_sum<L>(v) : v;
}

template <int L>
__global__ void __launch_bounds__(GDI_MAX_BLOCK) k_sweep_dense(GdiSweepArgs a)
{
    extern __shared__ int32_t dyn[];
    __shared__ int32_t acc[3];
    const int c_round = (a.C + 3) & ~3;
    int32_t *Psh = dyn;
    int8_t *sp = reinterpret_cast<int8_t *>(dyn + c_round);
    int8_t *snap = sp + a.n_pad;
    const int tid = threadIdx.x, nth = blockDim.x;
    const int sub = tid / L, lane = tid % L, nsub = nth / L;
    for (int i = tid; i < a.C; i += nth) Psh[i] = a.P[i];
    for (int i = tid; i < a.n_pad; i += nth) sp[i] = a.spin[i];
    if (tid < 3) acc[tid] = 0;
    int32_t M = (int32_t)a.state[0];
    __syncthreads();

    int64_t dcut = 0, dcut_total = 0;
    uint32_t p = 0;
    for (uint32_t t = a.t0; t < a.S; ++t) {
        const uint32_t *thr_row = a.thr + (size_t)t * (uint32_t)(a.K + 1);
        for (int32_t c = 0; c < a.C; ++c, ++p) {
            const int32_t beg = a.cbeg[c];
            const int32_t size = a.csz[c];
            for (int i = tid; i < a.n_pad; i += nth) snap[i] = sp[i];
            __syncthreads();
            int32_t dM = 0;
            for (int32_t j = sub; j < size; j += nsub) {
                const int32_t v = beg + j;
                int32_t m = 0;
                for (int32_t i = lane; i < a.n_pad; i += L) m += snap[i];
                m = subgroup_sum<L>(m);
                const int32_t sg = (m > 0) - (m < 0);
                int32_t o = 0;
                if (sg != 0)
                    for (int32_t i = lane; i < size; i += L) o += snap[beg + i] == sg;
                o = subgroup_sum<L>(o);
                PhaseView pv;
                pv.M0 = m;
                pv.s = sg;
                pv.D = (m < 0 ? -m : m) >> 1;
                pv.O = (uint32_t)o;
                int32_t h, sigma;
                const bool flip = node_decide<L>(a, sp, v, a.rp[v], a.rp[v + 1], lane, t, pv, thr_row, nullptr, &h,
                                                 &sigma);
                if (flip && lane == 0) {
                    sp[v] = (int8_t)(-sigma);
                    dM -= 2 * sigma;
                    dcut += (int64_t)sigma * h;
                }
            }
            dM = wave_sum_i32(dM);
            if ((tid & 63) == 0 && dM != 0) atomicAdd(&acc[p % 3], dM);
            __syncthreads();
            const int32_t tot = acc[p % 3];
            M += tot;
            if (tid == 0) {
                if (a.C > 1) Psh[c] += tot / 2;
                acc[(p + 2) % 3] = 0;
            }
        }
        if (a.trace_m) {
            if (tid == 0) a.trace_m[t] = M;
            const int64_t w = wave_sum_i64(dcut);
            if ((tid & 63) == 0 && w != 0) atomicAdd((unsigned long long *)&a.trace_dcut[t], (unsigned long long)w);
            dcut_total += dcut;
            dcut = 0;
        }
    }
    dcut_total += dcut;
    __syncthreads();
    for (int i = tid; i < a.n_pad; i += nth) a.spin[i] = sp[i];
    for (int i = tid; i < a.C; i += nth) a.P[i] = Psh[i];
    if (tid == 0) a.state[0] = M;
    const int64_t w = wave_sum_i64(dcut_total);
    if ((tid & 63) == 0 && w != 0) atomicAdd((unsigned long long *)&a.state[1], (unsigned long long)w);
}

// ------------------------------------------------------------------ asynchronous sweep
// Alg. 3 as printed (Sec. V-C), racy by design, in one persistent cooperative launch:
// in every sweep each thread takes its nodes in turn (node v goes to thread
// v mod #threads, as when there are more spins than threads); for each node it reads
// the neighbour spins as it finds them (agent-scope loads: another node may or may
// not have flipped already, Sec. V-B), reads the global magnetisation G itself, makes
// the decision with the balance term of G, and when the spin flips stores it and adds
// its change to G with one atomic add. There are no colour phases and no gate; a
// device-wide barrier separates the sweeps (the schedule moves on only once every
// spin has updated). Results are not reproducible. G ends equal to the sum of the
// spins, since every change of a spin comes with its own atomic add.
__global__ void __launch_bounds__(1024) k_sweep_async(GdiSweepArgs a)
{
    __shared__ int32_t abort_flag;
    const uint32_t G = gridDim.x, b = blockIdx.x;
    const uint32_t ngroups = G < GDI_BAR_GROUPS ? G : GDI_BAR_GROUPS;
    const uint32_t x = b % ngroups;
    const uint32_t gsz = G / ngroups + (x < G % ngroups ? 1u : 0u);
    const int32_t nthr = (int32_t)(G * blockDim.x);
    const int32_t gid = (int32_t)(b * blockDim.x + threadIdx.x);
    if (threadIdx.x == 0) abort_flag = 0;
    __syncthreads();
    uint32_t p = 0;
    for (uint32_t t = a.t0; t < a.S; ++t, ++p) {
        const uint32_t *thr_row = a.thr + (size_t)t * (uint32_t)(a.K + 1);
        for (int32_t v = gid; v < a.n_pad; v += nthr) {
            const int32_t o = a.orig[v];
            if (o < 0) continue;  // padding
            int32_t h = 0;
            for (int32_t k = a.rp[v]; k < a.rp[v + 1]; ++k) {
                const int2 e = a.adj[k];
                h += e.y * (int32_t)__hip_atomic_load(&a.spin[e.x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            const int32_t sigma = a.spin[v];  // only this thread writes it
            const int32_t Mg = (int32_t)__hip_atomic_load(&a.state[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const int32_t dE = a.B * sigma * h + a.A4 * (1 - sigma * Mg);
            const Words4 xw = philox10((uint32_t)o, t, a.replica, 0u, a.key0, a.key1);
            bool flip;
            if (a.rule) flip = paper_flip(dE, sigma, xw.w0, xw.w2, thr_row[0]);
            else flip = dE <= 0 || (dE <= a.K && xw.w0 < thr_row[dE]);
            if (flip) {
                __hip_atomic_store(&a.spin[v], (int8_t)(-sigma), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_fetch_add(&a.state[0], (int64_t)(-2 * sigma), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        // the sweep ends when every thread has finished its nodes
        __syncthreads();
        if (threadIdx.x == 0) {
            int32_t tot = 0;
            if (!grid_phase_sync(a, p, 0, x, gsz, ngroups, &tot)) {
                abort_flag = 1;
                __hip_atomic_store(&a.state[3], (int64_t)1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        __syncthreads();
        if (abort_flag) return;
    }
}

inline int status(hipError_t e) { return (int)e; }

template <int L>
const void *wg_kernel(bool lds)
{
    return lds ? (const void *)k_sweep_wg<L, true> : (const void *)k_sweep_wg<L, false>;
}

const void *pick_wg(int lanes, bool lds)
{
    switch (lanes) {
    case 1: return wg_kernel<1>(lds);
    case 2: return wg_kernel<2>(lds);
    case 4: return wg_kernel<4>(lds);
    case 8: return wg_kernel<8>(lds);
    case 16: return wg_kernel<16>(lds);
    case 32: return wg_kernel<32>(lds);
    case 64: return wg_kernel<64>(lds);
    default: return nullptr;
    }
}

const void *pick_grid(int lanes)
{
    switch (lanes) {
    case 1: return (const void *)k_sweep_grid<1>;
    case 2: return (const void *)k_sweep_grid<2>;
    case 4: return (const void *)k_sweep_grid<4>;
    case 8: return (const void *)k_sweep_grid<8>;
    case 16: return (const void *)k_sweep_grid<16>;
    case 32: return (const void *)k_sweep_grid<32>;
    case 64: return (const void *)k_sweep_grid<64>;
    default: return nullptr;
    }
}

inline unsigned blocks_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

// ------------------------------------------------------------------ launchers
int gdi_launch_init_spins(const int32_t *orig, const int8_t *init_orig, int8_t *spin, int32_t n_pad,
                          uint32_t key0, uint32_t key1, uint32_t replica, void *stream)
{
    hipLaunchKernelGGL(k_init_spins, dim3(blocks_for(n_pad, 256)), dim3(256), 0, (hipStream_t)stream,
                       orig, init_orig, spin, n_pad, key0, key1, replica);
    return status(hipGetLastError());
}

int gdi_launch_gather_in(const int32_t *orig, const int8_t *in_orig, int32_t n_pad, int8_t *spin,
                         void *stream)
{
    hipLaunchKernelGGL(k_gather_in, dim3(blocks_for(n_pad, 256)), dim3(256), 0, (hipStream_t)stream,
                       orig, in_orig, n_pad, spin);
    return status(hipGetLastError());
}

int gdi_launch_scatter_out(const int32_t *orig, const int8_t *spin, int32_t n_pad, int8_t *out_orig,
                           void *stream)
{
    hipLaunchKernelGGL(k_scatter_out, dim3(blocks_for(n_pad, 256)), dim3(256), 0, (hipStream_t)stream,
                       orig, spin, n_pad, out_orig);
    return status(hipGetLastError());
}

int gdi_launch_fill_u64(uint64_t *p, int64_t count, void *stream)
{
    if (count <= 0) return 0;
    const unsigned g = (unsigned)std::min<int64_t>(blocks_for(count, 256), 4096);
    hipLaunchKernelGGL(k_fill_u64, dim3(g), dim3(256), 0, (hipStream_t)stream, p, count);
    return status(hipGetLastError());
}

int gdi_launch_reduce(const int32_t *rp, const int2 *adj, const int8_t *spin, int32_t n_pad, int64_t nnz,
                      const int32_t *cbeg, const int32_t *csz, int32_t C, int64_t *out3, int32_t *P,
                      uint32_t *bits, void *stream)
{
    if ((n_pad & 63) || (reinterpret_cast<uintptr_t>(spin) & 15)) return (int)hipErrorInvalidValue;
    const int32_t words = n_pad / 32;
    // the accumulators: out3[0..3] and P[0 .. 2 ((C + 2) / 2)), cleared by the first threads
    const int32_t zero32 = 2 * ((C + 2) / 2);
    const int32_t threads = std::max(std::max(words, zero32), 4);
    hipLaunchKernelGGL(k_pack_spins, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, (hipStream_t)stream, spin,
                       words, bits, out3, 4, P, zero32);
    // lanes per row: rows in flight matter more than lanes per row (each row is a chain of
    // row bound, entry and neighbour-spin loads); measured on MI355X over 1..32 lanes:
    // 2 or 4 best on RGGs of mean degree 8 (1M and 8M nodes) and on an ER graph of mean
    // degree 40, 16 and 32 up to 3.6x slower
    const double avg = n_pad ? (double)nnz / n_pad : 0.0;
    const int L = avg < 12.0 ? 2 : 4;
    // workgroups of 1024: one per 2048 padded nodes, between 256 and 1024, never more than
    // the rows need; every workgroup ends with a few atomic adds to the same words, which
    // the device serialises, so fewer and larger workgroups win (measured on MI355X, whole
    // cut call: 1M-node RGG 49.9 us with 1024 workgroups of 256 threads, 42.8 us with 256
    // of 1024, 39.6 us with 512 of 1024; 200k-node RGG 28.5, 19.2 and 20.1 us; 200k-node
    // ER graph of mean degree 40 48.7, 42.3 and 46.5 us)
    const int64_t rows_per_block = 16 * (64 / L);
    const int64_t want = std::min<int64_t>(1024, std::max<int64_t>(256, (int64_t)n_pad / 2048));
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>((n_pad + rows_per_block - 1) / rows_per_block, want));
    hipStream_t st = (hipStream_t)stream;
    if (L == 2)
        hipLaunchKernelGGL(k_reduce<2>, dim3(grid), dim3(1024), 0, st, rp, adj, spin, bits, n_pad, cbeg, csz, C, out3, P);
    else
        hipLaunchKernelGGL(k_reduce<4>, dim3(grid), dim3(1024), 0, st, rp, adj, spin, bits, n_pad, cbeg, csz, C, out3, P);
    return status(hipGetLastError());
}

int gdi_launch_cut_finish(const int64_t *red, int64_t *out3, void *stream)
{
    hipLaunchKernelGGL(k_cut_finish, dim3(1), dim3(64), 0, (hipStream_t)stream, red, out3);
    return status(hipGetLastError());
}

// Address of this GPU's scratch array: looked up once per device, with the device
// current, through hipGetSymbolAddress, and kept (each GPU holds its own copy).
int gdi_scratch_ptr(void **out)
{
    static std::mutex mu;
    static void *addr[GDI_NOALLOC_MAX_DEVICES] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return status(e);
    if (dev < 0 || dev >= GDI_NOALLOC_MAX_DEVICES) return (int)hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return status(e);
        addr[dev] = p;
    }
    *out = addr[dev];
    return 0;
}

int gdi_dense_lds_bytes(int32_t n_pad, int32_t C) { return ((C + 3) & ~3) * 4 + 2 * n_pad; }

int gdi_async_capacity(int block, int *max_grid)
{
    int dev = 0, cus = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)k_sweep_async, block, 0);
    if (e != hipSuccess) return status(e);
    // one workgroup per compute unit: with the occupancy figure above one (two
    // 1024-thread workgroups per CU) the sweep barrier was not reached by every
    // workgroup (bounded wait expired), so co-residency is only relied on at one
    *max_grid = cus * std::min(per_cu, 1);
    return 0;
}

int gdi_launch_sweep_async(const GdiSweepArgs &a, int grid, int block, void *stream)
{
    GdiSweepArgs copy = a;
    void *args[] = {&copy};
    return status(hipLaunchCooperativeKernel((const void *)k_sweep_async, dim3(grid), dim3(block), args, 0u,
                                             (hipStream_t)stream));
}

int gdi_launch_sweep_dense(const GdiSweepArgs &a, int block, int lanes, void *stream)
{
    const void *f = nullptr;
    switch (lanes) {
    case 1: f = (const void *)k_sweep_dense<1>; break;
    case 2: f = (const void *)k_sweep_dense<2>; break;
    case 4: f = (const void *)k_sweep_dense<4>; break;
    case 8: f = (const void *)k_sweep_dense<8>; break;
    case 16: f = (const void *)k_sweep_dense<16>; break;
    case 32: f = (const void *)k_sweep_dense<32>; break;
    case 64: f = (const void *)k_sweep_dense<64>; break;
    default: return (int)hipErrorInvalidValue;
    }
    const int lds = gdi_dense_lds_bytes(a.n_pad, a.C);
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return status(e);
    GdiSweepArgs copy = a;
    void *args[] = {&copy};
    e = hipLaunchKernel(f, dim3(1), dim3(block), args, (size_t)lds, (hipStream_t)stream);
    return status(e);
}

int gdi_wg_lds_bytes(int32_t n_pad, int32_t C, int spins_in_lds)
{
    const int c_round = (C + 3) & ~3;
    return c_round * 4 + (spins_in_lds ? n_pad : 0);
}

int gdi_launch_sweep_wg(const GdiSweepArgs &a, int block, int lanes, int spins_in_lds, void *stream)
{
    const void *f = pick_wg(lanes, spins_in_lds != 0);
    if (!f) return (int)hipErrorInvalidValue;
    const int lds = gdi_wg_lds_bytes(a.n_pad, a.C, spins_in_lds);
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return status(e);
    GdiSweepArgs copy = a;
    void *args[] = {&copy};
    e = hipLaunchKernel(f, dim3(1), dim3(block), args, (size_t)lds, (hipStream_t)stream);
    return status(e);
}

int gdi_wgl_lds_bytes(int32_t n_pad, int32_t C, int32_t nnz)
{
    return wgl_c_round(C) * 4 + n_pad * 4 + ((n_pad + 2) & ~1) * 2 + ((nnz + 1) & ~1) * 2 + n_pad;
}

int gdi_launch_sweep_wgl(const GdiSweepArgs &a, const uint16_t *rp16, const uint16_t *ent16, int32_t nnz, int block,
                         int lanes, void *stream)
{
    const void *f = nullptr;
    switch (lanes) {
    case 1: f = (const void *)k_sweep_wgl<1>; break;
    case 2: f = (const void *)k_sweep_wgl<2>; break;
    case 4: f = (const void *)k_sweep_wgl<4>; break;
    case 8: f = (const void *)k_sweep_wgl<8>; break;
    case 16: f = (const void *)k_sweep_wgl<16>; break;
    case 32: f = (const void *)k_sweep_wgl<32>; break;
    case 64: f = (const void *)k_sweep_wgl<64>; break;
    default: return (int)hipErrorInvalidValue;
    }
    const int lds = gdi_wgl_lds_bytes(a.n_pad, a.C, nnz);
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return status(e);
    GdiSweepArgs copy = a;
    void *args[] = {&copy, &rp16, &ent16, &nnz};
    e = hipLaunchKernel(f, dim3(1), dim3(block), args, (size_t)lds, (hipStream_t)stream);
    return status(e);
}

int gdi_active_lds_bytes(int32_t n_pad, int32_t C)
{
    return (n_pad / 32) * 4 + (4 * C + 2) * 4;
}

int gdi_launch_sweep_active(const GdiSweepArgs &a, GdiActiveRec *rec, void *stream)
{
    const void *f = (const void *)k_sweep_active;
    if ((a.n_pad & 63) || (reinterpret_cast<uintptr_t>(a.spin) & 15) || (reinterpret_cast<uintptr_t>(a.mask) & 7))
        return (int)hipErrorInvalidValue;
    // the bits and counts, then the launch's threshold rows if they fit beside them
    int dev = 0, lds_max = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    if (e != hipSuccess) return status(e);
    const int base = gdi_active_lds_bytes(a.n_pad, a.C);
    int32_t thr_off = (base + 15) & ~15;
    const int64_t want = a.S > a.t0 ? (int64_t)(a.S - a.t0) * (a.K + 1) * 4 : 0;
    int32_t thr_bytes = (int64_t)thr_off + want + 512 <= (int64_t)lds_max ? (int32_t)want : 0;
    const int lds = thr_bytes > 0 ? thr_off + thr_bytes : base;
    e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return status(e);
    GdiSweepArgs copy = a;
    void *args[] = {&copy, &rec, &thr_off, &thr_bytes};
    e = hipLaunchKernel(f, dim3(1), dim3(GDI_MAX_BLOCK), args, (size_t)lds, (hipStream_t)stream);
    return status(e);
}

int gdi_grid_capacity(int block, int lanes, int *max_grid)
{
    const void *f = pick_grid(lanes);
    if (!f) return (int)hipErrorInvalidValue;
    int dev = 0, cus = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, block, 256);
    if (e != hipSuccess) return status(e);
    *max_grid = cus * per_cu;
    return 0;
}

int gdi_launch_sweep_grid(const GdiSweepArgs &a, int grid, int block, int lanes, void *stream)
{
    const void *f = pick_grid(lanes);
    if (!f) return (int)hipErrorInvalidValue;
    const int lds = ((a.C + 3) & ~3) * 4;
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return status(e);
    GdiSweepArgs copy = a;
    void *args[] = {&copy};
    e = hipLaunchCooperativeKernel(f, dim3(grid), dim3(block), args, (unsigned)lds, (hipStream_t)stream);
    return status(e);
}



int gdi_batch_lds_bytes(int32_t n_pad, int32_t C)
{
    return ((C + 3) & ~3) * 4 + n_pad;
}

int gdi_launch_sweep_batch(const GdiBatchArgs &ba, int grid, int block, int lds_bytes, int cooperative, void *stream)
{
    const void *f = (const void *)k_sweep_batch;
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
    if (e != hipSuccess) return status(e);
    GdiBatchArgs copy = ba;
    void *args[] = {&copy};
    // clusters wait for each other: their launch must be co-resident
    e = cooperative ? hipLaunchCooperativeKernel(f, dim3(grid), dim3(block), args, (unsigned)lds_bytes, (hipStream_t)stream)
                    : hipLaunchKernel(f, dim3(grid), dim3(block), args, (size_t)lds_bytes, (hipStream_t)stream);
    return status(e);
}

int gdi_batch_occupancy(int block, int lds_bytes, int *per_cu)
{
    const void *f = (const void *)k_sweep_batch;
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, f, block, lds_bytes);
    return status(e);
}

const char *gdi_hip_error_string(int code) { return hipGetErrorString((hipError_t)code); }
