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

// ------------------------------------------------------------------ Philox4x32-10
// Counter-based generator of Salmon, Moraes, Dror and Shaw (SC'11): ten rounds of
// two 32x32->64 multiplies (multipliers 0xD2511F53, 0xCD9E8D57) whose high halves
// are xored into the other counter words together with the key, and a Weyl key
// schedule (0x9E3779B9, 0xBB67AE85).
struct Words4 {
    uint32_t w0, w1, w2, w3;
};

__device__ __forceinline__ Words4 philox10(uint32_t x0, uint32_t x1, uint32_t x2, uint32_t x3,
                                           uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // each 32 x 32 -> 64-bit product as one multiply-add (both halves at once)
        const uint64_t pa = (uint64_t)0xD2511F53u * x0;
        const uint64_t pb = (uint64_t)0xCD9E8D57u * x2;
        x0 = (uint32_t)(pb >> 32) ^ x1 ^ k0;
        x1 = (uint32_t)pb;
        x2 = (uint32_t)(pa >> 32) ^ x3 ^ k1;
        x3 = (uint32_t)pa;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return {x0, x1, x2, x3};
}

// Wave-wide sum with DPP lane moves (no LDS round trips): within quads, then mirrored
// half-rows and rows, then rows 1 and 3 add the last lane of rows 0 and 2, rows 2 and 3
// that of row 1; lane 63 ends with the total. All 64 lanes must be active.
__device__ __forceinline__ int32_t wave_sum_i32(int32_t v)
{
    v += __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xf, 0xf, false);   // quad_perm [1,0,3,2]
    v += __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xf, 0xf, false);   // quad_perm [2,3,0,1]
    v += __builtin_amdgcn_update_dpp(0, v, 0x141, 0xf, 0xf, false);  // row_half_mirror
    v += __builtin_amdgcn_update_dpp(0, v, 0x140, 0xf, 0xf, false);  // row_mirror
    v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);  // row_bcast:15
    v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);  // row_bcast:31
    return __builtin_amdgcn_readlane(v, 63);
}

// Sum over each aligned group of L lanes, left in every lane of the group: DPP moves
// within quads, half-rows and rows (every lane they read belongs to the same group),
// then lane shuffles for groups of 32 and 64.
template <int L>
__device__ __forceinline__ int32_t group_sum(int32_t v)
{
    if (L >= 2) v += __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xf, 0xf, false);   // quad_perm [1,0,3,2]
    if (L >= 4) v += __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xf, 0xf, false);   // quad_perm [2,3,0,1]
    if (L >= 8) v += __builtin_amdgcn_update_dpp(0, v, 0x141, 0xf, 0xf, false);  // row_half_mirror
    if (L >= 16) v += __builtin_amdgcn_update_dpp(0, v, 0x140, 0xf, 0xf, false); // row_mirror
    if (L >= 32) v += __shfl_xor(v, 16, 64);
    if (L >= 64) v += __shfl_xor(v, 32, 64);
    return v;
}

__device__ __forceinline__ int64_t wave_sum_i64(int64_t v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Magnetisation snapshot of one phase: what every node of the class reads.
struct PhaseView {
    int32_t M0;   // magnetisation at the start of the phase
    int32_t s;    // sign(M0)
    int32_t D;    // floor(|M0| / 2): flips that would restore balance
    uint32_t O;   // over-side spins (s_i == s) in the class
};

__device__ __forceinline__ PhaseView make_view(int32_t M0, int32_t P_c, int32_t size_c, int32_t C,
                                               int32_t n)
{
    PhaseView v;
    v.M0 = M0;
    v.s = (M0 > 0) - (M0 < 0);
    v.D = (M0 < 0 ? -M0 : M0) >> 1;
    // with a single class P_c is implied by M: (M + n) / 2 spins are +1
    const int32_t pc = (C == 1) ? (M0 + n) / 2 : P_c;
    v.O = (uint32_t)(v.s > 0 ? pc : (v.s < 0 ? size_c - pc : 0));
    return v;
}

// Threshold i of the current row, from LDS when staged there, else from global
// memory. The LDS read goes through an LDS-qualified pointer: a choice between two
// generic pointers would become one flat load, whose wait also waits for every
// outstanding global load of the wave.
typedef __attribute__((address_space(3))) const uint32_t gdi_lds_cu32;
__device__ __forceinline__ uint32_t thr_at(const uint32_t *thr_l, const uint32_t *thr_g, bool in_lds, int32_t i)
{
    if (in_lds) return ((gdi_lds_cu32 *)thr_l)[i];
    return thr_g[i];
}

// The paper's acceptance rule (Sec. V, Alg. 2/3): the spin takes the value of lower
// local energy -- flip iff dE < 0; on a tie (dE = 0, a zero local field) the value is
// random (Sec. III), +1 iff Philox word x2 is odd -- and then flips with probability
// P_f, i.e. iff x0 < pf_thr = min(2^32 - 1, floor(2^32 P_f)). The two flips compose.
__device__ __forceinline__ bool paper_flip(int32_t dE, int32_t sigma, uint32_t x0, uint32_t x2, uint32_t pf_thr)
{
    const bool argmin_flips = dE < 0 || (dE == 0 && ((x2 & 1u) ? 1 : -1) != sigma);
    return argmin_flips != (x0 < pf_thr);
}

// Metropolis decision of one node (original id o) given its local field h and spin
// sigma (eq. 5 / eq. 6 flip cost with the gated balance term). Philox words are
// drawn only when the gate or the threshold lookup needs them. The threshold row is
// thr_l in LDS when staged there (non-null), else thr_row in global memory.
__device__ __forceinline__ bool decide_id(const GdiSweepArgs &a, uint32_t o, uint32_t t, int32_t sigma,
                                          int32_t h, const PhaseView &pv, const uint32_t *thr_row,
                                          const uint32_t *thr_l = nullptr)
{
    const bool need_gate = !a.snapshot && pv.D > 0 && sigma == pv.s;
    Words4 r{0u, 0u, 0u, 0u};
    bool have = false;
    if (need_gate) {
        r = philox10(o, t, a.replica, 0u, a.key0, a.key1);
        have = true;
    }
    int32_t m_seen;
    if (a.snapshot) {
        m_seen = pv.M0;
    } else {
        const bool gated = need_gate && ((uint64_t)r.w1 * pv.O < ((uint64_t)(uint32_t)pv.D << 32));
        m_seen = gated ? pv.M0 : 0;
    }
    const int32_t dE = a.B * sigma * h + a.A4 * (1 - sigma * m_seen);
    if (a.rule) {  // the paper's rule: the argmin value, then a random flip with probability P_f
        if (!have) r = philox10(o, t, a.replica, 0u, a.key0, a.key1);
        return paper_flip(dE, sigma, r.w0, r.w2, thr_at(thr_l, thr_row, thr_l != nullptr, 0));
    }
    if (dE <= 0) return true;
    if (dE > a.K) return false;
    if (!have) r = philox10(o, t, a.replica, 0u, a.key0, a.key1);
    return r.w0 < thr_at(thr_l, thr_row, thr_l != nullptr, dE);
}

// Launch gate of the masked sweeps: the active-set kernel and the full-graph
// kernels are both enqueued and exactly one of them runs, chosen on the device from
// the number of active nodes (the same value for every workgroup).
__device__ __forceinline__ bool gate_open(const GdiSweepArgs &a)
{
    if (!a.skip_count) return true;
    const int64_t active = (int64_t)a.n - (int64_t)*a.skip_count;
    return (active <= a.active_max) == (a.gate_small != 0);
}

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

// ------------------------------------------------------------------ workgroup scope
// All sweeps of one instance inside one workgroup: phases are separated by
// s_barrier, dM is summed in an LDS triple buffer (one barrier per phase).
// sp points to the instance's spins (LDS, or global for large instances),
// Psh to its per-class +1 counts in LDS, acc to three zeroed LDS words.
template <int L, int U = 4>
__device__ void wg_run_sweeps(const GdiSweepArgs &a, int8_t *sp, int32_t *Psh, int32_t *acc, int32_t &M,
                              int64_t &dcut_total)
{
    const int tid = threadIdx.x;
    const int nth = blockDim.x;
    const int sub = tid / L, lane = tid % L, nsub = nth / L;
    int64_t dcut = 0;
    uint32_t p = 0;
    // the current and the next threshold row in LDS when they fit (staged during the
    // last phase of each sweep, whose barrier publishes them)
    __shared__ uint32_t thr_s[2 * GDI_WG_THR_MAX];
    const int32_t K1 = a.K + 1;
    const bool thr_lds = K1 <= GDI_WG_THR_MAX;
    if (thr_lds && a.t0 < a.S)
        for (int i = tid; i < K1; i += nth) thr_s[(a.t0 & 1u) * GDI_WG_THR_MAX + i] = a.thr[(size_t)a.t0 * K1 + i];
    __syncthreads();
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
            if (sub < size) {
                nr0 = a.rp[beg + sub];
                nr1 = a.rp[beg + sub + 1];
            }
            for (int32_t j = sub; j < size; j += nsub) {
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
    wg_run_sweeps<L>(a, sp, Psh, acc, M, dcut_total);

    __syncthreads();
    if (SPIN_LDS)
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
// Masked sweeps of the learned proposal in one workgroup when few nodes are active:
// every spin of the graph is one bit in LDS (so neighbour reads never leave the CU),
// the active nodes (mask bit clear, real ids) are compacted at the start into
// records {new id, row, original id} in class order, and a class with no active node
// takes no phase at all -- nothing in it can change, so M and the class counts stay.
// The decisions are those of the full-graph kernels with the mask applied.
__global__ void __launch_bounds__(GDI_MAX_BLOCK) k_sweep_active(GdiSweepArgs a, GdiActiveRec *rec)
{
    if (!gate_open(a)) return;
    extern __shared__ uint32_t lds[];
    const int32_t nw = a.n_pad >> 5;
    uint32_t *bits = lds;                                           // n_pad spin bits (1 = +1)
    int32_t *abeg = reinterpret_cast<int32_t *>(lds + nw);          // C + 1 record offsets
    int32_t *Psh = abeg + a.C + 1;                                  // C counts of +1
    __shared__ int32_t acc[3];
    __shared__ int32_t wtot[GDI_MAX_BLOCK / 64];
    __shared__ int32_t base_sh;
    const int tid = threadIdx.x, nth = blockDim.x;
    const int lane = tid & 63, wave = tid >> 6, nwaves = nth >> 6;

    // spins -> bits, 64 ids per wave step (n_pad is a multiple of 64)
    for (int32_t b0 = wave * 64; b0 < a.n_pad; b0 += nwaves * 64) {
        const uint64_t b = __ballot(a.spin[b0 + lane] > 0);
        if (lane == 0) {
            bits[b0 >> 5] = (uint32_t)b;
            bits[(b0 >> 5) + 1] = (uint32_t)(b >> 32);
        }
    }
    for (int i = tid; i < a.C; i += nth) Psh[i] = a.P[i];
    if (tid < 3) acc[tid] = 0;
    if (tid == 0) base_sh = 0;
    int32_t M = (int32_t)a.state[0];
    __syncthreads();

    // compaction: one 64-id chunk per thread per round; chunks never straddle classes
    const int32_t nch = a.n_pad >> 6;
    for (int32_t r0 = 0; r0 < nch; r0 += nth) {
        const int32_t ch = r0 + tid;
        uint64_t act = 0;
        int32_t c = -1;
        if (ch < nch) {
            const int32_t v0 = ch << 6;
            c = class_of(a.cbeg, a.C, v0);
            const int32_t nv = min(64, max(0, a.cbeg[c] + a.csz[c] - v0));
            const uint64_t valid = nv == 64 ? ~0ull : ((1ull << nv) - 1ull);
            const uint64_t m = a.mask ? ((uint64_t)a.mask[2 * ch] | ((uint64_t)a.mask[2 * ch + 1] << 32)) : 0ull;
            act = valid & ~m;
            if (v0 != a.cbeg[c]) c = -1;  // c >= 0 only on the first chunk of a class
        }
        const int32_t cnt = __popcll(act);
        int32_t incl = cnt;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int32_t y = __shfl_up(incl, off, 64);
            if (lane >= off) incl += y;
        }
        if (lane == 63) wtot[wave] = incl;
        __syncthreads();
        int32_t before = 0, round_total = 0;
        for (int w = 0; w < nwaves; ++w) {
            before += w < wave ? wtot[w] : 0;
            round_total += wtot[w];
        }
        int32_t pos = base_sh + before + incl - cnt;
        if (c >= 0) abeg[c] = pos;
        for (uint64_t x = act; x; x &= x - 1) {
            const int32_t v = (ch << 6) + __ffsll((unsigned long long)x) - 1;
            rec[pos++] = GdiActiveRec{v, a.rp[v], a.rp[v + 1], a.orig[v]};
        }
        __syncthreads();
        if (tid == 0) base_sh += round_total;
        __syncthreads();
    }
    if (tid == 0) abeg[a.C] = base_sh;
    __syncthreads();

    int64_t dcut = 0;
    uint32_t p = 0;
    for (uint32_t t = a.t0; t < a.S; ++t) {
        const uint32_t *thr_row = a.thr + (size_t)t * (uint32_t)(a.K + 1);
        for (int32_t c = 0; c < a.C; ++c) {
            const int32_t jb = abeg[c], je = abeg[c + 1];
            if (jb == je) continue;
            const PhaseView pv = make_view(M, Psh[c], a.csz[c], a.C, a.n);
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
                if (decide_id(a, (uint32_t)r.orig, t, sigma, h, pv, thr_row)) {
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
    __shared__ int32_t next_idx;
    __shared__ int64_t red[2];
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
        if (in.wide) {
            switch (in.lanes) {
            case 1: wg_run_sweeps<1, 8>(a, sp, Psh, acc, M, dcut_total); break;
            case 2: wg_run_sweeps<2, 8>(a, sp, Psh, acc, M, dcut_total); break;
            case 4: wg_run_sweeps<4, 8>(a, sp, Psh, acc, M, dcut_total); break;
            case 8: wg_run_sweeps<8, 8>(a, sp, Psh, acc, M, dcut_total); break;
            case 16: wg_run_sweeps<16, 8>(a, sp, Psh, acc, M, dcut_total); break;
            case 32: wg_run_sweeps<32, 8>(a, sp, Psh, acc, M, dcut_total); break;
            default: wg_run_sweeps<64, 8>(a, sp, Psh, acc, M, dcut_total); break;
            }
        } else {
            switch (in.lanes) {
            case 1: wg_run_sweeps<1>(a, sp, Psh, acc, M, dcut_total); break;
            case 2: wg_run_sweeps<2>(a, sp, Psh, acc, M, dcut_total); break;
            case 4: wg_run_sweeps<4>(a, sp, Psh, acc, M, dcut_total); break;
            case 8: wg_run_sweeps<8>(a, sp, Psh, acc, M, dcut_total); break;
            case 16: wg_run_sweeps<16>(a, sp, Psh, acc, M, dcut_total); break;
            case 32: wg_run_sweeps<32>(a, sp, Psh, acc, M, dcut_total); break;
            default: wg_run_sweeps<64>(a, sp, Psh, acc, M, dcut_total); break;
            }
        }
        __syncthreads();
        if (in.out)
            for (int32_t v = tid; v < in.n_pad; v += nth) {
                const int32_t o = in.orig[v];
                if (o >= 0) in.out[o] = sp[v];
            }
        if (tid < 2) red[tid] = 0;
        __syncthreads();
        const int64_t w = wave_sum_i64(dcut_total);
        if ((tid & 63) == 0 && w != 0) atomicAdd((unsigned long long *)&red[1], (unsigned long long)w);
        __syncthreads();
        if (tid == 0) {
            in.result[0] = M;
            in.result[1] = cut0 + red[1];
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

__device__ __forceinline__ uint64_t ld_agent(const uint64_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void st_agent(uint64_t *p, uint64_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The abort flag lives in LDS; workgroup-scope atomics keep it an LDS access
// (a volatile generic pointer would become a flat access whose wait also waits
// for every outstanding global load of the wave).
__device__ __forceinline__ bool aborted(int32_t *flag)
{
    return __hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) != 0;
}

__device__ __forceinline__ void set_abort(int32_t *flag)
{
    __hip_atomic_store(flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

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

// Bounded poll of one epoch-tagged word; returns false on timeout or abort.
__device__ __forceinline__ bool poll_word(const uint64_t *w, uint32_t epoch, int64_t limit,
                                          int32_t *abort_v, int32_t *payload)
{
    for (int64_t tries = 0;; ++tries) {
        const uint64_t v = ld_agent(w);
        if ((uint32_t)(v >> 32) >= epoch) {
            *payload = (int32_t)(uint32_t)v;
            return true;
        }
        if (tries >= limit || aborted(abort_v)) return false;
        __builtin_amdgcn_s_sleep(1);
    }
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
    if (!gate_open(a)) return;
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
    if (thr_lds && a.t0 < a.S)
        for (int i = tid; i < K1; i += nth) thr_sh[(a.t0 & 1u) * K1 + i] = a.thr[(size_t)a.t0 * K1 + i];
    if (tid == 0) {
        wg_acc = 0;
        total_sh = 0;
        abort_sh = 0;
    }
    if (tid < 3) tacc[tid] = 0;
    if (tid == 0) wdone = 0;
    int32_t M = (int32_t)a.state[0];
    __syncthreads();

    // prologue: the foreign-word ids, then every own, foreign and gather word and the tail
    // region straight from the spin array, which no workgroup writes before its epilogue,
    // so no workgroup waits for another here (words published during the launch carry
    // epochs >= 2)
    for (int32_t i = tid; i < h.flist_len; i += nth) bits[h.list_off + i] = (uint32_t)h.flist[(size_t)b * h.flist_len + i];
    __syncthreads();
    for (int32_t c = 0; c < T0; ++c) {
        const GdiHaloEntry e = tab[c];
        const int32_t w0 = e.node_lo >> 5, nown = e.node_hi > e.node_lo ? ((e.node_hi + 31) >> 5) - w0 : 0;
        for (int32_t wd = tid; wd < nown; wd += nth) bits[e.own_off + wd] = pack_spins(a.spin, w0 + wd);
        for (int32_t i = tid; i < e.for_len; i += nth)
            bits[e.for_off + i] = pack_spins(a.spin, (int32_t)bits[e.list_off + i]);
    }
    if (has_tail)
        for (int32_t i = tid; i < h.gat_beg[T0]; i += nth) bits[h.gather_off + i] = pack_spins(a.spin, h.gat_words[i]);
    for (int32_t b0 = tail_base + wave * 64; b0 < a.n_pad; b0 += nwaves * 64) {
        const uint64_t m = __ballot(a.spin[b0 + lane] > 0);
        if (lane == 0) {
            bits[h.tail_off + ((b0 - tail_base) >> 5)] = (uint32_t)m;
            bits[h.tail_off + ((b0 - tail_base) >> 5) + 1] = (uint32_t)(m >> 32);
        }
    }
    // the tail's CSR (row offsets, then entries as LDS bit index and weight) stays in LDS
    int32_t *trp = reinterpret_cast<int32_t *>(bits + h.trp_off);
    uint32_t *tent = bits + h.tent_off;
    if (has_tail) {
        for (int32_t i = tid; i <= h.tail_n; i += nth) trp[i] = h.tail_rp[i];
        for (int32_t i = tid; i < h.tail_nnz; i += nth) tent[i] = h.tail_ent[i];
    }
    // overflow entries of this workgroup's long rows
    for (int32_t i = tid; i < h.ovf_len; i += nth) bits[h.ovf_off + i] = h.ovf[(size_t)b * h.ovf_len + i];
    // pipeline fill: phase 0 entries, phase 1 rows
    NodePrefetch pf;
    RowAhead ra;
    {
        const uint32_t t1 = T0 > 1 ? a.t0 : a.t0 + 1u;
        const int32_t s1 = T0 > 1 ? 1 : 0;
        const int32_t v0 = step_node(h, tab, 0, tid);
        if (worker && a.t0 < a.S && v0 >= 0) {
            load_row(a, v0, ra);
            load_entries(h, ra, a.t0, pf);
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
    for (uint32_t t = a.t0; t < a.S; ++t) {
        const uint32_t *thr_l = thr_sh + (t & 1u) * K1;
        const uint32_t *thr_g = a.thr + (size_t)t * K1;
        for (int32_t c = 0; c < T0; ++c, ++p) {
            const GdiHaloEntry e = tab[c];
            const uint32_t epoch = p + 2u;
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
                for (int32_t base = e.node_lo; base < e.node_hi; base += nwork) {
                    const int32_t v = base + tid;
                    const bool active = v < e.node_hi;
                    bool flip = false;
                    int32_t sigma_l = 0;
                    if (active && !(a.mask && ((a.mask[v >> 5] >> (v & 31)) & 1u))) {
                        NodePrefetch q;
                        if (base != e.node_lo) {
                            RowAhead rq;
                            load_row(a, v, rq);
                            load_entries(h, rq, t, q);
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
                const bool want1 = t1 < a.S && v1 >= 0 && !(a.mask && ((a.mask[v1 >> 5] >> (v1 & 31)) & 1u));
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
            if (worker && !poll_gather(h, T0 - 1, bits, p + 1u, tid, nwork, abort_v)) set_abort(abort_v);
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
                if (worker && my_tc == tc && !(a.mask && ((a.mask[my_tail >> 5] >> (my_tail & 31)) & 1u))) {
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
    const int64_t w = wave_sum_i64(dcut_total);
    if (lane == 0 && w != 0) atomicAdd((unsigned long long *)&a.state[1], (unsigned long long)w);
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
__global__ void __launch_bounds__(256) k_reduce(const int32_t *rp, const int2 *adj, const int8_t *spin, int32_t n_pad,
                                                const int32_t *cbeg, const int32_t *csz, int32_t C, int64_t *out3,
                                                int32_t *P)
{
    __shared__ int64_t red[3][4];
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
    int64_t m = 0, cw = 0, ce = 0;
    for (int32_t base = blockIdx.x * blockDim.x; base < n_pad; base += gridDim.x * blockDim.x) {
        const int32_t v0 = base + (wave << 6);
        const int32_t v = v0 + lane;
        int32_t s = 0;
        if (v < n_pad) {
            s = spin[v];
            m += s;
            // eight entries per round, every load of a round issued before any is used;
            // entries past the row are not loaded and count for nothing
            const int32_t r0 = rp[v], r1 = rp[v + 1];
            for (int32_t k = r0; k < r1; k += 8) {
                int2 e[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) e[u] = k + u < r1 ? adj[k + u] : make_int2(v, 0);
                int8_t sj[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) sj[u] = spin[e[u].x];
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    if (k + u < r1 && sj[u] != s) {
                        cw += e[u].y;
                        ce += 1;
                    }
            }
        }
        const int32_t plus = __popcll(__ballot(s > 0));
        if (lane == 0 && plus && v0 < n_pad) {
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

int gdi_launch_reduce(const int32_t *rp, const int2 *adj, const int8_t *spin, int32_t n_pad,
                      const int32_t *cbeg, const int32_t *csz, int32_t C, int64_t *out3, int32_t *P,
                      void *stream)
{
    const unsigned grid = (unsigned)std::min<int64_t>(blocks_for(n_pad, 256), 2048);
    hipLaunchKernelGGL(k_reduce, dim3(grid), dim3(256), 0, (hipStream_t)stream, rp, adj, spin, n_pad, cbeg, csz, C,
                       out3, P);
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

int gdi_active_lds_bytes(int32_t n_pad, int32_t C)
{
    return (n_pad / 32) * 4 + (2 * C + 1) * 4;
}

int gdi_launch_sweep_active(const GdiSweepArgs &a, GdiActiveRec *rec, void *stream)
{
    const void *f = (const void *)k_sweep_active;
    const int lds = gdi_active_lds_bytes(a.n_pad, a.C);
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return status(e);
    GdiSweepArgs copy = a;
    void *args[] = {&copy, &rec};
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

int gdi_batch_lds_bytes(int32_t n_pad, int32_t C)
{
    return ((C + 3) & ~3) * 4 + n_pad;
}

int gdi_launch_sweep_batch(const GdiBatchArgs &ba, int grid, int block, int lds_bytes, void *stream)
{
    const void *f = (const void *)k_sweep_batch;
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
    if (e != hipSuccess) return status(e);
    GdiBatchArgs copy = ba;
    void *args[] = {&copy};
    e = hipLaunchKernel(f, dim3(grid), dim3(block), args, (size_t)lds_bytes, (hipStream_t)stream);
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
