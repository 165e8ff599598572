// gdi_device.h -- device helpers shared by the sweep kernels (gdi_kernels.hip,
// gdi_halo.hip): the Philox4x32-10 generator, wave reductions, the per-phase view of
// the magnetisation, the acceptance decision, and agent-scope word access with
// bounded polls. Include after hip_runtime.h and gdi_internal.h.
#pragma once

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

// First sweep of a launch that can start late: t0 with the gate open, else gate_t0.
__device__ __forceinline__ uint32_t launch_begin(const GdiSweepArgs &a)
{
    return gate_open(a) ? a.t0 : a.gate_t0;
}

// Node v sits out sweep t (the proposal's mask, for sweeps before mask_end).
__device__ __forceinline__ bool masked_out(const GdiSweepArgs &a, int32_t v, uint32_t t)
{
    return a.mask && t < a.mask_end && ((a.mask[v >> 5] >> (v & 31)) & 1u);
}

// ------------------------------------------------------------------ words shared between workgroups
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

}  // namespace
