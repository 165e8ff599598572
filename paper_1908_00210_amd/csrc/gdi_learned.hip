// gdi_learned.hip -- kernels of the learned frozen-node proposal (gfx950).
//
// A small network predicts, from six per-node features, whether a node will stay
// frozen for the next sweeps; masked sweeps then skip the nodes it flags, and a
// full sweep runs every k sweeps. The network is 6 -> 64 -> 64 -> 1 with ReLU
// hidden layers and a logistic output, BF16 weights and FP32 accumulation; both
// dense layers of the forward pass run on gfx950's v_mfma_f32_16x16x32_bf16.
//
// The layers are evaluated transposed, hidden x node: for a tile of 16 nodes,
// layer 1 computes H1^T = W1^T X^T and layer 2 H2^T = W2^T H1^T. A 16x16 accumulator
// leaves lane l with rows 4(l/16)..4(l/16)+3 of column l%16. The 16x16x32 product
// pairs element j of lane group g = l/16 in A (row l%16) and in B (column l%16) for
// the same reduction index, and the order of that index is free: so layer 2 takes,
// for K rows 32q..32q+31, the eight values a lane already holds from the two layer-1
// blocks 2q and 2q+1 (rows 32q + 4g + i and 32q + 16 + 4g + i) as its B operand, and
// the matching weights as A. Activations stay in registers between the layers. The
// backward pass keeps the 16x16x16 form, whose operand layout is the accumulator's.
//
// Training computes the mean logistic loss on a minibatch and its gradients
// with the same MFMA layout (dH1 = W2 dPre2 directly in registers; the weight
// gradients, sums over nodes, through per-wave LDS tiles), then Adam updates
// FP32 master weights that are re-packed to BF16.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>

#include "gdi_internal.h"

namespace {

typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ floatx4 mfma16(bf16x4 a, bf16x4 b, floatx4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ floatx4 mfma32(bf16x8 a, bf16x8 b, floatx4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0)
    __builtin_amdgcn_wave_barrier();
}

// ------------------------------------------------------------------ features
// Six features per node (new-id order), rounded to BF16, two zero pads:
//   f0 = degree / 16, f1 = sum |w| / 16, f2 = fraction of neighbours on the other side,
//   f3 = clamp(B s h / T, -16, 16) / 4 (local field in units of T, positive = stable),
//   f4 = min(|4A(1 - s M)| / T, 64) / 16 (balance cost of a flip in units of T),
//   f5 = min(t - last_flip, 255) / 64 (sweeps since the last flip).
// The six features of one node from its row sums (FP32; the callers round them to BF16).
__device__ __forceinline__ void node_features(int32_t deg, int32_t wabs, int32_t other, int32_t h, int32_t s,
                                              int32_t M, float T, int32_t t, int32_t A, int32_t B, int32_t lf,
                                              float f[6])
{
    f[0] = deg / 16.0f;
    f[1] = wabs / 16.0f;
    f[2] = deg ? (float)other / (float)deg : 0.0f;
    f[3] = fminf(fmaxf((float)(B * s * h) / T, -16.0f), 16.0f) / 4.0f;
    const int32_t bal = 4 * A * (1 - s * M);
    f[4] = fminf(fabsf((float)bal) / T, 64.0f) / 16.0f;
    f[5] = (float)min(t - lf, 255) / 64.0f;
}

__global__ void k_features(const int32_t *rp, const int2 *adj, const int8_t *spin, const int32_t *last_flip,
                           int32_t n_pad, const int64_t *state, float T, int32_t t, int32_t A, int32_t B,
                           const int32_t *orig, __bf16 *X, int32_t x_stride_rows, int64_t x_base)
{
    const int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n_pad) return;
    const int32_t o = orig[v];
    if (o < 0) return;  // padding id
    const int32_t s = spin[v];
    const int32_t M = (int32_t)state[0];
    int32_t wabs = 0, other = 0, h = 0;
    const int32_t r0 = rp[v], r1 = rp[v + 1];
    const int32_t deg = r1 - r0;
    // eight entries per round, every load of a round issued before any is used; entries
    // past the row are not loaded and count for nothing
    for (int32_t k = r0; k < r1; k += 8) {
        int2 e[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) e[u] = k + u < r1 ? adj[k + u] : make_int2(v, 0);
        int32_t sj[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) sj[u] = spin[e[u].x];
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (k + u < r1) {
                wabs += e[u].y < 0 ? -e[u].y : e[u].y;
                other += sj[u] != s;
                h += e[u].y * sj[u];
            }
    }
    float f[8];
    node_features(deg, wabs, other, h, s, M, T, t, A, B, last_flip[v], f);
    f[6] = 0.0f;
    f[7] = 0.0f;
    // x_stride_rows < 0: row = new id (inference); otherwise row = x_base + original id (dataset)
    const int64_t row = x_stride_rows < 0 ? (int64_t)v : x_base + o;
    __bf16 *dst = X + row * 8;
#pragma unroll
    for (int i = 0; i < 8; ++i) dst[i] = (__bf16)f[i];
}

// Nodes not flipped since sweep t_cut get label 1 (frozen); original-id rows.
__global__ void k_labels(const int32_t *last_flip, const int32_t *orig, int32_t n_pad, int32_t t_cut,
                         uint8_t *y, int64_t y_base)
{
    const int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n_pad) return;
    const int32_t o = orig[v];
    if (o < 0) return;
    y[y_base + o] = last_flip[v] <= t_cut ? 1 : 0;
}

// Age proposal: skip the real ids that have not flipped for at least k sweeps. A thread
// takes a mask word (32 ids: their last flips and original ids as 16-byte loads), in
// turn over the grid; each workgroup stores its count of skipped nodes in
// part[blockIdx.x] for k_sum_counts (workgroups of 256; n_pad a multiple of 32).
__global__ void __launch_bounds__(256) k_mask_age(const int32_t *last_flip, const int32_t *orig, int32_t n_pad,
                                                   int32_t t, int32_t k, uint32_t *mask, uint32_t *part)
{
    __shared__ uint32_t ws[4];
    const int32_t words = n_pad >> 5;
    uint32_t cnt = 0;
    for (int32_t w = blockIdx.x * blockDim.x + threadIdx.x; w < words; w += gridDim.x * blockDim.x) {
        const int4 *lf4 = reinterpret_cast<const int4 *>(last_flip + (size_t)w * 32);
        const int4 *or4 = reinterpret_cast<const int4 *>(orig + (size_t)w * 32);
        uint32_t bits = 0;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int4 l = lf4[q], o = or4[q];
            const int32_t lv[4] = {l.x, l.y, l.z, l.w}, ov[4] = {o.x, o.y, o.z, o.w};
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (ov[j] >= 0 && t - lv[j] >= k) bits |= 1u << (4 * q + j);
        }
        mask[w] = bits;
        cnt += (uint32_t)__popc(bits);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off, 64);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = ws[0] + ws[1] + ws[2] + ws[3];
}

__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t value)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) p[i] = value;
}

// ------------------------------------------------------------------ MLP parameters
// LDS copy of the parameters. The weight rows are padded (W1 rows to 24 values, W2 rows
// to 72) so that the 16 rows a lane group reads at once fall into distinct LDS banks;
// unpadded 128-byte W2 rows put all of them into one bank.
constexpr int kW1S = 24, kW2S = 72;
struct __align__(16) MlpLds {
    __bf16 w1t[64 * kW1S];
    __bf16 w2t[64 * kW2S];
    float b1[64], b2[64], w3[64], b3, pad[3];
};
static_assert(sizeof(GdiMlpDev) == 11024, "device parameter layout");
static_assert(offsetof(MlpLds, b1) == 64 * (kW1S + kW2S) * 2, "LDS parameter layout");

// Copies the parameters in 16-byte pieces: 128 of W1 (two per row), 512 of W2 (eight per
// row), 49 of the biases and output weights, which follow in the same order in both
// layouts. Workgroups of 256 threads: thread i copies pieces i, i + 256 and i + 512
// (if below 689), all three loads issued before the stores.
__device__ __forceinline__ int param_piece_offset(int c)
{
    if (c < 128) return (c >> 1) * kW1S * 2 + (c & 1) * 16;
    if (c < 640) return (int)offsetof(MlpLds, w2t) + ((c - 128) >> 3) * kW2S * 2 + ((c - 128) & 7) * 16;
    return (int)offsetof(MlpLds, b1) + (c - 640) * 16;
}

__device__ void load_params(const GdiMlpDev *p, MlpLds *m)
{
    constexpr int kPieces = 128 + 512 + 49;
    const uint4 *src = reinterpret_cast<const uint4 *>(p);
    char *dst = reinterpret_cast<char *>(m);
    const int c0 = threadIdx.x, c1 = c0 + 256, c2 = c0 + 512;
    const uint4 v0 = src[c0], v1 = src[c1];
    const uint4 v2 = c2 < kPieces ? src[c2] : uint4{0u, 0u, 0u, 0u};
    *reinterpret_cast<uint4 *>(dst + param_piece_offset(c0)) = v0;
    *reinterpret_cast<uint4 *>(dst + param_piece_offset(c1)) = v1;
    if (c2 < kPieces) *reinterpret_cast<uint4 *>(dst + param_piece_offset(c2)) = v2;
    __syncthreads();
}

// Forward pass of one 16-node tile. Lane l: g = l/16 (row group), r = l%16 (node).
// xb: B operand of layer 1 (features 4g..4g+3 of node r). Outputs the H1 B operands,
// the layer-2 pre-activations and the logit (identical in the four lanes of a node).
struct TileFwd {
    bf16x4 h1[4];      // H1^T rows 16m + 4g + i, node r (BF16, post-ReLU)
    floatx4 pre2[4];   // layer-2 pre-activations rows 16m + 4g + i
    float z;
};

__device__ __forceinline__ void tile_forward(const MlpLds *m, bf16x4 xb, int g, int r, TileFwd &o)
{
    // layer 1 (K = 6 features, padded): lane group 0 carries features 0..7 of its node
    // (xb holds features 4g..4g+3 for g < 2), the other groups zeros
    bf16x8 x8;
    {
        const __bf16 z = (__bf16)0.0f;
        const bf16x4 hi = __builtin_bit_cast(bf16x4, __shfl_down(__builtin_bit_cast(uint64_t, xb), 16, 64));
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            x8[j] = g == 0 ? xb[j] : z;
            x8[4 + j] = g == 0 ? hi[j] : z;
        }
    }
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) {
        // one 16-byte read of row 16 mb + r (rows are 48 bytes apart), zero for g > 0
        bf16x8 a = *reinterpret_cast<const bf16x8 *>(&m->w1t[(16 * mb + r) * kW1S]);
        if (g != 0) a = bf16x8{};
        const floatx4 acc = mfma32(a, x8, floatx4{0.f, 0.f, 0.f, 0.f});
#pragma unroll
        for (int i = 0; i < 4; ++i) o.h1[mb][i] = (__bf16)fmaxf(acc[i] + m->b1[16 * mb + 4 * g + i], 0.0f);
    }
    float part = 0.0f;
#pragma unroll
    for (int mo = 0; mo < 4; ++mo) {
        floatx4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            // two 8-byte reads (row offsets are multiples of four values)
            const __bf16 *row = &m->w2t[(16 * mo + r) * kW2S + 32 * q + 4 * g];
            const bf16x4 alo = *reinterpret_cast<const bf16x4 *>(row);
            const bf16x4 ahi = *reinterpret_cast<const bf16x4 *>(row + 16);
            bf16x8 a, b;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                a[j] = alo[j];
                a[4 + j] = ahi[j];
                b[j] = o.h1[2 * q][j];
                b[4 + j] = o.h1[2 * q + 1][j];
            }
            acc = mfma32(a, b, acc);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int hrow = 16 * mo + 4 * g + i;
            acc[i] += m->b2[hrow];
            part += m->w3[hrow] * fmaxf(acc[i], 0.0f);
        }
        o.pre2[mo] = acc;
    }
    part += __shfl_xor(part, 16, 64);
    part += __shfl_xor(part, 32, 64);
    o.z = part + m->b3;
}

__device__ __forceinline__ bf16x4 load_xb(const __bf16 *X, const int32_t *idx, int64_t node, int64_t count, int g)
{
    bf16x4 xb;
    const bool ok = node < count && g < 2;
    const int64_t row = ok ? (idx ? (int64_t)idx[node] : node) : 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) xb[j] = ok ? X[row * 8 + 4 * g + j] : (__bf16)0.0f;
    return xb;
}

// ------------------------------------------------------------------ inference
// Logit per node; mask bit = logit > thr_logit (32 nodes per mask word).
__global__ void __launch_bounds__(256) k_mlp_infer(const __bf16 *X, int32_t count, const GdiMlpDev *p,
                                                    float thr_logit, uint32_t *mask, float *logits)
{
    __shared__ MlpLds m;
    load_params(p, &m);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, r = lane & 15;
    const int64_t words = ((int64_t)count + 31) / 32;
    for (int64_t w = (int64_t)blockIdx.x * 4 + wave; w < words; w += (int64_t)gridDim.x * 4) {
        uint32_t bits = 0;
#pragma unroll
        for (int half = 0; half < 2; ++half) {
            const int64_t node = w * 32 + 16 * half + r;
            TileFwd f;
            tile_forward(&m, load_xb(X, nullptr, node, count, g), g, r, f);
            const bool frozen = g == 0 && node < count && f.z > thr_logit;
            if (g == 0 && node < count && logits) logits[node] = f.z;
            const uint64_t b = __ballot(frozen);
            bits |= (uint32_t)(b & 0xFFFFu) << (16 * half);
            __builtin_amdgcn_sched_barrier(0);  // one tile at a time (register use)
        }
        if (lane == 0 && mask) mask[w] = bits;
    }
}

// Per-node values a row scan starts from: original id, spin, row bounds, last flip.
struct NodeHead {
    int32_t o, s, r0, r1, lf;
};

__device__ __forceinline__ NodeHead load_head(const int32_t *rp, const int8_t *spin, const int32_t *last_flip,
                                              const int32_t *orig, int32_t n_pad, int32_t v)
{
    NodeHead x{-1, 0, 0, 0, 0};
    if (v < n_pad) {
        x.o = orig[v];
        x.s = spin[v];
        x.r0 = rp[v];
        x.r1 = rp[v + 1];
        x.lf = last_flip[v];
    }
    return x;
}

// The proposal's mask for one block in one pass (what k_features, k_mlp_infer and
// k_mask_finish compute in turn, without the feature rows in memory). A wave takes a
// mask word, two 16-node tiles: the four lanes of a node (r, r + 16, r + 32, r + 48)
// split both tiles' row scans, which run in one loop so that their loads overlap, and
// then hold the node's features for the tile's network. The next word's row bounds are
// loaded before the network runs. The mask bit is set for real ids whose logit exceeds
// thr_logit; each workgroup stores its count of skipped nodes in part[blockIdx.x]
// (k_sum_counts adds them up: atomics on one shared counter from every workgroup cost
// about as much as the rest of the kernel).
__global__ void __launch_bounds__(256) k_mlp_mask(const int32_t *rp, const int2 *adj, const int8_t *spin,
                                                   const int32_t *last_flip, int32_t n_pad, const int64_t *state,
                                                   float T, int32_t t, int32_t A, int32_t B, const int32_t *orig,
                                                   const GdiMlpDev *p, float thr_logit, uint32_t *mask, uint32_t *part)
{
    __shared__ MlpLds m;
    __shared__ uint32_t cnt_s[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, r = lane & 15;
    const int64_t words = ((int64_t)n_pad + 31) / 32;
    const int64_t stride = (int64_t)gridDim.x * 4;
    int64_t w = (int64_t)blockIdx.x * 4 + wave;
    NodeHead hd[2];
#pragma unroll
    for (int hf = 0; hf < 2; ++hf)
        hd[hf] = load_head(rp, spin, last_flip, orig, n_pad, (int32_t)(w * 32 + 16 * hf + r));
    load_params(p, &m);
    const int32_t M = (int32_t)state[0];
    uint32_t cnt = 0;
    for (; w < words; w += stride) {
        // this lane's entries g, g + 4, ... of both rows, four per row and round (a row of
        // up to 16 entries in one round), every load of a round issued before any is used
        int32_t wabs[2] = {0, 0}, other[2] = {0, 0}, h[2] = {0, 0};
        const int32_t deg0 = hd[0].r1 - hd[0].r0, deg1 = hd[1].r1 - hd[1].r0;
        const int32_t dmax = max(deg0, deg1);
        for (int32_t j = g; j < dmax; j += 16) {
            int2 e[2][4];
            int32_t sj[2][4];
#pragma unroll
            for (int hf = 0; hf < 2; ++hf)
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    e[hf][u] = j + 4 * u < hd[hf].r1 - hd[hf].r0 ? adj[hd[hf].r0 + j + 4 * u] : make_int2(0, 0);
#pragma unroll
            for (int hf = 0; hf < 2; ++hf)
#pragma unroll
                for (int u = 0; u < 4; ++u) sj[hf][u] = spin[e[hf][u].x];
#pragma unroll
            for (int hf = 0; hf < 2; ++hf)
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    if (j + 4 * u < hd[hf].r1 - hd[hf].r0) {
                        wabs[hf] += e[hf][u].y < 0 ? -e[hf][u].y : e[hf][u].y;
                        other[hf] += sj[hf][u] != hd[hf].s;
                        h[hf] += e[hf][u].y * sj[hf][u];
                    }
        }
        bf16x4 xb[2];
        bool real[2];
#pragma unroll
        for (int hf = 0; hf < 2; ++hf) {
#pragma unroll
            for (int off = 16; off < 64; off <<= 1) {
                wabs[hf] += __shfl_xor(wabs[hf], off, 64);
                other[hf] += __shfl_xor(other[hf], off, 64);
                h[hf] += __shfl_xor(h[hf], off, 64);
            }
            float f[6];
            node_features(hd[hf].r1 - hd[hf].r0, wabs[hf], other[hf], h[hf], hd[hf].s, M, T, t, A, B, hd[hf].lf, f);
            real[hf] = hd[hf].o >= 0;
            // B operand of layer 1: features 4g .. 4g + 3 (zero past feature 5 and for padding);
            // constant indices into f, so that it stays in registers
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) {
                const float fv = g == 0 ? f[jj] : (jj < 2 ? f[4 + (jj & 1)] : 0.0f);
                xb[hf][jj] = (real[hf] && g < 2) ? (__bf16)fv : (__bf16)0.0f;
            }
        }
        const int64_t wn = w + stride;
        if (wn < words) {
#pragma unroll
            for (int hf = 0; hf < 2; ++hf)
                hd[hf] = load_head(rp, spin, last_flip, orig, n_pad, (int32_t)(wn * 32 + 16 * hf + r));
        }
        uint32_t bits = 0;
#pragma unroll
        for (int hf = 0; hf < 2; ++hf) {
            TileFwd tf;
            tile_forward(&m, xb[hf], g, r, tf);
            const uint64_t b = __ballot(g == 0 && real[hf] && tf.z > thr_logit);
            bits |= (uint32_t)(b & 0xFFFFu) << (16 * hf);
            // one tile at a time: interleaving the two tiles' products would double the
            // live registers and halve the waves per SIMD
            __builtin_amdgcn_sched_barrier(0);
        }
        if (lane == 0) {
            mask[w] = bits;
            cnt += (uint32_t)__popc(bits);
        }
    }
    if (lane == 0) cnt_s[wave] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = cnt_s[0] + cnt_s[1] + cnt_s[2] + cnt_s[3];
}

// One workgroup of 256: the skipped nodes of a block (sum of the nparts workgroup counts,
// below 2^31) go to block_skips, and times weight are added to skipped.
__global__ void __launch_bounds__(256) k_sum_counts(const uint32_t *part, int32_t nparts, uint32_t weight,
                                                     unsigned long long *skipped, unsigned long long *block_skips)
{
    __shared__ uint32_t ws[4];
    uint32_t c = 0;
    for (int i = threadIdx.x; i < nparts; i += 256) c += part[i];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned long long tot = (unsigned long long)ws[0] + ws[1] + ws[2] + ws[3];
        *skipped += tot * weight;
        *block_skips = tot;
    }
}

// ------------------------------------------------------------------ gradients
// Mean logistic loss over the minibatch rows idx[0..count) and its gradient with
// respect to the packed FP32 parameters (layout of gdi_mlp_weights: w1[64][6], b1,
// w2[64][64], b2, w3, b3). Every wave writes its own sums over its tiles, all
// GDI_MLP_PARAMS of them and its loss sum after them, to row blockIdx.x * 4 + wave of
// part (rows of kGradStride floats); k_grad_sum adds the rows up in row order. No
// atomics: the gradient is the same bits on every run (a float atomic sum is not), and
// a quarter of a million atomic adds on 4673 words cost more than the products.
struct WaveTiles {
    __bf16 dp2[64 * 16];  // dPre2^T [o][node]
    __bf16 h1[64 * 16];   // H1^T [k][node]
    __bf16 dp1[64 * 16];  // dPre1^T [k][node]
    __bf16 xt[16 * 16];   // X^T [f][node]
};

__device__ __forceinline__ bf16x4 lds4(const __bf16 *base)
{
    bf16x4 v;
#pragma unroll
    for (int j = 0; j < 4; ++j) v[j] = base[j];
    return v;
}

constexpr int kGradStride = (GDI_MLP_PARAMS + 1 + 3) & ~3;
constexpr int64_t kGradBlocks = 128;  // at most 512 partial rows (9.6 MB)

__global__ void __launch_bounds__(256) k_mlp_grad(const __bf16 *X, const uint8_t *Y, const int32_t *idx,
                                                   int32_t count, const GdiMlpDev *p, float inv_batch, float *part)
{
    __shared__ MlpLds m;
    __shared__ WaveTiles tiles[4];
    load_params(p, &m);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, r = lane & 15;
    WaveTiles &T = tiles[wave];

    floatx4 acc_w2[4][4];
    floatx4 acc_w1[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        acc_w1[a] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int b = 0; b < 4; ++b) acc_w2[a][b] = floatx4{0.f, 0.f, 0.f, 0.f};
    }
    float gb1[4][4], gb2[4][4], gw3[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) gb1[a][b] = gb2[a][b] = gw3[a][b] = 0.0f;
    float gb3 = 0.0f, lsum = 0.0f;

    const int64_t tiles_n = ((int64_t)count + 15) / 16;
    for (int64_t tile = (int64_t)blockIdx.x * 4 + wave; tile < tiles_n; tile += (int64_t)gridDim.x * 4) {
        const int64_t node = tile * 16 + r;
        const bool valid = node < count;
        const bf16x4 xb = load_xb(X, idx, node, count, g);
        TileFwd f;
        tile_forward(&m, xb, g, r, f);
        const float y = valid ? (float)Y[idx ? idx[node] : node] : 0.0f;
        const float pz = 1.0f / (1.0f + expf(-f.z));
        const float dz = valid ? (pz - y) * inv_batch : 0.0f;
        if (valid && g == 0) {
            // numerically stable logistic loss: softplus(z) - y z
            const float sp = fmaxf(f.z, 0.0f) + log1pf(expf(-fabsf(f.z)));
            lsum += sp - y * f.z;
            gb3 += dz;
        }
        // layer 2 backward: dPre2 = dz w3 [pre2 > 0]
        bf16x4 dp2b[4];
#pragma unroll
        for (int mo = 0; mo < 4; ++mo) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int hrow = 16 * mo + 4 * g + i;
                const float pre = f.pre2[mo][i];
                const float h2 = fmaxf(pre, 0.0f);
                gw3[mo][i] += dz * h2;
                const float d = pre > 0.0f ? dz * m.w3[hrow] : 0.0f;
                gb2[mo][i] += d;
                dp2b[mo][i] = (__bf16)d;
                T.dp2[hrow * 16 + r] = dp2b[mo][i];
                T.h1[(16 * mo + 4 * g + i) * 16 + r] = f.h1[mo][i];
            }
        }
        // dH1^T = W2 dPre2^T: A[k][o] = w2t[o][k]
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) {
            floatx4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int mo = 0; mo < 4; ++mo) {
                bf16x4 a;
#pragma unroll
                for (int j = 0; j < 4; ++j) a[j] = m.w2t[(16 * mo + 4 * g + j) * kW2S + 16 * kb + r];
                acc = mfma16(a, dp2b[mo], acc);
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int krow = 16 * kb + 4 * g + i;
                const float d = (float)f.h1[kb][i] > 0.0f ? acc[i] : 0.0f;
                gb1[kb][i] += d;
                T.dp1[krow * 16 + r] = (__bf16)d;
            }
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            // X^T tile: feature 4g + j of node r (features >= 8 are zero)
            T.xt[(4 * g + j) * 16 + r] = g < 2 ? xb[j] : (__bf16)0.0f;
        }
        wave_lds_sync();
        // dW2^T[o][k] += sum_node dPre2^T[o][node] H1^T[k][node]
#pragma unroll
        for (int mo = 0; mo < 4; ++mo) {
            const bf16x4 a = lds4(&T.dp2[(16 * mo + r) * 16 + 4 * g]);
#pragma unroll
            for (int kb = 0; kb < 4; ++kb) acc_w2[mo][kb] = mfma16(a, lds4(&T.h1[(16 * kb + r) * 16 + 4 * g]), acc_w2[mo][kb]);
        }
        // dW1^T[k][f] += sum_node dPre1^T[k][node] X^T[f][node]
        const bf16x4 bx = lds4(&T.xt[r * 16 + 4 * g]);
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) acc_w1[kb] = mfma16(lds4(&T.dp1[(16 * kb + r) * 16 + 4 * g]), bx, acc_w1[kb]);
        wave_lds_sync();
    }
    // flush: D layout row = 16a + 4g + i, column = 16b + r
    float *row = part + (size_t)(blockIdx.x * 4 + wave) * kGradStride;
    float *gw1 = row, *gb1p = row + 64 * 6, *gw2 = gb1p + 64, *gb2p = gw2 + 64 * 64, *gw3p = gb2p + 64,
          *gb3p = gw3p + 64;
#pragma unroll
    for (int mo = 0; mo < 4; ++mo)
#pragma unroll
        for (int kb = 0; kb < 4; ++kb)
#pragma unroll
            for (int i = 0; i < 4; ++i) gw2[(16 * mo + 4 * g + i) * 64 + 16 * kb + r] = acc_w2[mo][kb][i];
#pragma unroll
    for (int kb = 0; kb < 4; ++kb)
#pragma unroll
        for (int i = 0; i < 4; ++i)
            if (r < 6) gw1[(16 * kb + 4 * g + i) * 6 + r] = acc_w1[kb][i];
    // per-hidden-unit sums over nodes: reduce the 16 node lanes of each row group
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            float v1 = gb1[a][i], v2 = gb2[a][i], v3 = gw3[a][i];
#pragma unroll
            for (int off = 1; off < 16; off <<= 1) {
                v1 += __shfl_xor(v1, off, 64);
                v2 += __shfl_xor(v2, off, 64);
                v3 += __shfl_xor(v3, off, 64);
            }
            if (r == 0) {
                const int hrow = 16 * a + 4 * g + i;
                gb1p[hrow] = v1;
                gb2p[hrow] = v2;
                gw3p[hrow] = v3;
            }
        }
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        gb3 += __shfl_xor(gb3, off, 64);
        lsum += __shfl_xor(lsum, off, 64);
    }
    if (lane == 0) {
        gb3p[0] = gb3;
        row[GDI_MLP_PARAMS] = lsum;
    }
}

// grad[i] = sum over the rows of part[row][i] for i < GDI_MLP_PARAMS; the rows' loss
// sums are added to *loss. Workgroups of 1024: 64 columns, 16 slices of rows (slice s
// sums rows s, s + 16, ... in order), then the 16 slice sums in order: a fixed order,
// with 16 loads in flight per column.
__global__ void __launch_bounds__(1024) k_grad_sum(const float *part, int32_t rows, float *grad, float *loss)
{
    __shared__ float red[16][64];
    const int pi = threadIdx.x & 63, sl = threadIdx.x >> 6;
    const int32_t i = blockIdx.x * 64 + pi;
    float acc = 0.0f;
    if (i <= GDI_MLP_PARAMS)
        for (int32_t w = sl; w < rows; w += 16) acc += part[(size_t)w * kGradStride + i];
    red[sl][pi] = acc;
    __syncthreads();
    if (sl == 0 && i <= GDI_MLP_PARAMS) {
        float t = 0.0f;
#pragma unroll
        for (int k = 0; k < 16; ++k) t += red[k][pi];
        if (i < GDI_MLP_PARAMS) grad[i] = t;
        else if (loss) *loss += t;
    }
}

// ------------------------------------------------------------------ optimiser
// Adam on the FP32 master parameters, then repack the BF16 device weights.
__global__ void k_adam(float *w, const float *gr, float *mo, float *ve, int32_t P, float lr, float b1, float b2,
                       float eps, float bc1, float bc2)
{
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P) return;
    const float gi = gr[i];
    const float m1 = b1 * mo[i] + (1.0f - b1) * gi;
    const float v1 = b2 * ve[i] + (1.0f - b2) * gi * gi;
    mo[i] = m1;
    ve[i] = v1;
    w[i] -= lr * (m1 / bc1) / (sqrtf(v1 / bc2) + eps);
}

__global__ void k_mlp_pack(const float *w, GdiMlpDev *p)
{
    const float *w1 = w, *b1 = w + 64 * 6, *w2 = b1 + 64, *b2 = w2 + 64 * 64, *w3 = b2 + 64, *b3 = w3 + 64;
    for (int i = threadIdx.x; i < 64 * 16; i += blockDim.x) {
        const int h = i / 16, f = i % 16;
        p->w1t[i] = (__bf16)(f < 6 ? w1[h * 6 + f] : 0.0f);
    }
    for (int i = threadIdx.x; i < 64 * 64; i += blockDim.x) p->w2t[i] = (__bf16)w2[i];
    for (int i = threadIdx.x; i < 64; i += blockDim.x) {
        p->b1[i] = b1[i];
        p->b2[i] = b2[i];
        p->w3[i] = w3[i];
    }
    if (threadIdx.x == 0) p->b3 = b3[0];
}

inline unsigned nblk(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

int gdi_launch_features(const int32_t *rp, const int2 *adj, const int8_t *spin, const int32_t *last_flip,
                        int32_t n_pad, const int64_t *state, float T, int32_t t, int32_t A, int32_t B,
                        const int32_t *orig, void *X, int32_t dataset_rows, int64_t x_base, void *stream)
{
    hipLaunchKernelGGL(k_features, dim3(nblk(n_pad, 256)), dim3(256), 0, (hipStream_t)stream, rp, adj, spin,
                       last_flip, n_pad, state, T, t, A, B, orig, (__bf16 *)X, dataset_rows, x_base);
    return (int)hipGetLastError();
}

int gdi_launch_labels(const int32_t *last_flip, const int32_t *orig, int32_t n_pad, int32_t t_cut, uint8_t *y,
                      int64_t y_base, void *stream)
{
    hipLaunchKernelGGL(k_labels, dim3(nblk(n_pad, 256)), dim3(256), 0, (hipStream_t)stream, last_flip, orig, n_pad,
                       t_cut, y, y_base);
    return (int)hipGetLastError();
}

int gdi_launch_mask_age(const int32_t *last_flip, const int32_t *orig, int32_t n_pad, int32_t t, int32_t k,
                        uint32_t *mask, uint32_t *part, int32_t part_cap, uint64_t *skipped, uint32_t weight,
                        uint64_t *block_skips, void *stream)
{
    if (part_cap < 1 || (n_pad & 31) || (reinterpret_cast<uintptr_t>(last_flip) & 15) ||
        (reinterpret_cast<uintptr_t>(orig) & 15))
        return (int)hipErrorInvalidValue;
    const int64_t words = n_pad / 32;
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>((words + 255) / 256, part_cap));
    hipLaunchKernelGGL(k_mask_age, dim3(grid), dim3(256), 0, (hipStream_t)stream, last_flip, orig, n_pad, t, k, mask,
                       part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return (int)e;
    hipLaunchKernelGGL(k_sum_counts, dim3(1), dim3(256), 0, (hipStream_t)stream, part, (int32_t)grid, weight,
                       (unsigned long long *)skipped, (unsigned long long *)block_skips);
    return (int)hipGetLastError();
}

int gdi_launch_fill_i32(int32_t *p, int64_t n, int32_t value, void *stream)
{
    if (n <= 0) return 0;
    hipLaunchKernelGGL(k_fill_i32, dim3(nblk(n, 256)), dim3(256), 0, (hipStream_t)stream, p, n, value);
    return (int)hipGetLastError();
}

int gdi_launch_mlp_infer(const void *X, int32_t count, const GdiMlpDev *p, float thr_logit, uint32_t *mask,
                         float *logits, void *stream)
{
    const int64_t words = ((int64_t)count + 31) / 32;
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>((words + 3) / 4, 4096));
    hipLaunchKernelGGL(k_mlp_infer, dim3(grid), dim3(256), 0, (hipStream_t)stream, (const __bf16 *)X, count, p,
                       thr_logit, mask, logits);
    return (int)hipGetLastError();
}

int gdi_launch_mlp_mask(const int32_t *rp, const int2 *adj, const int8_t *spin, const int32_t *last_flip,
                        int32_t n_pad, const int64_t *state, float T, int32_t t, int32_t A, int32_t B,
                        const int32_t *orig, const GdiMlpDev *p, float thr_logit, uint32_t *mask, uint32_t *part,
                        int32_t part_cap, uint64_t *skipped, uint32_t weight, uint64_t *block_skips, void *stream)
{
    if (part_cap < 1) return (int)hipErrorInvalidValue;
    const int64_t words = ((int64_t)n_pad + 31) / 32;
    // no more workgroups than fit on the device at once: the parameters are copied to LDS
    // once per workgroup, and a wave takes further words in turn
    static const int64_t resident = [] {
        int dev = 0, cus = 0, per_cu = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_mlp_mask, 256, 0) != hipSuccess)
            return (int64_t)1024;
        return (int64_t)std::max(1, cus) * std::max(1, per_cu);
    }();
    const unsigned grid =
        (unsigned)std::max<int64_t>(1, std::min<int64_t>(std::min<int64_t>((words + 3) / 4, resident), part_cap));
    hipLaunchKernelGGL(k_mlp_mask, dim3(grid), dim3(256), 0, (hipStream_t)stream, rp, adj, spin, last_flip, n_pad,
                       state, T, t, A, B, orig, p, thr_logit, mask, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return (int)e;
    hipLaunchKernelGGL(k_sum_counts, dim3(1), dim3(256), 0, (hipStream_t)stream, part, (int32_t)grid, weight,
                       (unsigned long long *)skipped, (unsigned long long *)block_skips);
    return (int)hipGetLastError();
}

int gdi_mlp_grad_part_floats(int32_t count)
{
    const int64_t tiles = ((int64_t)count + 15) / 16;
    const int64_t grid = std::max<int64_t>(1, std::min<int64_t>((tiles + 3) / 4, kGradBlocks));
    return (int)(grid * 4 * kGradStride);
}

int gdi_launch_mlp_grad(const void *X, const uint8_t *Y, const int32_t *idx, int32_t count, const GdiMlpDev *p,
                        float inv_batch, float *part, float *grad, float *loss, void *stream)
{
    if (count < 1) return (int)hipErrorInvalidValue;
    const int64_t tiles = ((int64_t)count + 15) / 16;
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>((tiles + 3) / 4, kGradBlocks));
    hipLaunchKernelGGL(k_mlp_grad, dim3(grid), dim3(256), 0, (hipStream_t)stream, (const __bf16 *)X, Y, idx, count,
                       p, inv_batch, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return (int)e;
    hipLaunchKernelGGL(k_grad_sum, dim3((GDI_MLP_PARAMS + 1 + 63) / 64), dim3(1024), 0, (hipStream_t)stream, part,
                       (int32_t)(grid * 4), grad, loss);
    return (int)hipGetLastError();
}

int gdi_launch_adam(float *w, const float *g, float *m, float *v, int32_t P, float lr, float b1, float b2, float eps,
                    float bc1, float bc2, void *stream)
{
    hipLaunchKernelGGL(k_adam, dim3(nblk(P, 256)), dim3(256), 0, (hipStream_t)stream, w, g, m, v, P, lr, b1, b2, eps,
                       bc1, bc2);
    return (int)hipGetLastError();
}

int gdi_launch_mlp_pack(const float *w, GdiMlpDev *p, void *stream)
{
    hipLaunchKernelGGL(k_mlp_pack, dim3(1), dim3(256), 0, (hipStream_t)stream, w, p);
    return (int)hipGetLastError();
}
