// gdi_internal.h -- structures shared by the host library and the gfx950 kernels.
//
// Device layout of one graph (colour-major relabelling, built by gdi_create):
//   new ids: class c occupies [cbeg[c], cbeg[c] + csz[c]); cbeg[c] is a multiple of
//            GDI_CLASS_ALIGN, ids in the gaps are padding nodes with empty rows
//   rp      int32 [n_pad + 1]   row pointers over new ids
//   adj     int2  [nnz]         {new column id, weight}, interleaved so one 8-byte
//                               load fetches a whole CSR entry
//   orig    int32 [n_pad]       original id of each new id (-1 for padding); the
//                               Philox counter uses the original id
//   spin    int8  [n_pad]       +1 / -1 (0 for padding)
#pragma once

#include <stdint.h>

#include "gdi_layout.h"  // GDI_CLASS_ALIGN, halo constants, GdiHaloEntry

#define GDI_MAX_BLOCK 1024
#define GDI_WG_THR_MAX 256     // largest table width the workgroup sweep keeps in LDS (two rows)
#define GDI_BAR_GROUPS 8       // workgroups are grouped by blockIdx % 8 for the two-level barrier
#define GDI_BAR_PAD 16         // uint64 words between group counters (128 bytes)

struct GdiSweepArgs {
    const int32_t *rp;
    const int2 *adj;
    const int32_t *orig;
    int8_t *spin;
    const int32_t *cbeg;       // C class starts (device)
    const int32_t *csz;        // C class sizes (device)
    const uint32_t *thr;       // S rows of (K+1) thresholds, indexed by absolute sweep
    int64_t *state;            // [0] M, [1] cut delta accumulator, [2] flips, [3] error flag
    int32_t *P;                // C counts of +1 spins per class
    int64_t *trace_m;          // S entries or null
    int64_t *trace_dcut;       // S entries or null (per-sweep cut change, accumulated by atomics)
    uint64_t *bar_grp;         // phases * GDI_BAR_GROUPS * GDI_BAR_PAD
    uint64_t *bar_glob;        // phases * GDI_BAR_PAD
    int32_t n;                 // real nodes
    int32_t n_pad;
    int32_t C;
    int32_t K;                 // table width: thresholds exist for 1 <= dE <= K
    uint32_t t0;               // first sweep
    uint32_t S;                // one past the last sweep
    int32_t A4;                // 4*A
    int32_t B;
    uint32_t key0, key1;       // Philox key
    uint32_t replica;
    uint32_t snapshot;         // 1 = SNAPSHOT balance mode
    uint32_t rule;             // 0 = Metropolis, 1 = the paper's argmin + random flip (row entry 0 = P_f threshold)
    int64_t spin_limit;        // bounded waits: polls before giving up
    const uint32_t *mask;      // n_pad/32 words, bit set = node skipped in this launch, or null
    int32_t *last_flip;        // n_pad entries: sweep of each node's last flip, or null
    // launch gate (null = always run): with k = n - *skip_count nodes active, the launch
    // runs iff (k <= active_max) == (gate_small != 0); the decision is uniform over the grid
    const unsigned long long *skip_count;
    int32_t active_max;
    int32_t gate_small;
    // a launch whose gate is closed starts at sweep gate_t0 instead of t0 (gate_t0 >= S: it
    // does nothing); the mask applies to sweeps t < mask_end only (the grid sweep uses both
    // to run one block's masked sweeps and the next block's full sweep in one launch)
    uint32_t gate_t0;
    uint32_t mask_end;
};

// Record of one active node of a masked launch (k_sweep_active).
struct GdiActiveRec {
    int32_t v;                 // new id
    int32_t r0, r1;            // CSR row
    int32_t orig;              // original id (Philox counter)
};

struct GdiHaloArgs {
    GdiSweepArgs base;
    // CSR with each entry packed into 32 bits: (LDS word in the owner's image << 16) |
    // ((weight & 0x7FF) << 5) | bit in that word, weights in [-1024, 1023]; followed by
    // GDI_HALO_PF zero entries, so that GDI_HALO_PF entries can be read from any row start
    const uint32_t *adjL;
    int32_t unit_w;            // 1: every weight is 1
    const GdiHaloEntry *tab;   // grid x C entries
    uint64_t *words;           // packed spins: (epoch << 32) | 32 spin bits (bit = 1 for +1)
    uint64_t *member;          // 8 x 64 words: workgroup b posts (epoch << 32) | uint32(dM) at (b % 8) * 64 + b / 8
    uint64_t *group;           // 2 x 8 words (phase parity x group), GDI_HALO_GROUP_PAD apart
    int32_t lds_words;         // LDS words per workgroup: image (own and foreign words per class), the tail's gather and tail regions, the foreign-id lists
    int32_t thr_in_lds;        // 1: the current and next threshold rows are staged in LDS
    // epochs of this launch start above epoch0: words left by earlier launches carry
    // smaller ones, so the words need no clearing between launches
    uint32_t epoch0;
    // Redundant tail: the last classes T0..C-1 hold at most one node per worker thread
    // in total; every workgroup runs them itself (identical results everywhere), so
    // they take no grid-wide barrier. Tail spins live in a tail region of LDS (ids
    // [cbeg[T0], n_pad)); the neighbours of tail nodes in classes < T0 are gathered
    // into a gather region after their class's phase. T0 == C: no tail.
    int32_t T0;
    int32_t tail_n;            // tail nodes (<= worker threads)
    int32_t gather_off;        // LDS word of the gather region
    int32_t tail_off;          // LDS word of the tail region
    const int32_t *tail_v;     // tail_n new ids, in class order
    const int32_t *tail_beg;   // C - T0 + 1 offsets into tail_v per tail class
    const int32_t *gat_words;  // packed-word ids gathered for the tail, by source class
    const int32_t *gat_beg;    // T0 + 1 offsets into gat_words
    // the tail's CSR, copied into LDS at trp_off (tail_n + 1 row offsets) and tent_off
    // (tail_nnz packed entries); thread i of the tail owns tail_v[i]
    int32_t tail_nnz;
    int32_t trp_off, tent_off;
    const int32_t *tail_rp;
    const uint32_t *tail_ent;
    // Rows longer than GDI_HALO_PF (when ovf_len > 0): their entries from GDI_HALO_PF - 1
    // on sit in an overflow region of the owner workgroup's LDS image (ovf_len words at
    // ovf_off, copied from ovf + b * ovf_len at launch), and the row's entry GDI_HALO_PF - 1
    // holds the LDS word where they start. With ovf_len == 0 they are read from adjL.
    int32_t ovf_off, ovf_len;
    const uint32_t *ovf;
    // Foreign-word ids: workgroup b's lists for all classes, flist_len entries at
    // flist + b * flist_len, copied into LDS at list_off at launch (GdiHaloEntry.list_off
    // points into that copy).
    int32_t list_off, flist_len;
    const int32_t *flist;
};

// Batched form: one instance (graph, replica) per queue entry.
struct GdiBatchInstance {
    const int32_t *rp;
    const int2 *adj;
    const int32_t *orig;
    const int32_t *cbeg;
    const int32_t *csz;
    int8_t *out;               // n spins in original order (device) or null
    int64_t *result;           // [0] final M, [1] tracked weighted cut
    int32_t n, n_pad, C, lanes;
    uint32_t replica;
    uint32_t wide;             // 1: long rows for `lanes` (eight entries per lane and round)
    // cluster: the instance runs on `members` workgroups, this entry is member `rank`;
    // sync holds its epoch-tagged spin words (n_pad / 32 + 1) and two parities x 16 dM
    // slots, zeroed before the launch (members == 1: no cluster, sync unused)
    uint64_t *sync;
    int32_t members, rank;
};

struct GdiBatchArgs {
    const GdiBatchInstance *inst;  // queue order
    int32_t *queue;                // next instance to take (zeroed before launch)
    const uint32_t *thr;           // S rows of (K+1) thresholds
    int32_t n_inst;
    int32_t K;
    uint32_t S;
    int32_t A4, B;
    uint32_t key0, key1;
    uint32_t snapshot;
    uint32_t rule;                 // acceptance rule, as in GdiSweepArgs
    int64_t *error;                // set to 1 when a cluster's bounded wait expires
    int64_t spin_limit;            // polls before such a wait gives up
};
#define GDI_BATCH_MAX_MEMBERS 16

// Learned proposal: BF16 network parameters on the device (transposed weights).
struct GdiMlpDev {
    __bf16 w1t[64 * 16];       // [hidden][feature], features 6..15 zero
    __bf16 w2t[64 * 64];       // [output hidden][input hidden]
    float b1[64], b2[64], w3[64], b3, pad[3];
};
#define GDI_MLP_PARAMS (64 * 6 + 64 + 64 * 64 + 64 + 64 + 1)  // packed FP32 master parameters

// Allocation-free cut (gdi_cut_dev_noalloc): fixed per-GPU scratch array.
#define GDI_NOALLOC_SCRATCH_BYTES ((size_t)16 << 20)  // 16 MiB per GPU
#define GDI_NOALLOC_MAX_C 4094                         // colour classes
#define GDI_NOALLOC_SPIN_OFF 16640                     // 256 + 4 (GDI_NOALLOC_MAX_C + 2), 256-aligned
// then the relabelled spins (n_pad bytes, 256-aligned) and their bit-packed copy (n_pad / 8
// bytes): n_pad + n_pad / 8 must fit in the 16,760,064 bytes after the accumulators and
// the alignment padding
#define GDI_NOALLOC_MAX_NODES ((int64_t)14897664)
#define GDI_NOALLOC_MAX_DEVICES 64

// host-side launchers (gdi_kernels.hip)
int gdi_launch_init_spins(const int32_t *orig, const int8_t *init_orig, int8_t *spin, int32_t n_pad,
                          uint32_t key0, uint32_t key1, uint32_t replica, void *stream);
// From-scratch M, doubled cut, doubled crossing count into out3[0..2] and the per-class +1
// counts into P; out3[0..3] and P[0 .. 2 ((C + 2) / 2)) are cleared first (no fills
// needed). bits: n_pad / 32 words of scratch for the bit-packed spins the neighbour reads
// use; spin 16-byte aligned.
int gdi_launch_reduce(const int32_t *rp, const int2 *adj, const int8_t *spin, int32_t n_pad, int64_t nnz,
                      const int32_t *cbeg, const int32_t *csz, int32_t C, int64_t *out3, int32_t *P,
                      uint32_t *bits, void *stream);
int gdi_launch_fill_u64(uint64_t *p, int64_t count, void *stream);
int gdi_launch_cut_finish(const int64_t *red, int64_t *out3, void *stream);
int gdi_scratch_ptr(void **out);
int gdi_launch_scatter_out(const int32_t *orig, const int8_t *spin, int32_t n_pad, int8_t *out_orig,
                           void *stream);
int gdi_launch_gather_in(const int32_t *orig, const int8_t *in_orig, int32_t n_pad, int8_t *spin,
                         void *stream);
int gdi_active_lds_bytes(int32_t n_pad, int32_t C);
int gdi_launch_sweep_active(const GdiSweepArgs &a, GdiActiveRec *rec, void *stream);
int gdi_dense_lds_bytes(int32_t n_pad, int32_t C);
int gdi_async_capacity(int block, int *max_grid);
int gdi_launch_sweep_async(const GdiSweepArgs &a, int grid, int block, void *stream);
int gdi_launch_sweep_dense(const GdiSweepArgs &a, int block, int lanes, void *stream);
int gdi_launch_sweep_wg(const GdiSweepArgs &a, int block, int lanes, int spins_in_lds, void *stream);
int gdi_wgl_lds_bytes(int32_t n_pad, int32_t C, int32_t nnz);
int gdi_launch_sweep_wgl(const GdiSweepArgs &a, const uint16_t *rp16, const uint16_t *ent16, int32_t nnz, int block,
                         int lanes, void *stream);
int gdi_launch_sweep_grid(const GdiSweepArgs &a, int grid, int block, int lanes, void *stream);
int gdi_grid_capacity(int block, int lanes, int *max_grid);
int gdi_launch_sweep_halo(const GdiHaloArgs &h, int grid, int block, void *stream);
int gdi_halo_capacity(int block, int lds_bytes, int *max_grid);
int gdi_wg_lds_bytes(int32_t n_pad, int32_t C, int spins_in_lds);
int gdi_batch_lds_bytes(int32_t n_pad, int32_t C);
int gdi_launch_sweep_batch(const GdiBatchArgs &ba, int grid, int block, int lds_bytes, int cooperative, void *stream);
int gdi_batch_occupancy(int block, int lds_bytes, int *per_cu);
const char *gdi_hip_error_string(int code);

// learned proposal (gdi_learned.hip)
int gdi_launch_features(const int32_t *rp, const int2 *adj, const int8_t *spin, const int32_t *last_flip,
                        int32_t n_pad, const int64_t *state, float T, int32_t t, int32_t A, int32_t B,
                        const int32_t *orig, void *X, int32_t dataset_rows, int64_t x_base, void *stream);
int gdi_launch_labels(const int32_t *last_flip, const int32_t *orig, int32_t n_pad, int32_t t_cut, uint8_t *y,
                      int64_t y_base, void *stream);
// Age proposal of one block (k_mask_age: real ids unflipped for >= k sweeps), then its
// count of skipped nodes into *block_skips (set) and, times weight, into *skipped (added)
// (k_sum_counts); part: scratch of part_cap >= 1 workgroup counts.
int gdi_launch_mask_age(const int32_t *last_flip, const int32_t *orig, int32_t n_pad, int32_t t, int32_t k,
                        uint32_t *mask, uint32_t *part, int32_t part_cap, uint64_t *skipped, uint32_t weight,
                        uint64_t *block_skips, void *stream);
int gdi_launch_fill_i32(int32_t *p, int64_t n, int32_t value, void *stream);
// Features, network and mask of one proposal block (k_mlp_mask), then its count of skipped
// nodes into *block_skips (set) and, times weight, into *skipped (added) (k_sum_counts);
// part: scratch of part_cap >= 1 workgroup counts.
int gdi_launch_mlp_mask(const int32_t *rp, const int2 *adj, const int8_t *spin, const int32_t *last_flip,
                        int32_t n_pad, const int64_t *state, float T, int32_t t, int32_t A, int32_t B,
                        const int32_t *orig, const GdiMlpDev *p, float thr_logit, uint32_t *mask, uint32_t *part,
                        int32_t part_cap, uint64_t *skipped, uint32_t weight, uint64_t *block_skips, void *stream);
int gdi_launch_mlp_infer(const void *X, int32_t count, const GdiMlpDev *p, float thr_logit, uint32_t *mask,
                         float *logits, void *stream);
// Loss and gradient of a minibatch of count rows: per-wave partial sums in part (at least
// gdi_mlp_grad_part_floats(count) floats), then grad (written, GDI_MLP_PARAMS floats) and
// *loss (the summed loss added, if loss is not NULL), the same bits on every run.
int gdi_mlp_grad_part_floats(int32_t count);
int gdi_launch_mlp_grad(const void *X, const uint8_t *Y, const int32_t *idx, int32_t count, const GdiMlpDev *p,
                        float inv_batch, float *part, float *grad, float *loss, void *stream);
int gdi_launch_adam(float *w, const float *g, float *m, float *v, int32_t P, float lr, float b1, float b2, float eps,
                    float bc1, float bc2, void *stream);
int gdi_launch_mlp_pack(const float *w, GdiMlpDev *p, void *stream);
