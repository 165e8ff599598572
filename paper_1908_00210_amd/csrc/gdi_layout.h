// gdi_layout.h -- host-only graph preparation of the GDI annealer: CSR validation,
// first-fit greedy colouring, colour-major relabelling and the halo layout of the
// fence-free grid sweep. No HIP types or calls: the library builds it with the
// rest of the host code, and the host tests build it alone under the address and
// undefined-behaviour sanitizers.
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

#define GDI_CLASS_ALIGN 64

// Halo layout of the fence-free grid sweep (k_sweep_halo). Each workgroup b owns,
// for every class c, a chunk of nodes (interior bounds multiples of 64), and keeps in
// LDS the spin bits of its chunk's packed words and copies of the foreign words: the
// packed words of class c that its nodes read and that another workgroup owns.
#define GDI_HALO_MAX_GRID 512
#define GDI_HALO_GROUP_PAD 16  // uint64 words between group words (128 bytes)
#define GDI_HALO_PF 16         // CSR entries per node held in registers across a barrier
#define GDI_HALO_THR_MAX 4096  // largest table width kept in LDS (two rows)
#define GDI_HALO_WMAX 1023     // largest |weight| the packed entries of the halo sweep hold

struct GdiHaloEntry {          // one per (workgroup, class)
    int32_t node_lo, node_hi;  // own nodes: new ids [node_lo, node_hi), node_lo a multiple of 64
    int32_t own_off;           // LDS word holding packed word node_lo / 32 (the chunk's words follow)
    int32_t for_off;           // LDS word of the first foreign word's copy
    int32_t for_len;           // foreign words of this class
    int32_t list_off;          // LDS word where their packed-word ids are listed (ascending)
    int32_t pad0, pad1;
};

// Dynamic LDS bytes of one halo-sweep workgroup: the image, the class table, the class
// counts and sizes, and thr_words threshold words.
int gdi_halo_lds_bytes(int32_t lds_words, int32_t C, int32_t thr_words);

namespace gdi_layout {

// One CSR entry after relabelling: {new column id, weight} (the device's int2 layout).
struct Edge {
    int32_t x, y;
};

// Validates a symmetric CSR graph (Sec. IV-A with int32 weights): row_ptr[0] = 0 and
// non-decreasing, columns in [0, n), strictly increasing per row, no self-loops, every
// edge mirrored with the same weight, sum_j |w_ij| <= 2^30. Returns 0, or GDI_EINVAL /
// GDI_ERANGE with a message in *err.
int validate_csr(const int32_t *rp, const int32_t *col, const int32_t *w, int32_t n, int64_t *max_wdeg,
                 int32_t *max_deg, std::string *err);

// First-fit greedy colouring in ascending node id: colour[i] is the smallest colour
// not taken by a neighbour j < i. Returns the number of colours.
int32_t colour_first_fit(const int32_t *rp, const int32_t *col, int32_t n, int32_t *colour);

// Colour-major relabelling: class c occupies new ids [cbeg[c], cbeg[c] + csz[c]) in
// ascending original id, cbeg[c] a multiple of GDI_CLASS_ALIGN; ids in the gaps are
// padding (orig -1, class -1, empty row). Rows are sorted by new column id.
struct Relabelled {
    int32_t n_pad = 0;
    std::vector<int32_t> cbeg, csz;  // per class
    std::vector<int32_t> orig;       // new -> original id, -1 for padding
    std::vector<int32_t> cls;        // class of each new id, -1 for padding
    std::vector<int32_t> rp;         // n_pad + 1 row pointers over new ids
    std::vector<Edge> adj;           // nnz entries
};

// Returns 0 or GDI_ERANGE (padded node count beyond int32) with a message in *err.
int relabel(const int32_t *rp, const int32_t *col, const int32_t *w, int32_t n, const int32_t *colour, int32_t C,
            Relabelled *out, std::string *err);

// Workgroup b handles chunk chunk_of_block(b) of every class; consecutive block ids
// are spread over the 8 XCDs, so XCD x gets a contiguous chunk range. With `lead`
// dedicated group leaders (blocks 0..7) those hold no chunk (-1).
inline int32_t chunk_of_block(int32_t b, int32_t G, int32_t lead)
{
    if (b < lead) return -1;
    const int32_t Gw = G - lead, bw = b - lead;  // bw % 8 == b % 8
    return (Gw % 8 == 0) ? (bw % 8) * (Gw / 8) + bw / 8 : bw;
}

// Packed halo CSR entry from an LDS bit index lb: (lb / 32) << 16 | the weight's low 11
// bits << 5 | lb % 32.
inline uint32_t pack_entry(int32_t lb, int32_t w)
{
    return ((uint32_t)(lb >> 5) << 16) | (((uint32_t)w & 0x7FFu) << 5) | ((uint32_t)lb & 31u);
}

// Packed rows of a graph whose weights are all +-1 and whose n_pad is below 32767: every
// row is a whole number of 16-byte chunks of eight 16-bit entries, column | (weight < 0)
// << 15, the last chunk filled with entries naming node n_pad (a spin slot that always
// reads 0, so padding adds nothing to a local field). Row v occupies chunks
// [prow[v], prow[v + 1]).
#define GDI_P8_ENTRIES 8
struct PackedRows {
    std::vector<uint32_t> prow;   // n_pad + 1 chunk offsets
    std::vector<uint16_t> pent;   // 8 x prow[n_pad] entries (at least one chunk)
};

// Returns 0, or -1 (not applicable: a weight other than +-1, n_pad >= 32767, or more
// than 2^32 - 1 chunks) with a message in *err.
int pack_rows8(const Relabelled &g, PackedRows *out, std::string *err);

// The halo layout for G workgroups with the redundant tail from class T0 on.
struct HaloLayout {
    int32_t status = 0;    // 0 = built; -2 = does not fit the LDS budget; -3 = a weight beyond GDI_HALO_WMAX
    int32_t unit_w = 0;    // every weight is 1
    int32_t lds_words = 0, T0 = 0;
    int32_t gather_off = 0, tail_off = 0, trp_off = 0, tent_off = 0;
    int32_t ovf_off = 0, ovf_len = 0;
    int32_t list_off = 0, flist_len = 0;     // LDS word of the foreign-id list region; its length
    std::vector<GdiHaloEntry> tab;           // G x C
    std::vector<int32_t> flist;              // G x flist_len: each workgroup's foreign word ids by class
    std::vector<uint32_t> adjL;              // nnz + GDI_HALO_PF packed entries
    std::vector<int32_t> tail_v, tail_beg, tail_rp;
    std::vector<uint32_t> tail_ent;
    std::vector<int32_t> gat_words, gat_beg;
    std::vector<uint32_t> ovf;               // G x ovf_len
};

// Returns 0 (see status) or GDI_EDEVICE when an internal index check fails.
int halo_layout(const Relabelled &g, int32_t C, int32_t G, int lds_budget, int32_t T0, int32_t lead,
                HaloLayout *out, std::string *err);

}  // namespace gdi_layout
