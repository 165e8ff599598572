/*
 * gdi.h -- C ABI of the MI355X (gfx950) Globally Decoupled Ising annealer for
 * balanced 2-way min-cut partitioning.
 *
 * The method (paper: "GPU-based Ising Computing for Solving Balanced Min-Cut
 * Graph Partitioning Problem", Sec. IV eq. 4-6 and Sec. V Alg. 3):
 *
 *   spins s_i in {-1,+1} encode the two parts (s_i = +1 -> V1, -1 -> V2,
 *   Sec. IV-A); the energy is E = A*M^2 + B*cut_w with M = sum_i s_i (eq. 5,
 *   the balance penalty) and cut_w = sum over edges of w_ij*[s_i != s_j]
 *   (eq. 6, weighted). Instead of the dense all-to-all coupling of the balance
 *   term, every spin reads a separately tracked global magnetisation M
 *   (Alg. 3's global G), so a spin's flip cost is
 *       dE_i = B*s_i*h_i + 4A*(1 - s_i*M_seen),   h_i = sum_j w_ij s_j,
 *   and only its sparse neighbours are read.
 *
 * Deterministic execution (where the paper's asynchronous GPU update is
 * unspecified, Sec. V-B/V-C):
 *   - nodes are coloured by first-fit greedy colouring in ascending node id;
 *     each sweep visits the colour classes in ascending colour, one phase per
 *     class; all spins of a class decide against the same pre-phase state;
 *   - M_seen: GDI_BAL_GATED (default): an over-side spin (s_i == sign(M0))
 *     sees M0 iff x1 * O < floor(|M0|/2) * 2^32, where M0 is the magnetisation
 *     at the start of the phase and O the number of over-side spins in the
 *     class; every other spin sees 0. GDI_BAL_SNAPSHOT: every spin sees M0;
 *   - Metropolis acceptance: flip iff dE <= 0 or x0 < thr_t(dE) with
 *     thr_t(d) = min(2^32-1, floor(2^32*exp(-d/T_t))) built on the host in FP64;
 *   - x0, x1 are words 0 and 1 of Philox4x32-10 (Salmon et al., SC'11) with
 *     key (seed & 0xffffffff, seed >> 32) and counter (node, sweep, replica, 0);
 *     the initial state uses counter (node, 0, replica, 1): s = +1 iff x0 odd.
 * All arithmetic after the threshold table is integer, so results are
 * bit-identical across launch shapes and runs.
 *
 * Conventions:
 *   - Return codes: GDI_OK (0) or a negative GDI_E* code; gdi_last_error()
 *     returns a thread-local message for the last non-zero return.
 *   - Node ids are the caller's ids ("original order") in every input and
 *     output; the library relabels internally.
 *   - The caller owns every input array; gdi_create copies what it needs.
 *     The handle owns its device memory until gdi_destroy.
 *   - Host variants block until the result is on the host. The *_dev
 *     variants take device pointers and are ordered on the stream set with
 *     gdi_set_stream (default: the null stream); they return after enqueueing
 *     (device errors are then reported by the next call on the handle).
 *   - One handle must not be used from two threads at once.
 *   - No C++ exception crosses this interface.
 */
#ifndef GDI_H
#define GDI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ codes */
#define GDI_OK 0
#define GDI_EINVAL (-1)   /* malformed CSR, bad schedule, NULL argument */
#define GDI_ERANGE (-2)   /* a weight sum or an energy change does not fit int32 */
#define GDI_ENOMEM (-3)   /* host or device allocation failed */
#define GDI_EDEVICE (-4)  /* HIP error, no gfx950 device, or launch does not fit */
#define GDI_ESTATE (-5)   /* NULL handle or call out of order */
#define GDI_ETIMEOUT (-6) /* a bounded device-side wait expired (no hang) */

#define GDI_BAL_GATED 0u
#define GDI_BAL_SNAPSHOT 1u

/* Scope of the persistent sweep launch. GDI_SCOPE_AUTO: one workgroup up to 6144
 * padded nodes, else the grid sweep (GDI_SCOPE_GRID) on about one workgroup per 1,500
 * nodes (at least 64 where that leaves 128 nodes each, at most one per CU); graphs the
 * grid sweep cannot hold (|w| > 1023, too many spin words for LDS) run on one workgroup
 * up to 65536 padded nodes, above that on GDI_SCOPE_GRID_FENCED. */
#define GDI_SCOPE_AUTO 0u
#define GDI_SCOPE_WORKGROUP 1u /* whole instance inside one workgroup */
#define GDI_SCOPE_GRID 2u      /* instance spread over the whole device; spins exchanged through
                                  per-workgroup LDS copies of the spin words each
                                  workgroup reads, no cache-wide fences */
#define GDI_SCOPE_GRID_FENCED 3u /* whole device, spins gathered from global memory with
                                    release/acquire fences per phase (any graph) */

typedef struct gdi_graph gdi_graph;

/* Acceptance rules. Metropolis: flip iff dE <= 0 or x0 < floor(2^32 exp(-dE/T_t)).
 * Paper (Sec. V, Alg. 2/3): the spin first takes the value that minimises its local
 * energy (flip iff dE < 0; at dE = 0 the value is random, Sec. III: +1 iff Philox
 * word x2 is odd), then flips with probability P_f(t): flip iff
 * argmin_flips != (x0 < min(2^32 - 1, floor(2^32 P_f(t)))). */
#define GDI_ACCEPT_METROPOLIS 0u
#define GDI_ACCEPT_PAPER 1u

/* Annealing schedule (Alg. 3 outer loop). */
typedef struct {
    uint32_t n_sweeps;        /* S >= 1: length of temps */
    uint32_t start_sweep;     /* first sweep to run (resume); 0 = fresh start */
    const double *temps;      /* host, S values (FP64), read during the call: temperatures T_t > 0
                                 (Metropolis) or flip probabilities P_f(t) in [0, 1] (paper rule) */
    int32_t A;                /* balance coefficient (eq. 5) */
    int32_t B;                /* cut coefficient (eq. 6) */
    uint32_t replica;         /* Philox counter word 2 */
    uint32_t balance_mode;    /* GDI_BAL_GATED or GDI_BAL_SNAPSHOT */
    const int8_t *init_spins; /* host, n spins (original order) to start from, or NULL for the Philox state */
    int64_t *trace_m;         /* host, S entries or NULL: M after each sweep t >= start_sweep */
    int64_t *trace_cut;       /* host, S entries or NULL: weighted cut after each sweep t >= start_sweep */
    uint32_t acceptance;      /* GDI_ACCEPT_METROPOLIS or GDI_ACCEPT_PAPER (the learned schedule
                                 and trace collection take Metropolis only) */
    uint32_t flags;           /* GDI_FLAG_*; 0 for the batched and learned forms */
} gdi_schedule;

/* The standard solver of Alg. 2: every decision computes the balance term from the
 * whole spin vector (all n spins, plus its class's over-side count) instead of the
 * tracked magnetisation -- identical results, n reads per decision. Graphs that fit
 * one workgroup (n_pad <= 65536) only; GDI_ERANGE otherwise. */
#define GDI_FLAG_DENSE_BALANCE 1u

/* Alg. 3 as printed (Sec. V-C), asynchronous and racy, in one persistent launch: every
 * sweep, each thread takes its nodes in turn, reads the neighbour spins and the global
 * magnetisation G as it finds them (other nodes may or may not have flipped yet), and
 * when its spin flips stores it and adds the change to G with one atomic add; a
 * device-wide barrier separates sweeps. No colour phases, no gate; results are NOT
 * reproducible (for pricing determinism). The returned M is G as the atomic adds left
 * it (equal to the sum of the final spins); the cut is recounted from the final spins.
 * tuning.grid (0 = every co-resident workgroup of 1024 threads) sets how many nodes are
 * in flight at once. No traces. */
#define GDI_FLAG_RACY 2u

/* Launch tuning; zero fields mean "choose automatically". */
typedef struct {
    uint32_t scope;           /* GDI_SCOPE_* */
    uint32_t block;           /* threads per workgroup: 64..1024, multiple of 64 */
    uint32_t grid;            /* workgroups for GDI_SCOPE_GRID (<= co-resident capacity) */
    uint32_t lanes_per_node;  /* 1, 2, 4, 8, 16, 32 or 64 lanes share one CSR row */
    int32_t tail_max;         /* GDI_SCOPE_GRID: most nodes in the redundant tail of small
                                 classes run by every workgroup without grid barriers
                                 (0 = automatic: at most one node per worker thread;
                                 < 0 = no tail; > 0 = at most this many, capped at one
                                 per worker thread) */
    uint64_t spin_limit;      /* polls before a device-side barrier wait gives up with
                                 GDI_ETIMEOUT (0 = default, about a second) */
    int32_t leaders;          /* GDI_SCOPE_GRID: > 0 = the 8 workgroups that collect the
                                 phase sums of their XCD (blocks 0..7) hold no nodes, so
                                 that no node work queues ahead of their polls; < 0 =
                                 they hold nodes like every workgroup; 0 = automatic
                                 (dedicated on grids of 64 or more workgroups) */
    int32_t general_weights;  /* GDI_SCOPE_GRID: > 0 = run the general-weight form of the
                                 sweep even when every weight is 1 (for measuring what the
                                 unit-weight form saves; same results); 0 = automatic */
    int32_t csr_lds;          /* GDI_SCOPE_WORKGROUP: the whole graph (spins, ids, 16-bit
                                 CSR) in LDS; needs n_pad <= 32768, nnz <= 65535 and +-1
                                 weights. 0 = whenever it fits, < 0 = never, > 0 = required
                                 (GDI_ERANGE if it does not fit) */
    int32_t batch_members;    /* batched form: most workgroups one large instance may run on
                                 (a cluster; instances above twice the per-workgroup share
                                 of the batch's work); 0 = automatic (up to 16), < 0 or 1 =
                                 one workgroup per instance */
} gdi_tuning;

/* Outcome of the last anneal on a handle. */
typedef struct {
    int64_t magnetization;    /* M = sum of spins = |V1| - |V2| */
    int64_t cut_weighted;     /* tracked weighted cut */
    double sweep_ms;          /* device time of the persistent sweep launch */
    uint32_t n_colours;       /* number of colour classes (phases per sweep) */
    uint32_t scope;           /* GDI_SCOPE_WORKGROUP or GDI_SCOPE_GRID */
    uint32_t grid;            /* workgroups launched */
    uint32_t block;           /* threads per workgroup */
    uint32_t lanes_per_node;
    uint32_t table_width;     /* largest dE with a non-zero threshold (K) */
} gdi_result;

/* Graph facts after gdi_create. */
typedef struct {
    int32_t n;
    int32_t n_colours;
    int64_t nnz;              /* directed CSR entries = 2|E| */
    int64_t max_abs_wdeg;     /* max_i sum_j |w_ij| */
    int32_t max_degree;
    int32_t pad;
} gdi_graph_info;

/*
 * gdi_create -- validate a symmetric CSR graph (Sec. IV-A: G(V,E), here with
 * int32 edge weights), colour it, relabel it colour-major and upload it.
 *   row_ptr  host, n+1 int32, row_ptr[0] = 0, non-decreasing
 *   col_idx  host, row_ptr[n] int32 column ids in [0,n), strictly increasing within a row,
 *            no self-loops; every edge (i,j,w) must have its mirror (j,i,w)
 *   weights  host, row_ptr[n] int32 edge weights
 *   n        number of nodes, >= 2
 *   out      receives the handle
 * Errors: GDI_EINVAL (malformed or asymmetric CSR, NULL pointer, n < 2),
 *         GDI_ERANGE (sum_j |w_ij| > 2^30 for some i), GDI_ENOMEM, GDI_EDEVICE.
 * Validation runs before any device call, so malformed input fails without a GPU.
 */
int gdi_create(const int32_t *row_ptr, const int32_t *col_idx, const int32_t *weights, int32_t n,
               gdi_graph **out);

/* gdi_destroy -- release the handle and its device memory (NULL is a no-op). */
void gdi_destroy(gdi_graph *g);

/* gdi_set_stream -- order all later device work of the handle on this hipStream_t (NULL = null stream). */
int gdi_set_stream(gdi_graph *g, void *hip_stream);

/* gdi_set_tuning -- override launch parameters (NULL restores automatic choice). */
int gdi_set_tuning(gdi_graph *g, const gdi_tuning *tune);

/*
 * gdi_anneal -- run sweeps start_sweep..S-1 of the GDI schedule (Alg. 3 with
 * the deterministic readings above) in one persistent device launch and copy
 * the final spins (original node order) to spins_out (host, n int8).
 * The final state is returned, not the best one seen.
 * Errors: GDI_EINVAL (schedule), GDI_ERANGE (|B|*max_wdeg + 4|A|(n+1) >= 2^31),
 *         GDI_ESTATE, GDI_EDEVICE, GDI_ETIMEOUT, GDI_ENOMEM.
 */
int gdi_anneal(gdi_graph *g, const gdi_schedule *s, uint64_t seed, int8_t *spins_out);

/* gdi_anneal_dev -- as gdi_anneal, with d_spins_out a device pointer (n int8, original order);
 * stream-ordered, returns after enqueueing. trace_* pointers must be NULL. */
int gdi_anneal_dev(gdi_graph *g, const gdi_schedule *s, uint64_t seed, int8_t *d_spins_out);

/* gdi_last_result -- outcome of the last anneal (synchronises the handle's stream). */
int gdi_last_result(gdi_graph *g, gdi_result *out);

/*
 * gdi_cut -- from-scratch weighted cut, crossing-edge count (the paper's "cut",
 * Sec. VI) and magnetisation M of a spin vector (host, n int8, original order,
 * any non-positive value counts as -1). The paper's imbalance "bal" is |M|/2.
 * Any output pointer may be NULL.
 */
int gdi_cut(gdi_graph *g, const int8_t *spins, int64_t *cut_weighted, int64_t *cut_edges,
            int64_t *magnetization);

/* gdi_cut_dev -- as gdi_cut with d_spins a device pointer; blocks until the three values are on the host. */
int gdi_cut_dev(gdi_graph *g, const int8_t *d_spins, int64_t *cut_weighted, int64_t *cut_edges,
                int64_t *magnetization);

/*
 * gdi_cut_dev_noalloc -- for callers that cannot allocate device memory (code under
 * HIP graph capture, serving loops, harnesses that forbid hipMalloc): gdi_cut_dev
 * without any allocation. d_spins: device, n int8 in original order (any non-positive
 * value counts as -1); d_out: device, 3 int64 receiving the weighted cut, the
 * crossing-edge count and M. Stream-ordered on the handle's stream (gdi_set_stream);
 * returns after enqueueing and leaves a pending anneal's outcome untouched. Its scratch
 * (the relabelled spin copy, its bit-packed copy and the reduction's accumulators) lives
 * in one fixed 16 MiB device array per GPU, held until the process ends: graphs with
 * n + 64 * colours <= 14,897,664 and at most 4094 colour classes; GDI_ERANGE otherwise.
 * Every call on one
 * GPU uses that GPU's array, so calls that overlap on one GPU (any handle, any stream)
 * race and must be serialised by the caller.
 */
int gdi_cut_dev_noalloc(gdi_graph *g, const int8_t *d_spins, int64_t *d_out);

/* gdi_get_info -- graph facts. */
int gdi_get_info(const gdi_graph *g, gdi_graph_info *out);

/* gdi_get_colouring -- colour of every node (original order) and class sizes (n_colours entries). */
int gdi_get_colouring(const gdi_graph *g, int32_t *colour_out, int32_t *class_size_out);

/*
 * gdi_colour_csr -- host-only: first-fit greedy colouring in ascending node id of a
 * validated CSR (colour_out: n int32). Returns the number of colours (> 0) or a GDI_E* code.
 */
int gdi_colour_csr(const int32_t *row_ptr, const int32_t *col_idx, int32_t n, int32_t *colour_out);

/*
 * gdi_threshold_table -- host-only: out[t*(width+1) + d] = min(2^32-1, floor(2^32*exp(-d/T_t)))
 * for t < n_sweeps, 1 <= d <= width; entry d = 0 is 2^32-1. temps must be > 0.
 */
int gdi_threshold_table(const double *temps, uint32_t n_sweeps, int32_t width, uint32_t *out);

/*
 * gdi_philox4x32_10 -- host-only: the Philox4x32-10 block of one counter under
 * key (seed low, seed high). For checking the generator the kernels use.
 */
int gdi_philox4x32_10(uint64_t seed, const uint32_t ctr[4], uint32_t out[4]);

/* ------------------------------------------------------------------ batched form
 * Many independent anneals (graph, replica) in ONE persistent launch: every
 * workgroup repeatedly takes the next instance from a device-side queue (longest
 * first) and runs all sweeps of that instance; the result of each instance is
 * bit-identical to gdi_anneal on the same graph, schedule, seed and replica.
 * The paper keeps the best of 10 independent runs per graph (Sec. VI-B); this is
 * the device-side form of running many such runs at once.
 */
typedef struct {
    gdi_graph *graph;          /* the instance's graph (must outlive the call) */
    uint32_t replica;          /* Philox counter word 2 */
    uint32_t pad;
    int8_t *spins_out;         /* n spins, original order: host memory for gdi_anneal_batch, device
                                  memory for gdi_anneal_batch_dev; NULL to skip */
    int64_t magnetization;     /* out: final M */
    int64_t cut_weighted;      /* out: final weighted cut */
} gdi_instance;

/*
 * gdi_anneal_batch -- run all instances with one schedule (start_sweep must be 0,
 * init_spins and traces NULL) and seed. tune: block, grid (workgroups) and
 * lanes_per_node (0 = per-graph choice) of the launch, or NULL for the cached
 * autotuned choice (gdi_autotune_batch runs on the first call for a batch shape).
 * Blocks until the results are on the host; kernel_ms (may be NULL) receives the
 * device time of the launch. Runs on the stream of the first instance's graph.
 * Errors: GDI_EINVAL (empty batch, NULL graph, bad schedule), GDI_ERANGE (an instance
 * does not fit one workgroup's LDS or its energy range int32), GDI_EDEVICE, GDI_ENOMEM.
 */
int gdi_anneal_batch(gdi_instance *inst, uint32_t n_inst, const gdi_schedule *s, uint64_t seed,
                     const gdi_tuning *tune, double *kernel_ms);

/* gdi_anneal_batch_dev -- as gdi_anneal_batch with device spins_out pointers. */
int gdi_anneal_batch_dev(gdi_instance *inst, uint32_t n_inst, const gdi_schedule *s, uint64_t seed,
                         const gdi_tuning *tune, double *kernel_ms);

/*
 * gdi_autotune_batch -- time candidate launches (block size, lanes per node, workgroups
 * per CU and cluster size, by coordinate descent) on the first probe_sweeps
 * sweeps of the schedule and return the fastest in best (and its time in best_ms).
 * The choice is cached per batch shape and used by gdi_anneal_batch with tune == NULL.
 * Results never depend on the choice. Outputs of inst are not written. The search also
 * covers the cluster size of the large instances (tuning.batch_members). Not in the
 * paper: launch tuning of the batched form above.
 */
int gdi_autotune_batch(gdi_instance *inst, uint32_t n_inst, const gdi_schedule *s, uint64_t seed,
                       uint32_t probe_sweeps, gdi_tuning *best, double *best_ms);

/*
 * gdi_autotune -- time launch choices for one graph (the workgroup sweep with the CSR in
 * LDS or global memory, lanes per node and block size; the halo grid sweep on 8 to 256
 * workgroups, with and without the redundant tail and dedicated leaders) on the first
 * probe_sweeps sweeps of the schedule (0 = n_sweeps / 50, at least 1; flags must be 0),
 * install the fastest on the handle as gdi_set_tuning does, and return it in best (and
 * its device time in best_ms, may be NULL). With use_cache != 0 a cached choice for this
 * device and graph shape (n, nnz, colours, maximum degree, weight kind) is installed
 * without timing. Results never depend on the choice. Runs anneals on the handle, so its
 * last result is overwritten. Errors: GDI_ESTATE (NULL handle), GDI_EINVAL (NULL best,
 * bad schedule), GDI_EDEVICE, GDI_ENOMEM, GDI_ETIMEOUT; on an error the handle's tuning
 * is left as it was. Not in the paper: launch tuning of the sweep that gdi_anneal runs
 * (Alg. 3 with colour phases, Sec. V).
 */
int gdi_autotune(gdi_graph *g, const gdi_schedule *s, uint64_t seed, uint32_t probe_sweeps, int use_cache,
                 gdi_tuning *best, double *best_ms);

/*
 * The autotuners' cache: choices keyed by device ("<arch>/<CUs>cu") and problem shape,
 * used by gdi_autotune (use_cache) and by gdi_anneal_batch (tune == NULL). If the
 * environment variable GDI_TUNE_CACHE names a file, the cache is read from it at the
 * first lookup of the process and written back after every tuning run (a missing or
 * malformed file is ignored there). The file is JSON:
 *   {"format": "gdi-tune-1", "entries": {"<key>": {"scope": .., "block": .., "grid": ..,
 *    "lanes_per_node": .., "tail_max": .., "leaders": .., "general_weights": ..,
 *    "csr_lds": .., "batch_members": .., "ms": <measured time>}, ...}}
 * Entries whose fields are missing or out of range are ignored at lookup. No GPU needed.
 * gdi_tune_cache_load -- merge the entries of a file (same keys replaced); GDI_EINVAL
 *   (NULL path, unreadable file, not this format: then nothing is merged).
 * gdi_tune_cache_save -- write the whole cache to path (through a temporary file and a
 *   rename); GDI_EINVAL (NULL path, cannot write).
 * gdi_tune_cache_clear -- empty the in-memory cache (the file is not touched).
 * gdi_tune_cache_size -- number of entries in the in-memory cache.
 * Not in the paper (bookkeeping of the launch tuners above).
 */
int gdi_tune_cache_load(const char *path);
int gdi_tune_cache_save(const char *path);
int gdi_tune_cache_clear(void);
int gdi_tune_cache_size(void);

/* ------------------------------------------------------------------ learned proposal
 * A network predicts which nodes stay frozen at the current temperature; masked
 * sweeps skip them and a full sweep runs every k_full sweeps. The network is
 * 6 -> 64 -> 64 -> 1 (ReLU, logistic output), BF16 weights and FP32 accumulation
 * on the GPU (dense layers on MFMA). Per-node features, computed on the device
 * after each full sweep t (FP32, then rounded to BF16):
 *   f0 = degree/16, f1 = sum_j |w_ij| / 16, f2 = fraction of neighbours on the other side,
 *   f3 = clamp(B s_i h_i / T_t, -16, 16) / 4, f4 = min(|4A(1 - s_i M)| / T_t, 64) / 16,
 *   f5 = min(t - last flip of i, 255) / 64  (last flip = start_sweep - 1 before any flip).
 * Not in the paper: this is a systems form built on top of its annealer.
 */
#define GDI_MLP_FEATURES 6
#define GDI_MLP_HIDDEN 64

typedef struct {
    float w1[64][6];           /* hidden x feature */
    float b1[64];
    float w2[64][64];          /* output hidden x input hidden */
    float b2[64];
    float w3[64];
    float b3;
} gdi_mlp_weights;             /* FP32 master weights; the device uses BF16 copies of w1, w2 */

#define GDI_SKIP_NONE 0u       /* every sweep is full (same trajectory as gdi_anneal) */
#define GDI_SKIP_MLP 1u        /* skip nodes with p(frozen) > skip_threshold */
#define GDI_SKIP_HEURISTIC 2u  /* skip nodes that did not flip in the last heuristic_k sweeps */

typedef struct {
    uint32_t k_full;           /* sweeps start_sweep, start_sweep + k_full, ... are full sweeps */
    uint32_t skip_mode;        /* GDI_SKIP_* */
    float skip_threshold;      /* GDI_SKIP_MLP: probability threshold in (0, 1) */
    uint32_t heuristic_k;      /* GDI_SKIP_HEURISTIC */
    uint8_t *mask_trace;       /* host or NULL: ceil((S - b0) / k_full) x n bytes with
                                  b0 = max(start_sweep, learn_from), original order:
                                  1 = node skipped in the masked sweeps after that full sweep */
    int32_t active_max;        /* masked sweeps with at most this many active nodes run in one
                                  workgroup over the active nodes only (spins as LDS bits);
                                  0 = automatic, < 0 = never (the full-graph kernel skips nodes) */
    uint32_t learn_from;       /* sweeps before this one run without a proposal, in one launch;
                                  full sweeps then fall on max(start_sweep, learn_from) + m k_full */
} gdi_learned_cfg;

typedef struct {
    int64_t magnetization;
    int64_t cut_weighted;
    double total_ms;           /* device time of all launches of the anneal */
    uint64_t node_visits;      /* decisions made */
    uint64_t node_skips;       /* decisions skipped by the proposal */
} gdi_learned_result;

/*
 * gdi_anneal_learned -- the schedule of gdi_anneal (same RNG counters, same
 * acceptance) with nodes flagged by the proposal skipped in the masked sweeps: a
 * skipped node keeps its spin and draws nothing; the phase's magnetisation and
 * class counts are those of all nodes. w may be NULL unless skip_mode is
 * GDI_SKIP_MLP. Blocks until spins_out (host, original order) is written.
 */
int gdi_anneal_learned(gdi_graph *g, const gdi_schedule *s, uint64_t seed, const gdi_mlp_weights *w,
                       const gdi_learned_cfg *cfg, int8_t *spins_out, gdi_learned_result *res);

/*
 * gdi_collect_traces -- training data from a plain anneal: after each sweep
 * t_s = every-1, 2*every-1, ... with t_s + k_label < S, the features of all n
 * nodes are written to d_x (device, BF16 rows of 8: six features and two zeros,
 * row = snapshot * n + original id) and d_y (device, 1 = the node does not flip in
 * sweeps t_s+1 .. t_s+k_label). At most max_snapshots snapshots; *n_snapshots
 * receives the number written.
 */
int gdi_collect_traces(gdi_graph *g, const gdi_schedule *s, uint64_t seed, uint32_t every, uint32_t k_label,
                       void *d_x, uint8_t *d_y, uint32_t max_snapshots, uint32_t *n_snapshots);

typedef struct {
    uint32_t epochs;
    uint32_t batch;            /* minibatch rows */
    float lr, beta1, beta2, eps;   /* Adam */
    uint64_t seed;             /* minibatch shuffling */
} gdi_train_cfg;

/* gdi_mlp_init -- He-uniform initial weights from a seeded splitmix64 stream (host). */
int gdi_mlp_init(gdi_mlp_weights *w, uint64_t seed);

/*
 * gdi_mlp_train -- minimise the mean logistic loss on (d_x, d_y) (device rows as
 * written by gdi_collect_traces) with the library's forward / backward / Adam
 * kernels; w holds the initial weights and receives the trained ones;
 * epoch_loss (host, epochs entries) may be NULL. Runs on hip_stream. The gradient
 * sums run in a fixed order (no floating-point atomics), so equal inputs give the
 * same weights and losses bit for bit on every run. Device scratch of about
 * 73 KB per 64 minibatch rows (at most 9.6 MB) is allocated for the call.
 */
int gdi_mlp_train(const void *d_x, const uint8_t *d_y, uint64_t n, gdi_mlp_weights *w, const gdi_train_cfg *cfg,
                  float *epoch_loss, void *hip_stream);

/* gdi_mlp_forward -- logits of n device rows into d_logits (device); for checking the kernels. */
int gdi_mlp_forward(const gdi_mlp_weights *w, const void *d_x, uint32_t n, float *d_logits, void *hip_stream);

/* gdi_mlp_gradient -- mean logistic loss of n device rows (n < 2^31) and its gradient
 * (host outputs); the same bits on every call (sums in a fixed order). */
int gdi_mlp_gradient(const gdi_mlp_weights *w, const void *d_x, const uint8_t *d_y, uint32_t n,
                     gdi_mlp_weights *grad, float *loss, void *hip_stream);

/* gdi_last_error -- thread-local message of the last failing call ("" if none). */
const char *gdi_last_error(void);

/* gdi_version -- ABI version (major*10000 + minor*100 + patch). */
int gdi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* GDI_H */
