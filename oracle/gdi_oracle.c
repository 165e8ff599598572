/*
 * gdi_oracle.c -- plain CPU oracle of the Globally Decoupled Ising (GDI) annealer
 * for balanced 2-way min-cut.
 *
 * TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load this library. The product path (the HIP
 * library) shares no code, header, table or helper with it.
 *
 * What it computes (paper: Sec. IV eq. 4-6 for the energy, Sec. V Alg. 3 for the
 * decoupled update), with the readings this project fixes where the paper is
 * silent:
 *
 *   E(s)  = A * M^2 + B * cut_w(s),    M = sum_i s_i,
 *   cut_w = sum over undirected edges {i,j} of w_ij * [s_i != s_j]        (eq. 5, eq. 6)
 *
 * Flipping spin i changes the cut by s_i*h_i (h_i = sum_j w_ij s_j) and the
 * balance term by 4A(1 - s_i M), so dE_i = B s_i h_i + 4A (1 - s_i M) with M
 * read from the separately tracked magnetisation instead of the dense
 * all-to-all coupling (Alg. 3: the global G is read, not recomputed).
 *
 * Deterministic schedule:
 *   - nodes are split into colour classes by first-fit greedy colouring in
 *     ascending node id; classes are visited in ascending colour, each class is
 *     one phase (an independent set, so neighbour spins are exact);
 *   - at the start of each phase the magnetisation M0 is read once; in GATED
 *     mode an over-side spin (s_i == sign(M0)) sees the true M0 only if its gate
 *     word x1 satisfies x1 * O < floor(|M0|/2) * 2^32 (O = over-side spins in
 *     the class), every other spin sees a balanced M = 0; in SNAPSHOT mode every
 *     spin sees M0;
 *   - acceptance is Metropolis: flip iff dE <= 0, or x0 < thr_t(dE) with
 *     thr_t(d) = min(2^32-1, floor(2^32 exp(-d/T_t))) computed in FP64;
 *   - x0, x1 are words 0 and 1 of Philox4x32-10 (Salmon et al., SC'11) with
 *     key = (seed low, seed high) and counter = (node, sweep, replica, 0);
 *     initial spins use counter (node, 0, replica, 1): s_i = +1 iff x0 is odd;
 *   - after all decisions of a phase, the flips are applied and M, the per-class
 *     count of +1 spins and the cut are updated incrementally.
 *
 * All arithmetic after the threshold table is integer (int64 here).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_ENOMEM (-3)

#define OR_MODE_GATED 0
#define OR_MODE_SNAPSHOT 1
/* Acceptance rules. Metropolis: flip iff dE <= 0 or x0 < thr_t(dE). The paper's
 * rule (Sec. V, Alg. 2 and 3): the spin takes the value minimising its local energy
 * (flip iff dE < 0; at dE = 0 the local field is zero and the value is random,
 * Sec. III: +1 iff x2 is odd) and is then flipped with probability P_f(t), drawn as
 * x0 < min(2^32 - 1, floor(2^32 P_f(t))); the two flips compose. */
#define OR_RULE_METROPOLIS 0
#define OR_RULE_PAPER 1

/* ---------------------------------------------------------------- Philox4x32-10
 * Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3"
 * (SC'11). One round maps (c0,c1,c2,c3) with key (k0,k1) to
 *   (hi(R1*c2) ^ c1 ^ k0, lo(R1*c2), hi(R0*c0) ^ c3 ^ k1, lo(R0*c0))
 * with R0 = 0xD2511F53, R1 = 0xCD9E8D57; the key is bumped by the Weyl
 * constants (0x9E3779B9, 0xBB67AE85) between rounds; ten rounds.
 */
void oracle_philox4x32_10(uint32_t k0, uint32_t k1, const uint32_t ctr[4], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Batched form for tests: m counters, out is m x 4. */
void oracle_philox_many(uint64_t seed, int64_t m, const uint32_t *ctrs, uint32_t *out)
{
    for (int64_t q = 0; q < m; ++q)
        oracle_philox4x32_10((uint32_t)seed, (uint32_t)(seed >> 32), ctrs + 4 * q, out + 4 * q);
}

/* ---------------------------------------------------------------- thresholds
 * thr(d; T) = min(2^32 - 1, floor(2^32 * exp(-d / T))), FP64 with libm exp.
 */
uint32_t oracle_threshold(int64_t d, double T)
{
    double v = ldexp(exp(-(double)d / T), 32);
    double f = floor(v);
    if (f >= 4294967295.0) return 0xFFFFFFFFu;
    if (f <= 0.0) return 0u;
    return (uint32_t)f;
}

/* Fills out[t*(width+1) + d] = thr(d; T[t]) for d = 0..width (entry 0 is unused and set to 2^32-1). */
void oracle_thresholds(const double *T, int32_t S, int32_t width, uint32_t *out)
{
    for (int32_t t = 0; t < S; ++t) {
        out[(int64_t)t * (width + 1)] = 0xFFFFFFFFu;
        for (int32_t d = 1; d <= width; ++d)
            out[(int64_t)t * (width + 1) + d] = oracle_threshold(d, T[t]);
    }
}

/* ---------------------------------------------------------------- colouring
 * First-fit greedy in ascending node id: colour[i] is the smallest c >= 0 not
 * used by any neighbour j < i. Returns the number of colours C, or < 0 on error.
 */
int32_t oracle_colour(int32_t n, const int32_t *row_ptr, const int32_t *col, int32_t *colour)
{
    if (n <= 0) return OR_EINVAL;
    /* stamp[c] == i + 1 marks colour c as used by a lower neighbour of i */
    int64_t *stamp = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    if (!stamp) return OR_ENOMEM;
    int32_t ncol = 0;
    for (int32_t i = 0; i < n; ++i) {
        for (int32_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
            int32_t j = col[k];
            if (j < i) stamp[colour[j]] = (int64_t)i + 1;
        }
        int32_t c = 0;
        while (stamp[c] == (int64_t)i + 1) ++c;
        colour[i] = c;
        if (c + 1 > ncol) ncol = c + 1;
    }
    free(stamp);
    return ncol;
}

/* ---------------------------------------------------------------- cut / energy */

/* From-scratch weighted cut, crossing-edge count and magnetisation. */
void oracle_cut(int32_t n, const int32_t *row_ptr, const int32_t *col, const int32_t *w,
                const int8_t *spin, int64_t *cut_w, int64_t *cut_edges, int64_t *mag)
{
    int64_t cw2 = 0, ce2 = 0, m = 0;
    for (int32_t i = 0; i < n; ++i) {
        m += spin[i];
        for (int32_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
            if (spin[i] != spin[col[k]]) {
                cw2 += w[k];
                ce2 += 1;
            }
        }
    }
    /* every undirected edge is seen from both endpoints */
    *cut_w = cw2 / 2;
    *cut_edges = ce2 / 2;
    *mag = m;
}

/* E = A M^2 + B cut_w (eq. 4 with eq. 5 and the weighted eq. 6). */
int64_t oracle_energy(int32_t n, const int32_t *row_ptr, const int32_t *col, const int32_t *w,
                      const int8_t *spin, int64_t A, int64_t B)
{
    int64_t cw, ce, m;
    oracle_cut(n, row_ptr, col, w, spin, &cw, &ce, &m);
    return A * m * m + B * cw;
}

/* Exact single-flip energy change of node i against the true magnetisation. */
int64_t oracle_flip_delta(int32_t n, const int32_t *row_ptr, const int32_t *col, const int32_t *w,
                          const int8_t *spin, int64_t A, int64_t B, int32_t i)
{
    int64_t h = 0, m = 0;
    for (int32_t j = 0; j < n; ++j) m += spin[j];
    for (int32_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) h += (int64_t)w[k] * spin[col[k]];
    return B * spin[i] * h + 4 * A * (1 - spin[i] * m);
}

/* ---------------------------------------------------------------- annealer */

typedef struct {
    int32_t A, B;
    int32_t mode;          /* OR_MODE_GATED or OR_MODE_SNAPSHOT */
    int32_t n_sweeps;      /* S: length of T */
    int32_t start_sweep;   /* first sweep to run (resume) */
    uint32_t replica;
    int32_t n_threads;     /* OpenMP threads for the decision loop (<= 0: runtime default) */
    int32_t rule;          /* OR_RULE_METROPOLIS, or OR_RULE_PAPER: T holds flip probabilities */
    uint64_t seed;
} oracle_params;

/*
 * Runs sweeps start_sweep .. n_sweeps-1.
 *   T           n_sweeps temperatures (FP64)
 *   init        n spins to start from, or NULL for the Philox initial state
 *   spins_out   n spins, final state
 *   trace_m/trace_cut  optional, n_sweeps entries: M and cut after sweep t
 *   phase_m/phase_cut  optional, n_sweeps*C entries: M and cut after each phase
 *   phase_spins optional, n_sweeps*C*n spins after each phase (small n only)
 *   result[0..4] = final M, final cut (tracked), number of colours, total flips,
 *                  wall time of the sweep loop in nanoseconds (timing only)
 *   skip        optional, n bytes: a node with a non-zero byte makes no decision in
 *               these sweeps (it keeps its spin and draws nothing) but still counts
 *               in M and in its class's over-side count
 *   last_flip   optional, n entries, updated in place: the sweep of each node's last flip
 */
int oracle_anneal(int32_t n, const int32_t *row_ptr, const int32_t *col, const int32_t *w,
                  const double *T, const oracle_params *p, const int8_t *init,
                  int8_t *spins_out, int64_t *trace_m, int64_t *trace_cut,
                  int64_t *phase_m, int64_t *phase_cut, int8_t *phase_spins,
                  int64_t *result, const uint8_t *skip, int32_t *last_flip)
{
    if (n < 2 || p->n_sweeps < 1 || p->start_sweep < 0 || p->start_sweep > p->n_sweeps)
        return OR_EINVAL;
    if (p->rule != OR_RULE_METROPOLIS && p->rule != OR_RULE_PAPER) return OR_EINVAL;
    for (int32_t t = 0; t < p->n_sweeps; ++t)
        if (p->rule == OR_RULE_PAPER ? !(T[t] >= 0.0 && T[t] <= 1.0) : !(T[t] > 0.0)) return OR_EINVAL;

    const int64_t A = p->A, B = p->B;
    const uint32_t k0 = (uint32_t)p->seed, k1 = (uint32_t)(p->seed >> 32);
    int rc = OR_OK;
    int32_t *colour = NULL, *members = NULL;
    int8_t *s = NULL;
    int64_t *cls_off = NULL, *fill = NULL, *P = NULL, *hval = NULL;
    uint8_t *flip = NULL;
    uint32_t *thr = NULL;

    colour = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    s = (int8_t *)malloc((size_t)n);
    if (!colour || !s) { rc = OR_ENOMEM; goto done; }
    const int32_t C = oracle_colour(n, row_ptr, col, colour);
    if (C < 0) { rc = C; goto done; }

    /* members of each class, ascending id */
    cls_off = (int64_t *)calloc((size_t)C + 1, sizeof(int64_t));
    members = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    fill = (int64_t *)calloc((size_t)C, sizeof(int64_t));
    P = (int64_t *)calloc((size_t)C, sizeof(int64_t));
    hval = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    flip = (uint8_t *)malloc((size_t)n);
    if (!cls_off || !members || !fill || !P || !hval || !flip) { rc = OR_ENOMEM; goto done; }
    for (int32_t i = 0; i < n; ++i) cls_off[colour[i] + 1]++;
    for (int32_t c = 0; c < C; ++c) cls_off[c + 1] += cls_off[c];
    for (int32_t i = 0; i < n; ++i) members[cls_off[colour[i]] + fill[colour[i]]++] = i;

    /* largest possible |dE|: B * max weighted degree + 4A(n+1) */
    int64_t wmax = 0;
    for (int32_t i = 0; i < n; ++i) {
        int64_t a = 0;
        for (int32_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) a += llabs((long long)w[k]);
        if (a > wmax) wmax = a;
    }
    const int64_t de_max = B * wmax + 4 * A * ((int64_t)n + 1);

    /* initial state */
    for (int32_t i = 0; i < n; ++i) {
        if (init) {
            s[i] = init[i] > 0 ? 1 : -1;
        } else {
            uint32_t ctr[4] = {(uint32_t)i, 0u, p->replica, 1u}, x[4];
            oracle_philox4x32_10(k0, k1, ctr, x);
            s[i] = (x[0] & 1u) ? 1 : -1;
        }
    }
    int64_t M, cut, ce;
    oracle_cut(n, row_ptr, col, w, s, &cut, &ce, &M);
    for (int32_t i = 0; i < n; ++i)
        if (s[i] > 0) P[colour[i]]++;

    /* per-sweep threshold row, filled up to the last non-zero entry (or de_max) */
    int64_t thr_cap = 1024;
    thr = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(thr_cap + 1));
    if (!thr) { rc = OR_ENOMEM; goto done; }
    int64_t total_flips = 0;
    const double wall0 = omp_get_wtime();

    for (int32_t t = p->start_sweep; t < p->n_sweeps; ++t) {
        int64_t width = 0;
        /* the paper's rule draws one flip probability per sweep */
        const double pf_scaled = floor(ldexp(p->rule == OR_RULE_PAPER ? T[t] : 0.0, 32));
        const uint32_t pf_thr = pf_scaled >= 4294967295.0 ? 0xFFFFFFFFu : (uint32_t)pf_scaled;
        for (int64_t d = 1; d <= de_max && p->rule == OR_RULE_METROPOLIS; ++d) {
            uint32_t v = oracle_threshold(d, T[t]);
            if (v == 0) break;
            if (d > thr_cap) {
                thr_cap *= 2;
                uint32_t *nt = (uint32_t *)realloc(thr, sizeof(uint32_t) * (size_t)(thr_cap + 1));
                if (!nt) { rc = OR_ENOMEM; goto done; }
                thr = nt;
            }
            thr[d] = v;
            width = d;
        }

        for (int32_t c = 0; c < C; ++c) {
            const int64_t M0 = M;
            const int64_t sg = (M0 > 0) - (M0 < 0);
            const int64_t D = (M0 < 0 ? -M0 : M0) / 2;
            const int64_t csize = cls_off[c + 1] - cls_off[c];
            const int64_t O = sg > 0 ? P[c] : (sg < 0 ? csize - P[c] : 0);

            /* decisions: every node of the class reads the same pre-phase state */
            #pragma omp parallel for schedule(static) num_threads(p->n_threads > 0 ? p->n_threads : omp_get_max_threads())
            for (int64_t q = cls_off[c]; q < cls_off[c + 1]; ++q) {
                const int32_t i = members[q];
                if (skip && skip[i]) {
                    flip[q] = 0;
                    continue;
                }
                uint32_t ctr[4] = {(uint32_t)i, (uint32_t)t, p->replica, 0u}, x[4];
                oracle_philox4x32_10(k0, k1, ctr, x);
                int64_t h = 0;
                for (int32_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) h += (int64_t)w[k] * s[col[k]];
                const int64_t si = s[i];
                int64_t Mi;
                if (p->mode == OR_MODE_SNAPSHOT) {
                    Mi = M0;
                } else {
                    int gated = (si == sg) && ((uint64_t)x[1] * (uint64_t)O < ((uint64_t)D << 32));
                    Mi = gated ? M0 : 0;
                }
                const int64_t dE = B * si * h + 4 * A * (1 - si * Mi);
                int accept;
                if (p->rule == OR_RULE_PAPER) {
                    /* the energy-minimising value; a tie leaves it to word x2 */
                    const int64_t tie_value = (x[2] & 1u) ? 1 : -1;
                    const int argmin_flips = dE < 0 || (dE == 0 && tie_value != si);
                    accept = argmin_flips != (x[0] < pf_thr);
                } else if (dE <= 0) accept = 1;
                else if (dE > width) accept = 0;
                else accept = x[0] < thr[dE];
                flip[q] = (uint8_t)accept;
                hval[q] = h;
            }
            /* apply */
            for (int64_t q = cls_off[c]; q < cls_off[c + 1]; ++q) {
                if (!flip[q]) continue;
                const int32_t i = members[q];
                cut += (int64_t)s[i] * hval[q];
                M -= 2 * (int64_t)s[i];
                P[c] -= s[i];
                s[i] = (int8_t)-s[i];
                if (last_flip) last_flip[i] = t;
                total_flips++;
            }
            if (phase_m) phase_m[(int64_t)t * C + c] = M;
            if (phase_cut) phase_cut[(int64_t)t * C + c] = cut;
            if (phase_spins) memcpy(phase_spins + ((int64_t)t * C + c) * n, s, (size_t)n);
        }
        if (trace_m) trace_m[t] = M;
        if (trace_cut) trace_cut[t] = cut;
    }
    const double wall1 = omp_get_wtime();
    memcpy(spins_out, s, (size_t)n);
    if (result) {
        result[0] = M;
        result[1] = cut;
        result[2] = C;
        result[3] = total_flips;
        result[4] = (int64_t)((wall1 - wall0) * 1e9);
    }
done:
    free(thr);
    free(cls_off); free(members); free(fill); free(P); free(hval); free(flip);
    free(colour); free(s);
    return rc;
}

/* Largest number of OpenMP threads the oracle would use by default. */
int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
