/*
 * oracle.h -- plain, slow CPU oracle for the ternary flip-graph random walk
 * (Perminov, "Fast Matrix Multiplication via Ternary Meta Flip Graphs",
 * arXiv 2511.20317).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * includes this code; only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark use it.  It shares no code, header, table or
 * helper with the GPU path.
 *
 * Representation: every coefficient is one int8_t in {-1,0,1} (Z_T) or {0,1}
 * (Z2).  A scheme (m,n,p:r) is r terms u(l) (x) v(l) (x) w(l), paper Sec. 3.1,
 * flattened as in the worked (2,2,3:11) example of Sec. 3.1.1:
 *     u[i*n + j] <-> a_ij,   v[j*p + k] <-> b_jk,   w[k*m + i] <-> c_ik
 * (the C^T convention of Sec. 3.1).
 *
 * Every "reading" of a point on which the paper is silent is stated at the
 * function that takes it; the walk follows Algorithm 1 (RandomWalk kernel,
 * Sec. 3.4.2) in the paper's order.
 */
#ifndef TSF_ORACLE_H
#define TSF_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OR_MAXL 64   /* factor vectors fit one 64-bit mask in the paper (Sec. 3.5, 4.1) */
#define OR_MAXT 512  /* terms held by one oracle scheme */
#define OR_MAXREC 512

enum { OR_U = 0, OR_V = 1, OR_W = 2 };

typedef struct {
    int m, n, p;   /* format (m,n,p) */
    int r;         /* rank = number of live terms */
    int z2;        /* 0: ternary Z_T, 1: binary field Z2 */
    int8_t f[3][OR_MAXT][OR_MAXL]; /* f[X][l][e]: factor X of term l, entry e */
} or_scheme;

/* --- Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) ------------------- */
void or_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* --- schemes (Sec. 3.1, 3.3, 3.6) ----------------------------------------- */
int  or_len(const or_scheme *s, int X);
void or_standard(or_scheme *s, int m, int n, int p, int z2);
long or_brent_violations(const or_scheme *s);
long or_naive_additions(const or_scheme *s);
long or_nonzeros(const or_scheme *s);
void or_normalise_term(or_scheme *s, int l);
int  or_is_normalised(const or_scheme *s);
int  or_project(const or_scheme *in, int axis, int index, or_scheme *out);
int  or_extend(const or_scheme *in, int axis, or_scheme *out);
int  or_full_reduce(or_scheme *s);
int  or_swap_sizes(const or_scheme *in, or_scheme *out);
int  or_merge(const or_scheme *a, const or_scheme *b, int axis, or_scheme *out);
int  or_product(const or_scheme *a, const or_scheme *b, or_scheme *out);
int  or_resize(const or_scheme *s, const or_scheme *best, int n_best, uint64_t seed,
               int64_t round, uint64_t t_resize, int cap, or_scheme *out);
int  or_lift(const or_scheme *z2s, int64_t max_nodes, or_scheme *out, int64_t *nodes);

/* --- the walk (Algorithm 1) ------------------------------------------------ */
typedef struct {
    uint64_t seed;          /* walk seed = base seed + walk id                */
    int64_t  max_iters;     /* iteration budget of the walk                   */
    int64_t  plateau;       /* restart after this many iterations without a
                               strict improvement; <= 0 disables restarts     */
    int32_t  target_rank;   /* stop once best rank <= target                  */
    int32_t  r_cap;         /* expand refused when rank >= r_cap              */
    int32_t  flip_tries;    /* random flip attempts before the full search    */
    int32_t  restart_from_best;
    uint64_t t_eq;          /* Bernoulli thresholds: event iff word < t       */
    uint64_t t_reduce;
    uint64_t t_expand;
    int32_t  objective;     /* 0: rank (Algorithm 1); 1: naive additions at a
                               fixed rank (the complexity-minimisation mode of
                               Sec. 3.9); target_rank is then the target
                               number of naive additions                      */
    int32_t  pad;
} or_params;

typedef struct {
    int64_t iters, flips, attempts, fallbacks, dead_ends, zero_removed,
            merges, expands, expand_fails, restarts, eq_accepts, improvements;
} or_counters;

typedef struct {
    or_scheme cur, best, start;
    int32_t  best_rank;
    int32_t  done;
    int32_t  best_nnz;       /* non-zero coefficients of the best scheme       */
    int32_t  pad;
    int64_t  t;              /* iterations completed                          */
    int64_t  plateau_start;  /* iteration of the last strict improvement or restart */
    or_counters c;
    int32_t  n_rec;          /* strict improvements recorded (may exceed OR_MAXREC) */
    int64_t  rec_iter[OR_MAXREC];
    int32_t  rec_rank[OR_MAXREC];
} or_walk;

void or_walk_init(or_walk *w, const or_scheme *start);
void or_walk_run(or_walk *w, const or_params *prm, int64_t n_iters);

/* One logged iteration: the applied flip's two terms before the flip, in role
 * order (x_i, y_i, z_i, x_j, y_j, z_j), as (non-zero mask, minus mask) pairs;
 * rank before and after the iteration; rank_before = -1 without a flip. */
typedef struct {
    int64_t iter;
    int32_t rank_before, rank_after, format_slot, reserved;
    uint64_t f[12];
    uint64_t pad;
} or_log;

/* or_walk_run that also logs iteration t to log[t-1] while t <= log_cap */
void or_walk_run_logged(or_walk *w, const or_params *prm, int64_t n_iters, or_log *log,
                        int64_t log_cap, int32_t format_slot);

/* Walk with externally chosen proposals: at iteration t the first
 * prm->flip_tries attempts each yield their candidate (as in try_flip);
 * choices[t-1] names the attempt applied (255 = none had a candidate, then
 * the fallback search runs).  Counts choices that name an attempt without a
 * candidate, or 255 while one had a candidate, in *bad (the walk then stops).
 * choices covers iterations 1..n_choices. */
void or_walk_run_choices(or_walk *w, const or_params *prm, int64_t n_iters,
                         const uint8_t *choices, int64_t n_choices, int64_t *bad);

/* The candidate of flip attempt a at iteration t of a walk in state s: returns
 * the number of candidates of the attempt (0: none) and the chosen one. */
int or_attempt_candidate(const or_scheme *s, uint64_t seed, int64_t t, int a, int *pi, int *pj,
                         int *pX, int *prole);

/* run walks first_walk .. first_walk+n_walks-1 (seed = base_seed + walk id)
 * from one start scheme on n_threads host threads, n_iters iterations each */
void or_run_many(const or_scheme *start, const or_params *prm, uint64_t base_seed,
                 int64_t first_walk, int n_walks, int64_t n_iters, int n_threads,
                 or_walk *out);

/* single operators, exposed for the property and brute-force tests */
int or_flip(or_scheme *s, int i, int j, int X, int sigma, int role);
int or_flip_valid(const or_scheme *s, int i, int j, int X, int sigma, int role);
int or_plus(or_scheme *s, int i, int j, int perm);
int or_split(or_scheme *s, int i, int j, int perm);
int or_remove_zero_terms(or_scheme *s);
int or_ternary_add(const int8_t *a, const int8_t *b, int sign, int len, int z2, int8_t *out);

#ifdef __cplusplus
}
#endif
#endif
