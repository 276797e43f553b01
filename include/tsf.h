/*
 * tsf.h -- C ABI of the ternary flip-graph walk library (libtsf.so) for AMD
 * Instinct MI355X (gfx950).
 *
 * The library implements the hot path of the ternary meta flip graph method
 * (Perminov, "Fast Matrix Multiplication via Ternary Meta Flip Graphs",
 * arXiv 2511.20317): many independent random walks (Algorithm 1, Sec. 3.4.2)
 * over matrix multiplication schemes (m,n,p:r) whose coefficients lie in
 * Z_T = {-1,0,1} (Sec. 3.2) or in the binary field Z2 (Sec. 3.5).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Every function returns a tsf_status (0 = success, < 0 = error) and leaves
 *   a human-readable reason for the last error of the calling thread in
 *   tsf_last_error().  On error no output is modified unless stated.
 * - The library never allocates memory visible to the caller and never frees
 *   caller memory.  "host" pointers point to ordinary CPU memory, "device"
 *   pointers to GPU global memory (e.g. a torch CUDA/HIP tensor's data_ptr()).
 * - Scheme interchange (host, int8): a scheme (m,n,p:r) is r terms
 *   u(l) (x) v(l) (x) w(l) (Sec. 3.1).  Row l of U holds u(l) flattened as in
 *   the worked example of Sec. 3.1.1: a_ij -> i*n+j (length m*n); V: b_jk ->
 *   j*p+k (length n*p); W: c_ik -> k*m+i (length p*m, the C^T convention of
 *   Sec. 3.1).  Rows are stored back to back with no padding: U is
 *   capacity x (m*n) int8, V capacity x (n*p), W capacity x (p*m).  Rows at or
 *   beyond `rank` are ignored on input and zero-filled on output.
 * - Packed form (device and host): the one-bit representation of Sec. 3.5.1.
 *   Each factor vector is two uint64 masks, `digits` (bit e set iff entry e
 *   is non-zero) and `signs` (bit e set iff entry e is -1; always a subset of
 *   digits; zero in Z2).  A term is 6 uint64 words in the order
 *   u.digits, u.signs, v.digits, v.signs, w.digits, w.signs (48 bytes), and a
 *   packed scheme is `capacity` such terms.  Factor lengths are at most 64
 *   (Sec. 4.1 and 5.3).
 * - Walk results depend only on (parameters, base_seed, walk id, start
 *   scheme): never on the batch composition, the lanes-per-walk choice, the
 *   launch shape or how the iterations are split into calls.
 */
#ifndef TSF_H
#define TSF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TSF_OK = 0,
    TSF_E_ARG = -1,            /* null pointer, bad size or out-of-range argument    */
    TSF_E_FORMAT = -2,         /* a dimension < 1 or a factor length above 64        */
    TSF_E_CAPACITY = -3,       /* a scheme does not fit its capacity                 */
    TSF_E_NOT_TERNARY = -4,    /* a coefficient outside the mode's set, or signs
                                  not a subset of digits                             */
    TSF_E_INVALID_SCHEME = -5, /* the Brent equations do not hold                    */
    TSF_E_DEVICE = -6,         /* a HIP runtime call failed                          */
    TSF_E_STATE = -7           /* walk state inconsistent with the parameters        */
} tsf_status;

typedef enum { TSF_TERNARY = 0, TSF_Z2 = 1 } tsf_mode;

typedef struct {
    int32_t m, n, p;   /* format: A is m x n, B is n x p                        */
    int32_t rank;      /* number of live terms r                                */
    int32_t capacity;  /* rows allocated in U, V, W (>= rank)                   */
    int32_t mode;      /* tsf_mode                                              */
} tsf_dims;

typedef struct {
    tsf_dims d;
    int8_t *U, *V, *W; /* host, caller-owned, capacity rows each                */
} tsf_scheme;

/* Thread-local text of the last error reported on this thread. */
const char *tsf_last_error(void);

/* ------------------------------------------------------------------------ */
/* Host scheme operations                                                    */
/* ------------------------------------------------------------------------ */

/* The standard scheme of rank m*n*p: one term a_ij (x) b_jk (x) c_ik for every
 * (i,j,k), in lexicographic (i,j,k) order (the naive algorithm that Sec. 3.4.1
 * initialises populations with).  out->U/V/W must hold out->d.capacity >=
 * m*n*p rows; out->d's m, n, p, rank, mode are written.
 * Errors: TSF_E_FORMAT (dims < 1 or a factor length > 64), TSF_E_CAPACITY. */
tsf_status tsf_init_scheme(int32_t m, int32_t n, int32_t p, int32_t mode, tsf_scheme *out);

/* Brent equations (Eq. 1) in the C^T form of Sec. 3.1:
 *   sum_l u_l[a1*n+a2] v_l[b1*p+b2] w_l[c1*m+c2] = [a2=b1][b2=c1][c2=a1]
 * checked exactly over the integers (ternary) or modulo 2 (Z2).
 * *n_violated receives the number of equations that fail (0 = valid scheme).
 * Errors: TSF_E_ARG, TSF_E_FORMAT, TSF_E_NOT_TERNARY (entry outside the set). */
tsf_status tsf_verify(const tsf_scheme *s, int64_t *n_violated);

/* Sign-symmetry normalisation (Sec. 3.6), in place: per term, the first
 * non-zero entry of u and then of v is made positive, w absorbing each sign.
 * No-op in Z2.  Errors: TSF_E_ARG, TSF_E_FORMAT, TSF_E_NOT_TERNARY. */
tsf_status tsf_normalise(tsf_scheme *s);

/* Reduction operator (Sec. 3.3.1) applied to a fixpoint, in place: terms with
 * a zero factor are removed, then any two terms sharing two factors (w up to
 * sign) merge into one while the merged factor stays in the mode's set; the
 * result is normalised.  *n_reductions receives the number of merges.
 * Errors: TSF_E_ARG, TSF_E_FORMAT, TSF_E_NOT_TERNARY. */
tsf_status tsf_reduce(tsf_scheme *s, int32_t *n_reductions);

/* Project meta operator (Sec. 3.3.2): drop index `index` of `axis`
 * (0 = m, 1 = n, 2 = p) from every factor, remove the terms that became
 * zero, normalise.  out must have capacity >= in->d.rank.
 * Errors: TSF_E_ARG (axis/index out of range, dimension 1), TSF_E_CAPACITY. */
tsf_status tsf_meta_project(const tsf_scheme *in, int32_t axis, int32_t index, tsf_scheme *out);

/* Extend meta operator (Sec. 3.3.2): (m,n,p:r) -> (m,n,p+1:r+m*n) by
 * appending the naive (m,n,1) scheme for the new index (terms in (i,j)
 * order); along m the naive (1,n,p) scheme ((j,k) order, +n*p terms), along
 * n the naive (m,1,p) scheme ((i,k) order, +m*p terms).
 * Errors: TSF_E_ARG, TSF_E_FORMAT (a new length > 64), TSF_E_CAPACITY. */
tsf_status tsf_meta_extend(const tsf_scheme *in, int32_t axis, tsf_scheme *out);

/* Swap sizes meta operator (Sec. 3.3.2): (m,n,p:r) -> (m,p,n:r).  From
 * C^T = B^T A^T and the cyclic symmetry of the Brent equations in the C^T
 * layout: u' = w^T (m x p), v' = v^T (p x n), w' = u^T (n x m); terms
 * normalised.  out must have capacity >= rank.
 * Errors: TSF_E_ARG, TSF_E_FORMAT, TSF_E_NOT_TERNARY, TSF_E_CAPACITY. */
tsf_status tsf_meta_swap(const tsf_scheme *in, tsf_scheme *out);

/* Merge meta operator (Sec. 3.3.2): along axis 2 (m,n,p1:r1) + (m,n,p2:r2)
 * -> (m,n,p1+p2:r1+r2), C = A [B1 B2]; along axis 0 [A1; A2] B, along axis 1
 * [A1 A2][B1; B2].  The terms of a come first, b's indices shifted.
 * Errors: TSF_E_ARG (modes differ, the other two dimensions differ),
 * TSF_E_FORMAT (a factor over 64 entries), TSF_E_CAPACITY. */
tsf_status tsf_meta_merge(const tsf_scheme *a, const tsf_scheme *b, int32_t axis, tsf_scheme *out);

/* Product meta operator (Sec. 3.3.2): the Kronecker product, a scheme for
 * (m1 m2, n1 n2, p1 p2 : r1 r2); term l1*r2 + l2 = (u1 (x) u2, v1 (x) v2,
 * w1 (x) w2) with row i1*m2 + i2 and column j1*n2 + j2 in u (likewise v, w).
 * Errors: TSF_E_ARG, TSF_E_FORMAT, TSF_E_CAPACITY. */
tsf_status tsf_meta_product(const tsf_scheme *a, const tsf_scheme *b, tsf_scheme *out);

/* Ternary lifting (Sec. 3.10.1): signs for the non-zero coefficients of a Z2
 * scheme (entries 0/1, mode TSF_Z2) such that the Brent equations hold over
 * the integers.  An exhaustive search on the GPU: per term the first non-zero
 * entry of u and of v is +1 and the other non-zero entries (u ascending, then
 * v, then w) are the term's free signs, bit i of the term's pattern meaning
 * entry i is -1; assignments are ordered by the terms' patterns (term 0 most
 * significant); the search returns the first lifting in this order.  The
 * patterns of the leading terms split the space into at most max_subtrees
 * subtrees searched in parallel, each for at most max_nodes term
 * assignments.  res->status: 1 found (the first lifting in the order), 2
 * found (a valid lifting; a smaller subtree ran out of budget, so it may not
 * be the first), 0 no lifting exists (every subtree searched to the end), -1
 * unknown (none found, some subtree ran out of budget).  On 1 or 2, out
 * (host, capacity >= rank) receives the ternary scheme.  Synchronous; uses
 * the current device and temporary device memory.
 * Errors: TSF_E_ARG, TSF_E_FORMAT, TSF_E_NOT_TERNARY, TSF_E_CAPACITY (more
 * than 8192 equations, 512 terms or 40 free signs in a term), TSF_E_DEVICE. */
typedef struct {
    int32_t status;
    int32_t prefix_terms;      /* leading terms whose patterns name a subtree   */
    int64_t subtrees;
    int64_t exhausted;         /* subtrees searched to the end                  */
    int64_t subtree;           /* the subtree of the lifting returned, or -1    */
} tsf_lift_result;

tsf_status tsf_lift(const tsf_scheme *z2, int64_t max_nodes, int32_t max_subtrees,
                    tsf_scheme *out, tsf_lift_result *res);

/* Isotropy invariants (Sec. 3.7).  Each factor of term l is read as a matrix
 * (u: m x n, entry a_ij at row i, column j; v: n x p; w: p x m, entry c_ik at
 * row k, column i) and its rank taken over Q for ternary schemes, over GF(2)
 * for Z2 schemes; (a_l, b_l, c_l) are the ranks of term l's three factors
 * (each at most 8, since a factor has at most 64 entries).
 *   type polynomial      sum_l X^a_l Y^b_l Z^c_l        -> type_poly[a][b][c]
 *   symmetric polynomial sum over the permutations pi of (x,y,z) of
 *                        pi(sum_l x^a_l y^b_l z^c_l)    -> sym_poly[a][b][c]
 *   rank-sum polynomial  w^(sum a_l) + w^(sum b_l) + w^(sum c_l)
 *                                                        -> rank_sum[0..2]
 * (coefficients of the monomials; rank_sum holds the three exponents). */
typedef struct {
    int32_t rank_sum[3];
    int32_t type_poly[9][9][9];
    int32_t sym_poly[9][9][9];
} tsf_invariants;

/* Invariants of one scheme (host).  term_ranks (optional, host, rank x 3
 * bytes) receives (a_l, b_l, c_l) per term.
 * Errors: TSF_E_ARG, TSF_E_FORMAT, TSF_E_NOT_TERNARY. */
tsf_status tsf_scheme_invariants(const tsf_scheme *s, uint8_t *term_ranks, tsf_invariants *out);

/* int8 interchange <-> packed one-bit form (Sec. 3.5.1), host memory.
 * tsf_pack writes in->d.capacity terms (48 bytes each; rows >= rank zero).
 * tsf_unpack reads d->capacity packed terms into out (whose d is set to *d).
 * Errors: TSF_E_ARG, TSF_E_FORMAT, TSF_E_NOT_TERNARY (signs not within
 * digits, or bits beyond the factor length). */
tsf_status tsf_pack(const tsf_scheme *in, uint64_t *packed);
tsf_status tsf_unpack(const uint64_t *packed, const tsf_dims *d, tsf_scheme *out);

/* ------------------------------------------------------------------------ */
/* Batched random walks on the GPU (Algorithm 1, Sec. 3.4.2)                 */
/* ------------------------------------------------------------------------ */

/* Walk parameters.  Probabilities are integer thresholds on a 32-bit random
 * word: an event with probability p fires iff word < t, t = round(p * 2^32)
 * in [0, 2^32] (so 2^32 means "always"). */
typedef struct {
    uint64_t base_seed;        /* walk w draws from Philox4x32-10 keyed by
                                  base_seed + first_walk_id + w                   */
    int64_t  first_walk_id;    /* global id of the batch's walk 0                 */
    int64_t  max_iters;        /* iteration budget per walk                       */
    int64_t  plateau;          /* restart after this many iterations without a
                                  strict improvement of the best rank (<= 0: off) */
    int32_t  flip_tries;       /* random flip attempts per iteration (1..64)
                                  before the cyclic search over all (term, kind)
                                  pairs                                           */
    int32_t  restart_from_best;/* restart from the best scheme instead of the start */
    uint64_t t_eq;             /* accept an equal-rank scheme as best (Alg. 1: 0.01) */
    uint64_t t_reduce;         /* p_reduce of Alg. 1                              */
    uint64_t t_expand;         /* p_expand of Alg. 1                              */
    int32_t  objective;        /* TSF_OBJ_RANK or TSF_OBJ_ADDITIONS               */
    int32_t  reserved;
} tsf_walk_params;

/* Objectives of a walk.  TSF_OBJ_RANK: Algorithm 1 (the focused search of
 * Sec. 3.9).  TSF_OBJ_ADDITIONS: the complexity-minimisation mode of Sec. 3.9
 * (flips without reduction edges), scored by the naive additions of Sec. 4.5
 * (non-zero coefficients - 2r - mp): only flips that leave both modified
 * factors non-zero are candidates, so the rank never changes; there is no
 * reduce and no expand; the best scheme is replaced when the current one has
 * strictly fewer non-zero coefficients, or as many with probability t_eq; a
 * strict improvement is recorded (with its naive additions in the record's
 * rank field) and resets the plateau counter; the walk stops once the best
 * scheme's naive additions are at most target_rank.  t_reduce and t_expand
 * are ignored. */
#define TSF_OBJ_RANK 0
#define TSF_OBJ_ADDITIONS 1

/* Per-walk state header (device memory, one per walk, 176 bytes). */
typedef struct {
    int32_t m, n, p, mode;     /* the walk's format and coefficient set           */
    int32_t r_cap;             /* expand is refused at this rank (<= capacity)    */
    int32_t target_rank;       /* the walk stops once best_rank <= target_rank    */
    int32_t rank;              /* rank of the current scheme                      */
    int32_t best_rank;         /* rank of the best scheme                         */
    int32_t start_rank;        /* rank of the start scheme                        */
    int32_t done;              /* 1 once the target was reached; -1 header does
                                  not fit the batch; -2 invalid start scheme;
                                  -3 resumed with other walk parameters than the
                                  walk was run with (TSF_E_STATE); -4 an
                                  invariant check of tsf_walk_checked failed
                                  (error word in `reserved`)                     */
    int32_t n_rec;             /* strict improvements so far (records kept up to
                                  the batch's rec_cap)                            */
    int32_t best_nnz;          /* non-zero coefficients of the best scheme        */
    int64_t t;                 /* iterations completed                            */
    int64_t plateau_start;     /* iteration of the last strict improvement/restart */
    int64_t counters[12];      /* iters, flips, attempts, fallbacks, dead_ends,
                                  zero_removed, merges, expands, expand_fails,
                                  restarts, eq_accepts, improvements              */
    uint64_t params_hash;      /* tsf_params_hash of the parameters of the walk's
                                  last tsf_walk call; 0 after tsf_walk_init       */
    uint64_t reserved;         /* done = -4: (iteration << 8) | TSF_CHECK_* bits
                                  of the failed checks (iteration = t when the
                                  loaded state failed them); else unused          */
} tsf_walk_header;

/* One strict improvement of a walk's best rank (TSF_OBJ_ADDITIONS: of its
 * best naive additions). */
typedef struct {
    int64_t iter;              /* iteration at which it happened                 */
    int32_t rank;              /* the new best rank (or naive additions)         */
    int32_t reserved;
} tsf_record;

/* One logged walk iteration (128 bytes), for training the proposal network:
 * the flip applied at iteration `iter`, as the six factors of its two terms
 * before the flip in role order (x_i, y_i, z_i, x_j, y_j, z_j: x the shared
 * kind, y the kind that was added to, z the kind that was subtracted from),
 * each as a (digits, signs) pair, and the rank before and after the whole
 * iteration.  rank_before = -1 marks an iteration without a flip. */
typedef struct {
    int64_t iter;
    int32_t rank_before;
    int32_t rank_after;
    int32_t format_slot;       /* tsf_format_slot of the walk's format          */
    int32_t reserved;
    uint64_t f[12];
    uint64_t pad;
} tsf_flip_log;

/* Slot of a format in the proposal network's one-hot (0..14 for fifteen small
 * formats, independent of the order of m, n, p; 15 for any other). */
int32_t tsf_format_slot(int32_t m, int32_t n, int32_t p);

/* A batch of walks.  All buffers are device memory owned by the caller.
 * Walk w uses:  hdr[w];  cur, best, start: packed schemes of `capacity` terms
 * at offset w * capacity * 6 uint64;  rec: rec_cap records at w * rec_cap.
 * Walks of different formats and ranks may share one batch; a walk whose
 * header disagrees with the batch's mode or max_len, or does not fit its
 * capacity, is never advanced and gets done = -1. */
typedef struct {
    int32_t n_walks;
    int32_t capacity;          /* term slots per walk in cur/best/start (<= 512)  */
    int32_t rec_cap;           /* records kept per walk                           */
    int32_t mode;              /* tsf_mode shared by every walk of the batch      */
    int32_t max_len;           /* largest factor length of any walk (<= 64); 32
                                  or less selects the 32-bit kernels              */
    int32_t reserved;
    tsf_walk_header *hdr;
    uint64_t *cur;
    uint64_t *best;
    const uint64_t *start;
    tsf_record *rec;
    tsf_flip_log *log;         /* optional (NULL = off): log_cap records per walk;
                                  iteration t of walk w goes to w*log_cap + t-1
                                  while t <= log_cap (uniform proposals only)      */
    int32_t log_cap;
    int32_t reserved2;
} tsf_walk_batch;

/* Launch configuration.  strategy: 1 = attempt-parallel (each lane of a walk
 * evaluates a different random flip attempt; capacity <= 128 only),
 * 2 = term-parallel (the lanes of a walk split its terms; any capacity),
 * 3 = indexed attempt-parallel (strategy 1 over a match index kept in LDS:
 * per term and factor kind, a mask of the terms with an equal factor;
 * capacity <= 64 only).
 * lanes_per_walk: 4, 8, 16, 32 or 64 (16, 8, 4, 2 or 1 walks per 64-lane
 * wavefront; 4 to 32 for the attempt-parallel strategies, 8 to 64 for the
 * term-parallel one).  waves_per_block: 1..4.  A zero field lets the library
 * choose (a launch chosen by tsf_autotune for batches of this shape, else
 * strategy 3 with 8 lanes up to capacity 64, strategy 1 with 8 lanes up to
 * capacity 128 when max_len <= 32, strategy 2 with 64 lanes otherwise; one
 * wavefront per workgroup).
 * Results never depend on it. */
typedef struct {
    int32_t lanes_per_walk;
    int32_t waves_per_block;
    int32_t strategy;
} tsf_launch;

typedef struct tsf_ctx tsf_ctx;

/* Context: holds the autotuned launch table.  Not thread-safe per context. */
tsf_status tsf_ctx_create(tsf_ctx **ctx);
tsf_status tsf_ctx_destroy(tsf_ctx *ctx);

/* Autotuner: time every launch configuration that fits the batch (strategy,
 * lanes per walk, wavefronts per workgroup) for trial_iters iterations on a
 * private copy of the batch's state -- the batch itself is not changed -- and
 * remember the fastest for batches of the same capacity, max_len, mode and
 * size class; later tsf_walk calls with launch == NULL (or all fields 0) use
 * it.  The choice is also written to *chosen (may be NULL).  Results of walks
 * never depend on the configuration.  Synchronous.  The copy is allocated
 * inside the context and kept until tsf_ctx_destroy.
 * Errors: TSF_E_ARG, TSF_E_CAPACITY, TSF_E_DEVICE. */
tsf_status tsf_autotune(tsf_ctx *ctx, const tsf_walk_params *prm, const tsf_walk_batch *b,
                        int64_t trial_iters, tsf_launch *chosen, void *hip_stream);

/* Initialise every walk of the batch from its start scheme (device kernel):
 * cur := start, best := start, counters and records cleared.  Before the
 * call the caller fills, per walk, hdr[w].{m,n,p,mode,r_cap,target_rank,
 * start_rank} and the packed, normalised start scheme (tsf_pack of a scheme
 * passed through tsf_normalise).  Asynchronous on `hip_stream`.
 * Errors (checked on the host before launch): TSF_E_ARG, TSF_E_CAPACITY. */
tsf_status tsf_walk_init(tsf_ctx *ctx, const tsf_walk_batch *b, void *hip_stream);

/* Run up to n_iters further iterations of Algorithm 1 on every walk of the
 * batch (a walk stops early at its target rank or its iteration budget).
 * Random words (the paper leaves the sampling open): iteration t of a walk
 * uses Philox blocks (t, a, 0) for flip attempt a (term U(w0, r), kind
 * U(w1, 3), candidate U(w2, n) among the valid partners, role 0 then 1, j
 * ascending), the fourth words of blocks (t, 0, 0) and (t, 1, 0) for the
 * start pair and candidate of the cyclic search when every attempt failed,
 * (t, 0, 1) for the gates (equal-rank acceptance, reduce, expand) and
 * (t, a, 2) for expand attempt a; U(w, n) = floor(w * n / 2^32).  Results do
 * not depend on the launch configuration or on how iterations are split
 * into calls.
 * Asynchronous on `hip_stream`; `launch` may be NULL (library choice).
 * The host validates the batch shape against the chosen kernel.  Resuming:
 * a walk's header keeps the hash of the parameters it was last run with
 * (tsf_params_hash; everything but n_iters, which may differ per call); a
 * walk whose stored hash is neither 0 (fresh from tsf_walk_init) nor the
 * hash of `prm` is not advanced and gets done = -3, which tsf_walk_check
 * reports as TSF_E_STATE.  Errors: TSF_E_ARG, TSF_E_CAPACITY,
 * TSF_E_DEVICE. */
tsf_status tsf_walk(tsf_ctx *ctx, const tsf_walk_params *prm, const tsf_walk_batch *b,
                    int64_t n_iters, const tsf_launch *launch, void *hip_stream);

/* tsf_walk with the walk's invariants checked on the GPU after the scheme is
 * loaded and after every iteration -- a debugging aid for callers that want
 * a corrupted state (a damaged checkpoint, a kernel fault) to stop a walk at
 * once instead of producing schemes that only a later Brent check rejects.
 * The checks, on the terms below the rank: TSF_CHECK_RANK 1 <= rank <=
 * r_cap and best_rank <= start_rank; TSF_CHECK_ZERO_FACTOR no factor is
 * zero; TSF_CHECK_CODING signs only where digits are set (none in Z2) and no
 * entry beyond the factor's length; TSF_CHECK_NORMALISED the first non-zero
 * entry of u and of v is +1 (Sec. 3.6, ternary only); TSF_CHECK_INDEX (the
 * indexed strategy) every match mask equals the relation it indexes;
 * TSF_CHECK_DEAD_SLOTS (packed factors) the slots above the rank hold the
 * dead-slot word.  A walk that fails a check is not advanced further: its
 * header gets done = -4 and reserved = (t << 8) | the failed bits, and its
 * state is written back as it was at that point (not at all when the
 * loaded state failed).  Walks that pass every check end bit-identical to
 * tsf_walk with the same arguments.  Kernels exist for the library's
 * default launch shapes (strategy 0, 8 lanes per walk for the
 * attempt-parallel strategies, 64 for the term-parallel one, one
 * wavefront per workgroup); `launch` may be NULL or name one of them, else
 * TSF_E_ARG.  Slower than tsf_walk (the index check is quadratic in the
 * rank).  Errors as tsf_walk. */
#define TSF_CHECK_RANK 1u
#define TSF_CHECK_ZERO_FACTOR 2u
#define TSF_CHECK_CODING 4u
#define TSF_CHECK_NORMALISED 8u
#define TSF_CHECK_INDEX 16u
#define TSF_CHECK_DEAD_SLOTS 32u
tsf_status tsf_walk_checked(tsf_ctx *ctx, const tsf_walk_params *prm, const tsf_walk_batch *b,
                            int64_t n_iters, const tsf_launch *launch, void *hip_stream);

/* FNV-1a hash (64-bit) of the walk parameters that a resumed walk must keep:
 * base_seed, first_walk_id, max_iters, plateau, t_eq, t_reduce, t_expand,
 * flip_tries, restart_from_best, objective (each as its little-endian bytes,
 * in that order); never 0 (a hash of 0 is replaced by 1).  Host only. */
uint64_t tsf_params_hash(const tsf_walk_params *prm);

/* Resume check of a batch on the host (synchronous, for callers that resume
 * batches from checkpoints): `hdr` is a host copy of the batch's n_walks
 * headers.  Counts the walks whose stored parameter hash is neither 0 nor
 * tsf_params_hash(prm), or that a walk call already refused (done = -3),
 * into *n_mismatched (may be NULL).  Returns TSF_E_STATE if there is any,
 * TSF_E_ARG on null arguments or n_walks < 0, else TSF_OK.  Reads only the
 * headers; caller-owned memory. */
tsf_status tsf_walk_check(const tsf_walk_params *prm, const tsf_walk_header *hdr,
                          int32_t n_walks, int32_t *n_mismatched);

/* Host check of a batch's walk state before it is resumed, e.g. one read back
 * from a checkpoint, so that a damaged state is refused instead of walked.
 * hdr, cur, best, start: host copies of the batch's
 * n_walks headers and its three scheme buffers (capacity x 6 uint64 per walk,
 * the layout of tsf_walk_batch).  Walks flagged by a walk call (done < 0) are
 * skipped.  For every other walk, in order, the first failing check is
 * returned and its index written to *first_bad (may be NULL; -1 when all
 * pass): the format (TSF_E_FORMAT: dims >= 1, factors of at most 64
 * entries; TSF_E_ARG: mode neither ternary nor Z2); the ranks (TSF_E_CAPACITY:
 * 0 <= rank <= r_cap <= capacity, best and start ranks within the capacity);
 * the coding of the current, best and start schemes (TSF_E_NOT_TERNARY: signs
 * only under digits, none in Z2, no entry beyond a factor's length); with
 * check_brent != 0 their Brent equations (Eq. 1, TSF_E_INVALID_SCHEME) --
 * cheap for small formats; tsf_verify_batch does the same on the GPU.
 * Reads only caller-owned host memory; synchronous. */
tsf_status tsf_state_check(const tsf_walk_header *hdr, const uint64_t *cur, const uint64_t *best,
                           const uint64_t *start, int32_t n_walks, int32_t capacity,
                           int32_t check_brent, int32_t *first_bad);

/* Exact Brent verification (Eq. 1, C^T form of Sec. 3.1) on the GPU of one
 * scheme per walk of the batch: which = 0 checks cur (rank hdr[w].rank),
 * 1 checks best (hdr[w].best_rank), 2 checks start (hdr[w].start_rank).
 * n_violated (device, n_walks int64) receives the number of failed
 * equations per walk plus the number of mask bits that encode no
 * coefficient (a digit at or beyond the factor's length, a sign bit without
 * its digit, any sign bit of a Z2 scheme), so 0 = valid; -1 for a walk whose
 * header does not fit the batch.  Asynchronous on `hip_stream`.
 * Errors: TSF_E_ARG, TSF_E_DEVICE. */
tsf_status tsf_verify_batch(const tsf_walk_batch *b, int32_t which, int64_t *n_violated,
                            void *hip_stream);

/* Isotropy invariants (Sec. 3.7, see tsf_scheme_invariants) of the current
 * (which = 0), best (1) or start (2) scheme of every walk, on the GPU:
 * term_ranks (device, n_walks x capacity x 3 bytes) receives the factor ranks
 * (a_l, b_l, c_l) of each live term (slots past the scheme's rank are left
 * unchanged), rank_sums (device, n_walks x 3 int32) the three sums.  A walk
 * whose header does not fit the batch gets rank_sums -1.  Async on the
 * stream.  Errors: TSF_E_ARG, TSF_E_DEVICE. */
tsf_status tsf_invariants_batch(const tsf_walk_batch *b, int32_t which, uint8_t *term_ranks,
                                int32_t *rank_sums, void *hip_stream);

/* Population synchronisation (Sec. 3.4.1): the distinct formats among the
 * walks of a batch (walks flagged invalid excluded) and, per format, the walk
 * with the best rank (ties: the lowest walk id).  table (device, >= slots
 * entries) receives them in ascending (m, n, p) order, *n_entries (device)
 * their number.  work (device, 2*slots + 1 uint64) is scratch; slots
 * (1..4096) bounds the number of distinct formats (more are dropped and
 * counted in the last word of work).  Async on the stream.  Errors: TSF_E_ARG, TSF_E_DEVICE. */
typedef struct {
    int32_t m, n, p, rank;
    int64_t walk;
} tsf_best_entry;

tsf_status tsf_population_best(const tsf_walk_batch *b, tsf_best_entry *table, int32_t *n_entries,
                               uint64_t *work, int32_t slots, void *hip_stream);

/* tsf_population_best for callers that cannot allocate device memory (code
 * under HIP graph capture, serving loops, harnesses that forbid hipMalloc):
 * the same table from the same kernels, with no workspace argument.  The
 * working memory is a fixed array inside the library, 2*4096 + 1 uint64
 * (64 KiB) on each device it runs on, held until the process ends; slots is
 * limited to its size (1..4096, else TSF_E_ARG).  No call allocates or frees
 * memory.  Every call on a device uses that device's one array, and the
 * array keeps the last call's contents (each call clears what it reads):
 * calls that overlap on one device (two streams, two threads) race and must
 * be ordered by the caller.  dropped (optional, device int32) receives the
 * number of walks whose format did not fit `slots`.  Async on the stream.
 * Errors: TSF_E_ARG, TSF_E_DEVICE. */
tsf_status tsf_population_best_noalloc(const tsf_walk_batch *b, tsf_best_entry *table,
                                       int32_t *n_entries, int32_t slots, int32_t *dropped,
                                       void *hip_stream);

/* Resize (Algorithm 2, Sec. 3.4.3) of every walk, on the GPU: the current
 * (which = 0) or best (1) scheme of walk w of `in` becomes the start scheme
 * of walk w of `out` after: with probability 1/2 swap sizes; a merge with a
 * best scheme of the table (axes p, m, n: the first that exists and fits);
 * if there was none, with probability t_resize/2^32 one of project (5%),
 * product with a best scheme (50%), double (30%), extend (15%).  Random words:
 * Philox4x32-10 blocks b0 = (round, 0, 3) and b1 = (round, 1, 3) keyed by
 * base_seed + first_walk_id + w, U(x, n) = (x * n) >> 32:
 *   b0.w0 < 2^31           swap sizes, (m,n,p) -> (m,p,n) (before the rest);
 *   b0.w1                  merge partner table[U(b0.w1, n_entries)], axes
 *                          tried in the order p, m, n (the first that matches
 *                          and fits);
 *   b0.w2 < t_resize       (only without a merge) resize with one operator,
 *                          chosen by b0.w3 against round(0.05 * 2^32),
 *                          round(0.55 * 2^32), round(0.85 * 2^32): project /
 *                          product / double / extend;
 *   b1.w0                  product partner table[U(b1.w0, n_entries)];
 *   b1.w1                  axis U(b1.w1, 3) (0 = m, 1 = n, 2 = p) of project,
 *                          double and extend;
 *   b1.w2                  project index U(b1.w2, size of that axis).
 * An operator whose result would not fit (a factor over 64 entries, rank over
 * out->capacity), or a project of an axis of size 1, is skipped.  out->hdr[w] receives the format, mode, target,
 * start_rank and r_cap = min(start_rank + r_cap_extra, out->capacity);
 * follow with tsf_walk_init(out).  applied (optional, device, n_walks int32):
 * the operators applied, bit 0 swap, 1 merge, 2 project, 3 product, 4 double,
 * 5 extend (-1 for a walk that was skipped).  in and out are distinct
 * batches of equal n_walks; table and *n_entries as from tsf_population_best
 * on `in`.  Async on the stream.  Errors: TSF_E_ARG, TSF_E_DEVICE. */
typedef struct {
    uint64_t base_seed;
    int64_t first_walk_id;
    int64_t round;
    uint64_t t_resize;         /* p_resize of Alg. 2 as a threshold on 2^32     */
    int32_t r_cap_extra;
    int32_t reserved;
} tsf_resize_params;

tsf_status tsf_resize_batch(const tsf_walk_batch *in, int32_t which, const tsf_best_entry *table,
                            const int32_t *n_entries, const tsf_resize_params *prm,
                            const tsf_walk_batch *out, int32_t *applied, void *hip_stream);

/* Meta operators (Sec. 3.3.2) on every walk of a batch at once, on the GPU:
 * the current (which = 0) or best (which = 1) scheme of walk w of `in`
 * becomes the start scheme of walk w of `out`, after op[w]: 0 = copy,
 * 1 = project (drop index index[w] of axis axis[w], 0 = m, 1 = n, 2 = p, then
 * remove the terms that became zero, keeping the order of the others),
 * 2 = extend along axis[w] (append the naive scheme of the new index, as
 * tsf_meta_extend).  Every term is renormalised (Sec. 3.6).  out->hdr[w]
 * receives the new format, in's mode and target rank, start_rank and
 * r_cap = min(start_rank + r_cap_extra, out->capacity); a result that does
 * not fit out->capacity or 64-entry factors, or an invalid op, gets
 * start_rank = -1, which tsf_walk_init then flags.  op, axis, index: device
 * int32 arrays of n_walks.  in and out are distinct buffers of equal n_walks.
 * Follow with tsf_walk_init(out).  Async on the stream.
 * Errors: TSF_E_ARG, TSF_E_DEVICE. */
tsf_status tsf_meta_batch(const tsf_walk_batch *in, int32_t which, const int32_t *op,
                          const int32_t *axis, const int32_t *index, int32_t r_cap_extra,
                          const tsf_walk_batch *out, void *hip_stream);

/* Expand n log records into bf16 feature rows X (device, n x 512) of the
 * proposal network: entries 0..383 the six factors (64 entries each, +-1/0),
 * 384 + format_slot one-hot, 400 + min(rank_before, 95) one-hot, the rest 0.
 * Async on the stream.  Errors: TSF_E_ARG, TSF_E_DEVICE. */
tsf_status tsf_features_from_log(const tsf_flip_log *log, int64_t n, uint16_t *X,
                                 void *hip_stream);

/* ------------------------------------------------------------------------ */
/* Learned flip proposal: a scoring network run on the MFMA matrix cores     */
/* ------------------------------------------------------------------------ */

/* Not in the paper (its Sec. 5.4 names learned search as future work): a
 * multilayer perceptron that scores candidate flips so that a walk can try the
 * best-scored one first.  With X an M x 512 bf16 feature matrix:
 *   z1 = X W1 + b1, h1 = bf16(relu(z1)); z2 = h1 W2 + b2, h2 = bf16(relu(z2));
 *   logit = h2 . w3 + b3;  loss = mean(softplus(logit) - y logit).
 * bf16 operands, fp32 accumulation (MFMA).  Parameters are fp32 masters in one
 * vector: W1^T (256 x 512, row n = column n of W1), b1 (256), W2^T (256 x 256),
 * b2 (256), w3 (256), b3 (1, padded to 4).  bf16 compute copies: W1^T, W2^T,
 * W2 (256 x 256, for the backward pass) and w3. */
#define TSF_MLP_IN 512
#define TSF_MLP_HID 256
#define TSF_MLP_NPARAM 197380
#define TSF_MLP_NBF16 262400

typedef struct {
    float *param;      /* device, TSF_MLP_NPARAM fp32 masters                    */
    float *grad;       /* device, TSF_MLP_NPARAM (written by tsf_mlp_bwd)       */
    float *adam_m;     /* device, TSF_MLP_NPARAM Adam first moments             */
    float *adam_v;     /* device, TSF_MLP_NPARAM Adam second moments            */
    uint16_t *wbf;     /* device, TSF_MLP_NBF16 bf16 compute copies            */
} tsf_mlp;

/* Refresh the bf16 compute copies from the fp32 masters.  Async on the stream. */
tsf_status tsf_mlp_sync(const tsf_mlp *net, void *hip_stream);

/* Forward pass of M rows: X (device, M x 512 bf16, row-major) -> h1, h2
 * (device, M x 256 bf16 each, caller workspace) and logit (device, M fp32).
 * Async on the stream.  Errors: TSF_E_ARG, TSF_E_DEVICE. */
tsf_status tsf_mlp_fwd(const tsf_mlp *net, const uint16_t *X, int32_t M, uint16_t *h1,
                       uint16_t *h2, float *logit, void *hip_stream);

/* Backward pass of the mean binary cross-entropy against labels y (device, M
 * fp32 in {0,1}), using the forward's h1, h2, logit: writes every gradient into
 * net->grad (overwriting it) and the loss into *loss (device fp32).  d2, d1
 * (device, M x 256 bf16) and d3 (device, M fp32) are caller workspace.
 * Async on the stream.  Errors: TSF_E_ARG, TSF_E_DEVICE. */
tsf_status tsf_mlp_bwd(const tsf_mlp *net, const uint16_t *X, const float *y, int32_t M,
                       const uint16_t *h1, const uint16_t *h2, const float *logit, uint16_t *d2,
                       uint16_t *d1, float *d3, float *loss, void *hip_stream);

/* Walks with the learned proposal.  Each iteration: the first K = flip_tries
 * random attempts (K <= lanes_per_walk - 1, attempt-parallel strategy 1) each
 * yield their candidate flip exactly as with uniform proposals; the network
 * scores the K candidates (rows of the same feature layout as
 * tsf_features_from_log) and the walk applies the highest-scored one (ties:
 * the lower attempt).  If no attempt has a candidate the uniform fallback
 * search runs.  Everything else in the iteration is unchanged, so every scheme
 * is exact and verified as before.  The attempts counter grows by K per
 * iteration.  Workspace (device, caller-owned), R = 8 * n_walks rows:
 * cand R uint32, feat R x 512 bf16, h1 and h2 R x 256 bf16, logit R fp32.
 * choice (optional, device): choice_cap bytes per walk; the attempt applied at
 * iteration t (255 = fallback) goes to w*choice_cap + t-1 while t <= choice_cap.
 * Runs n_iters iterations (each a propose kernel, the network, an apply
 * kernel), asynchronous on `hip_stream`.  Errors: TSF_E_ARG, TSF_E_CAPACITY,
 * TSF_E_DEVICE. */
typedef struct {
    uint32_t *cand;
    uint16_t *feat;
    uint16_t *h1, *h2;
    float *logit;
    uint8_t *choice;
    int32_t choice_cap;
    int32_t reserved;
} tsf_learn_ws;

tsf_status tsf_walk_learned(tsf_ctx *ctx, const tsf_walk_params *prm, const tsf_walk_batch *b,
                            const tsf_mlp *net, const tsf_learn_ws *ws, int64_t n_iters,
                            const tsf_launch *launch, void *hip_stream);

/* One Adam step (Kingma & Ba 2015; step = 1, 2, ... for the bias correction)
 * on the fp32 masters from net->grad, then tsf_mlp_sync.  Async on the stream. */
tsf_status tsf_mlp_step(const tsf_mlp *net, float lr, float beta1, float beta2, float eps,
                        int32_t step, void *hip_stream);

#ifdef __cplusplus
}
#endif
#endif
