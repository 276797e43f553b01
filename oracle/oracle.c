/*
 * oracle.c -- plain CPU oracle of the ternary flip-graph random walk.
 * TEST INFRASTRUCTURE ONLY (see oracle.h).  Deliberately simple: int8 arrays,
 * linear scans, no bit tricks, no blocking or reordering of the steps.
 */
#include "oracle.h"

#include <pthread.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Philox4x32-10, from the published definition (Salmon et al., "Parallel    */
/* random numbers: as easy as 1, 2, 3", SC'11): ten rounds of two 32x32->64  */
/* multiplications with a Weyl-sequence key schedule.                        */
/* ------------------------------------------------------------------------ */
void or_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
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

/* The walk's random words.  Reading (the paper only says each scheme has its
 * own generator, Sec. 3.4.2): one Philox block per (iteration t, attempt a,
 * domain d), key = the 64-bit walk seed, counter = (t lo, t hi, a, d).
 * Domains: 0 flip attempts, 1 per-iteration gates, 2 expand attempts. */
static void draw(uint64_t seed, int64_t t, uint32_t a, uint32_t dom, uint32_t w[4])
{
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    uint32_t ctr[4] = { (uint32_t)(uint64_t)t, (uint32_t)((uint64_t)t >> 32), a, dom };
    or_philox(ctr, key, w);
}

/* uniform integer in [0, n): floor(word * n / 2^32) */
static int uniform_below(uint32_t word, int n)
{
    return (int)(((uint64_t)word * (uint64_t)(uint32_t)n) >> 32);
}

/* ------------------------------------------------------------------------ */
/* Schemes                                                                   */
/* ------------------------------------------------------------------------ */

/* lengths of the flattened factors: U is m x n, V is n x p, W is p x m (Sec. 3.1) */
int or_len(const or_scheme *s, int X)
{
    if (X == OR_U) return s->m * s->n;
    if (X == OR_V) return s->n * s->p;
    return s->p * s->m;
}

static int vec_zero(const int8_t *a, int len)
{
    for (int e = 0; e < len; ++e)
        if (a[e] != 0) return 0;
    return 1;
}

static int vec_eq(const int8_t *a, const int8_t *b, int len)
{
    for (int e = 0; e < len; ++e)
        if (a[e] != b[e]) return 0;
    return 1;
}

static int vec_neg_eq(const int8_t *a, const int8_t *b, int len)
{
    for (int e = 0; e < len; ++e)
        if (a[e] != -b[e]) return 0;
    return 1;
}

/* out = a + sign*b.  Ternary: valid iff every entry stays in {-1,0,1}
 * (the "valid" flag of the one-bit representation, Sec. 3.5.1-3.5.2).
 * Z2: addition modulo 2, always valid, sign ignored. */
int or_ternary_add(const int8_t *a, const int8_t *b, int sign, int len, int z2, int8_t *out)
{
    int ok = 1;
    for (int e = 0; e < len; ++e) {
        int x;
        if (z2) {
            x = (a[e] + b[e]) % 2;
        } else {
            x = a[e] + sign * b[e];
            if (x < -1 || x > 1) ok = 0;
        }
        out[e] = (int8_t)x;
    }
    return ok;
}

static void copy_term(or_scheme *s, int dst, int src)
{
    for (int X = 0; X < 3; ++X)
        memcpy(s->f[X][dst], s->f[X][src], OR_MAXL);
}

/* Standard rank-mnp scheme: one term a_ij (x) b_jk (x) c_ik for each (i,j,k),
 * in lexicographic (i,j,k) order. */
void or_standard(or_scheme *s, int m, int n, int p, int z2)
{
    memset(s, 0, sizeof(*s));
    s->m = m; s->n = n; s->p = p; s->z2 = z2;
    int l = 0;
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < n; ++j)
            for (int k = 0; k < p; ++k) {
                s->f[OR_U][l][i * n + j] = 1;
                s->f[OR_V][l][j * p + k] = 1;
                s->f[OR_W][l][k * m + i] = 1;
                ++l;
            }
    s->r = l;
}

/* Brent equations (Eq. 1) in the C^T form of Sec. 3.1: for every
 * a_{a1 a2}, b_{b1 b2} and c^T entry (c1,c2) = w[c1*m + c2],
 *     sum_l u_l[a1*n+a2] v_l[b1*p+b2] w_l[c1*m+c2] = [a2==b1][b2==c1][c2==a1].
 * Returns the number of violated equations (mod 2 in Z2). */
long or_brent_violations(const or_scheme *s)
{
    int m = s->m, n = s->n, p = s->p;
    long bad = 0;
    for (int a1 = 0; a1 < m; ++a1)
        for (int a2 = 0; a2 < n; ++a2)
            for (int b1 = 0; b1 < n; ++b1)
                for (int b2 = 0; b2 < p; ++b2)
                    for (int c1 = 0; c1 < p; ++c1)
                        for (int c2 = 0; c2 < m; ++c2) {
                            long sum = 0;
                            for (int l = 0; l < s->r; ++l)
                                sum += (long)s->f[OR_U][l][a1 * n + a2] *
                                       (long)s->f[OR_V][l][b1 * p + b2] *
                                       (long)s->f[OR_W][l][c1 * m + c2];
                            long want = (a2 == b1 && b2 == c1 && c2 == a1) ? 1 : 0;
                            if (s->z2) {
                                if (((sum % 2) + 2) % 2 != want) ++bad;
                            } else if (sum != want) {
                                ++bad;
                            }
                        }
    return bad;
}

/* Naive additive complexity (Sec. 4.5): non-zero coefficients - 2r - m*p. */
long or_nonzeros(const or_scheme *s)
{
    long nnz = 0;
    for (int X = 0; X < 3; ++X)
        for (int l = 0; l < s->r; ++l)
            for (int e = 0; e < or_len(s, X); ++e)
                if (s->f[X][l][e] != 0) ++nnz;
    return nnz;
}

/* Naive additive complexity (Sec. 4.5): non-zero coefficients - 2r - mp. */
long or_naive_additions(const or_scheme *s)
{
    return or_nonzeros(s) - 2L * s->r - (long)s->m * s->p;
}

/* Sign-symmetry normalisation (Sec. 3.6).  Reading, fixed by the worked
 * (2,2,2:7) example there: per term (row), the first non-zero entry (lowest
 * flattened index) of u and then of v is made positive; w absorbs each sign
 * change (alpha*beta*gamma = 1).  w itself is never normalised.  No-op in Z2. */
void or_normalise_term(or_scheme *s, int l)
{
    if (s->z2) return;
    for (int X = OR_U; X <= OR_V; ++X) {
        int len = or_len(s, X);
        for (int e = 0; e < len; ++e) {
            if (s->f[X][l][e] == 0) continue;
            if (s->f[X][l][e] < 0) {
                for (int q = 0; q < len; ++q) s->f[X][l][q] = (int8_t)-s->f[X][l][q];
                int lw = or_len(s, OR_W);
                for (int q = 0; q < lw; ++q) s->f[OR_W][l][q] = (int8_t)-s->f[OR_W][l][q];
            }
            break;
        }
    }
}

int or_is_normalised(const or_scheme *s)
{
    if (s->z2) return 1;
    for (int l = 0; l < s->r; ++l)
        for (int X = OR_U; X <= OR_V; ++X)
            for (int e = 0; e < or_len(s, X); ++e)
                if (s->f[X][l][e] != 0) {
                    if (s->f[X][l][e] < 0) return 0;
                    break;
                }
    return 1;
}

/* swap-remove: the last term moves into slot h.  Tracked indices follow the
 * move; a tracked index equal to h is dropped (-1). */
static void swap_remove(or_scheme *s, int h, int *track, int n_track)
{
    int last = s->r - 1;
    for (int q = 0; q < n_track; ++q)
        if (track[q] == h) track[q] = -1;
    if (h != last) {
        copy_term(s, h, last);
        for (int q = 0; q < n_track; ++q)
            if (track[q] == last) track[q] = h;
    }
    memset(s->f[OR_U][last], 0, OR_MAXL);
    memset(s->f[OR_V][last], 0, OR_MAXL);
    memset(s->f[OR_W][last], 0, OR_MAXL);
    s->r -= 1;
}

static int term_has_zero_factor(const or_scheme *s, int l)
{
    for (int X = 0; X < 3; ++X)
        if (vec_zero(s->f[X][l], or_len(s, X))) return 1;
    return 0;
}

/* Remove every term with a zero factor, highest index first (swap-remove). */
int or_remove_zero_terms(or_scheme *s)
{
    int removed = 0;
    for (int l = s->r - 1; l >= 0; --l)
        if (term_has_zero_factor(s, l)) {
            swap_remove(s, l, NULL, 0);
            ++removed;
        }
    return removed;
}

/* the two factor kinds other than X, in U<V<W order, swapped when role = 1 */
static void other_kinds(int X, int role, int *Y, int *Z)
{
    int a, b;
    if (X == OR_U) { a = OR_V; b = OR_W; }
    else if (X == OR_V) { a = OR_U; b = OR_W; }
    else { a = OR_U; b = OR_V; }
    if (role) { *Y = b; *Z = a; } else { *Y = a; *Z = b; }
}

/* Flip (Sec. 3.3.1) of the ordered pair (i,j) sharing factor X up to the sign
 * sigma (x_j = sigma*x_i), with (Y,Z) the other two kinds:
 *   x_i(x)y_i(x)z_i + x_j(x)y_j(x)z_j
 *     -> x_i(x)(y_i + sigma*y_j)(x)z_i + x_j(x)y_j(x)(z_j - z_i).
 * The paper writes sigma = +1 with (Y,Z) = (V,W); every permutation of the
 * roles is allowed (Sec. 3.3.1) and, since w keeps its sign freedom after
 * normalisation (Sec. 3.6), sigma = -1 occurs for X = W.
 * Returns 1 if both new factors are ternary-valid (Sec. 3.5.2). */
int or_flip_valid(const or_scheme *s, int i, int j, int X, int sigma, int role)
{
    int Y, Z;
    int8_t tmp[OR_MAXL] = { 0 };
    other_kinds(X, role, &Y, &Z);
    if (!or_ternary_add(s->f[Y][i], s->f[Y][j], sigma, or_len(s, Y), s->z2, tmp)) return 0;
    if (!or_ternary_add(s->f[Z][j], s->f[Z][i], -1, or_len(s, Z), s->z2, tmp)) return 0;
    return 1;
}

int or_flip(or_scheme *s, int i, int j, int X, int sigma, int role)
{
    int Y, Z;
    int8_t ny[OR_MAXL] = { 0 }, nz[OR_MAXL] = { 0 };
    other_kinds(X, role, &Y, &Z);
    if (!or_ternary_add(s->f[Y][i], s->f[Y][j], sigma, or_len(s, Y), s->z2, ny)) return 0;
    if (!or_ternary_add(s->f[Z][j], s->f[Z][i], -1, or_len(s, Z), s->z2, nz)) return 0;
    memcpy(s->f[Y][i], ny, OR_MAXL);
    memcpy(s->f[Z][j], nz, OR_MAXL);
    or_normalise_term(s, i);
    or_normalise_term(s, j);
    return 1;
}

/* sign relating factor X of terms i and j: +1 if equal, -1 if negated
 * (only for W, Sec. 3.6, and never in Z2), 0 otherwise */
static int shared_sign(const or_scheme *s, int i, int j, int X)
{
    int len = or_len(s, X);
    if (vec_eq(s->f[X][j], s->f[X][i], len)) return 1;
    if (!s->z2 && X == OR_W && vec_neg_eq(s->f[X][j], s->f[X][i], len)) return -1;
    return 0;
}

/* role permutations (X,Y,Z) of (U,V,W) in lexicographic order */
static const int PERMS[6][3] = {
    { OR_U, OR_V, OR_W }, { OR_U, OR_W, OR_V }, { OR_V, OR_U, OR_W },
    { OR_V, OR_W, OR_U }, { OR_W, OR_U, OR_V }, { OR_W, OR_V, OR_U },
};

/* Plus (Sec. 3.3.1), roles (X,Y,Z) = PERMS[perm]:
 *   x_i(x)y_i(x)z_i + x_j(x)y_j(x)z_j
 *     -> x_i(x)(y_i+y_j)(x)z_i + x_i(x)y_j(x)(z_j-z_i) + (x_j-x_i)(x)y_j(x)z_j,
 * allowed when x_i!=x_j, y_i!=y_j, z_i!=z_j.  Reading: also every new factor
 * must be ternary-valid and y_i+y_j non-zero.  The third term is appended. */
int or_plus(or_scheme *s, int i, int j, int perm)
{
    int X = PERMS[perm][0], Y = PERMS[perm][1], Z = PERMS[perm][2];
    int lx = or_len(s, X), ly = or_len(s, Y), lz = or_len(s, Z);
    int8_t a[OR_MAXL] = { 0 }, b[OR_MAXL] = { 0 }, c[OR_MAXL] = { 0 };
    if (s->r >= OR_MAXT) return 0;
    if (vec_eq(s->f[X][i], s->f[X][j], lx) || vec_eq(s->f[Y][i], s->f[Y][j], ly) ||
        vec_eq(s->f[Z][i], s->f[Z][j], lz))
        return 0;
    if (!or_ternary_add(s->f[Y][i], s->f[Y][j], 1, ly, s->z2, a) || vec_zero(a, ly)) return 0;
    if (!or_ternary_add(s->f[Z][j], s->f[Z][i], -1, lz, s->z2, b)) return 0;
    if (!or_ternary_add(s->f[X][j], s->f[X][i], -1, lx, s->z2, c)) return 0;
    int nw = s->r;
    memset(s->f[OR_U][nw], 0, OR_MAXL);
    memset(s->f[OR_V][nw], 0, OR_MAXL);
    memset(s->f[OR_W][nw], 0, OR_MAXL);
    memcpy(s->f[X][nw], c, OR_MAXL);
    memcpy(s->f[Y][nw], s->f[Y][j], OR_MAXL);
    memcpy(s->f[Z][nw], s->f[Z][j], OR_MAXL);
    memcpy(s->f[X][j], s->f[X][i], OR_MAXL);
    memcpy(s->f[Z][j], b, OR_MAXL);
    memcpy(s->f[Y][i], a, OR_MAXL);
    s->r += 1;
    or_normalise_term(s, i);
    or_normalise_term(s, j);
    or_normalise_term(s, nw);
    return 1;
}

/* Split (Sec. 3.3.1), X = PERMS[perm][0]:
 *   x_i(x)y_i(x)z_i + x_j(x)y_j(x)z_j
 *     -> x_j(x)y_i(x)z_i + x_j(x)y_j(x)z_j + (x_i-x_j)(x)y_i(x)z_i,
 * allowed when x_i != x_j; reading: x_i-x_j must be ternary-valid. */
int or_split(or_scheme *s, int i, int j, int perm)
{
    int X = PERMS[perm][0];
    int lx = or_len(s, X);
    int8_t c[OR_MAXL] = { 0 };
    if (s->r >= OR_MAXT) return 0;
    if (vec_eq(s->f[X][i], s->f[X][j], lx)) return 0;
    if (!or_ternary_add(s->f[X][i], s->f[X][j], -1, lx, s->z2, c)) return 0;
    int nw = s->r;
    copy_term(s, nw, i);
    memcpy(s->f[X][nw], c, OR_MAXL);
    memcpy(s->f[X][i], s->f[X][j], OR_MAXL);
    s->r += 1;
    or_normalise_term(s, i);
    or_normalise_term(s, j);
    or_normalise_term(s, nw);
    return 1;
}

/* Reduction (Sec. 3.3.1): terms t and k sharing two factors merge into one.
 * The shared pair is tried in the order (U,V)->merge W, (U,W)->merge V,
 * (V,W)->merge U; w may be shared up to sign (Sec. 3.6), u and v only
 * exactly.  On success returns the merged kind and writes the merged factor
 * into out; returns -1 if no ternary-valid merge exists for the pair. */
static int merge_candidate(const or_scheme *s, int t, int k, int8_t *out)
{
    int lu = or_len(s, OR_U), lv = or_len(s, OR_V), lw = or_len(s, OR_W);
    int eq_u = vec_eq(s->f[OR_U][k], s->f[OR_U][t], lu);
    int eq_v = vec_eq(s->f[OR_V][k], s->f[OR_V][t], lv);
    int sg_w = shared_sign(s, t, k, OR_W);
    if (eq_u && eq_v) {
        /* u(x)v(x)w_t + u(x)v(x)w_k = u(x)v(x)(w_t + w_k) */
        if (or_ternary_add(s->f[OR_W][t], s->f[OR_W][k], 1, lw, s->z2, out)) return OR_W;
    }
    if (eq_u && sg_w != 0) {
        /* u(x)v_t(x)w + u(x)v_k(x)(sg*w) = u(x)(v_t + sg*v_k)(x)w */
        if (or_ternary_add(s->f[OR_V][t], s->f[OR_V][k], sg_w, lv, s->z2, out)) return OR_V;
    }
    if (eq_v && sg_w != 0) {
        if (or_ternary_add(s->f[OR_U][t], s->f[OR_U][k], sg_w, lu, s->z2, out)) return OR_U;
    }
    return -1;
}

/* Reduce the tracked (modified) terms against every other term, cascading:
 * for each tracked term in order, scan k = 0..r-1 ascending for the first
 * pair with a valid merge; the merged term goes to slot min(t,k), slot
 * max(t,k) is swap-removed, and the scan restarts on the merged term.  A
 * merged factor of zero removes both terms (higher slot first).  Returns the
 * number of merges. */
static int reduce_tracked(or_scheme *s, int *track, int n_track)
{
    int merges = 0;
    int8_t merged[OR_MAXL] = { 0 };
    for (int q = 0; q < n_track; ++q) {
        for (;;) {
            int t = track[q];
            if (t < 0) break;
            int k, kind = -1;
            for (k = 0; k < s->r; ++k) {
                if (k == t) continue;
                kind = merge_candidate(s, t, k, merged);
                if (kind >= 0) break;
            }
            if (kind < 0) break;
            ++merges;
            int lo = t < k ? t : k, hi = t < k ? k : t;
            for (int o = 0; o < n_track; ++o)
                if (o != q && track[o] == k) track[o] = -1;
            if (vec_zero(merged, or_len(s, kind))) {
                /* both terms cancel; lo < hi <= r-1, so removing hi first
                 * never moves lo */
                track[q] = -1;
                swap_remove(s, hi, track, n_track);
                swap_remove(s, lo, track, n_track);
                break;
            }
            if (lo != t) copy_term(s, lo, t);
            memcpy(s->f[kind][lo], merged, OR_MAXL);
            or_normalise_term(s, lo);
            track[q] = lo;
            swap_remove(s, hi, track, n_track);
        }
    }
    return merges;
}

/* Full reduction pass used for imported schemes: remove zero terms, then
 * treat every term as modified and reduce to a fixpoint. */
int or_full_reduce(or_scheme *s)
{
    int total = 0;
    or_remove_zero_terms(s);
    for (int l = 0; l < s->r; ++l) or_normalise_term(s, l);
    for (;;) {
        int merged = 0;
        for (int l = 0; l < s->r; ++l) {
            int tr[1] = { l };
            int got = reduce_tracked(s, tr, 1);
            if (got) { merged += got; break; }
        }
        if (!merged) break;
        total += merged;
    }
    return total;
}

/* ------------------------------------------------------------------------ */
/* Meta operators (Sec. 3.3.2)                                               */
/* ------------------------------------------------------------------------ */

/* Project (m,n,p) -> one dimension smaller: drop index `index` of axis
 * (0 = m, 1 = n, 2 = p) from every factor it appears in, then remove the
 * terms that became zero (the others keep their order). */
int or_project(const or_scheme *in, int axis, int index, or_scheme *out)
{
    int m = in->m, n = in->n, p = in->p;
    int dims[3] = { m, n, p };
    if (axis < 0 || axis > 2 || index < 0 || index >= dims[axis] || dims[axis] < 2) return -1;
    int m2 = m - (axis == 0), n2 = n - (axis == 1), p2 = p - (axis == 2);
    memset(out, 0, sizeof(*out));
    out->m = m2; out->n = n2; out->p = p2; out->z2 = in->z2; out->r = in->r;
    for (int l = 0; l < in->r; ++l) {
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < n; ++j) {
                if ((axis == 0 && i == index) || (axis == 1 && j == index)) continue;
                int i2 = i - (axis == 0 && i > index), j2 = j - (axis == 1 && j > index);
                out->f[OR_U][l][i2 * n2 + j2] = in->f[OR_U][l][i * n + j];
            }
        for (int j = 0; j < n; ++j)
            for (int k = 0; k < p; ++k) {
                if ((axis == 1 && j == index) || (axis == 2 && k == index)) continue;
                int j2 = j - (axis == 1 && j > index), k2 = k - (axis == 2 && k > index);
                out->f[OR_V][l][j2 * p2 + k2] = in->f[OR_V][l][j * p + k];
            }
        for (int k = 0; k < p; ++k)
            for (int i = 0; i < m; ++i) {
                if ((axis == 2 && k == index) || (axis == 0 && i == index)) continue;
                int k2 = k - (axis == 2 && k > index), i2 = i - (axis == 0 && i > index);
                out->f[OR_W][l][k2 * m2 + i2] = in->f[OR_W][l][k * m + i];
            }
    }
    /* drop the terms that became zero, keeping the order of the others */
    int kept = 0;
    for (int l = 0; l < out->r; ++l) {
        if (term_has_zero_factor(out, l)) continue;
        if (kept != l) copy_term(out, kept, l);
        ++kept;
    }
    for (int l = kept; l < out->r; ++l) {
        memset(out->f[OR_U][l], 0, OR_MAXL);
        memset(out->f[OR_V][l], 0, OR_MAXL);
        memset(out->f[OR_W][l], 0, OR_MAXL);
    }
    out->r = kept;
    for (int l = 0; l < out->r; ++l) or_normalise_term(out, l);
    return 0;
}

/* Extend (Sec. 3.3.2): (m,n,p:r) -> (m,n,p+1:r+mn) by appending the naive
 * (m,n,1) scheme for the new index, terms in (i,j) order; likewise along m
 * (+np terms, (j,k) order) and n (+mp terms, (i,k) order). */
int or_extend(const or_scheme *in, int axis, or_scheme *out)
{
    int m = in->m, n = in->n, p = in->p;
    if (axis < 0 || axis > 2) return -1;
    int m2 = m + (axis == 0), n2 = n + (axis == 1), p2 = p + (axis == 2);
    if (m2 * n2 > OR_MAXL || n2 * p2 > OR_MAXL || p2 * m2 > OR_MAXL) return -1;
    int extra = axis == 0 ? n * p : axis == 1 ? m * p : m * n;
    if (in->r + extra > OR_MAXT) return -1;
    memset(out, 0, sizeof(*out));
    out->m = m2; out->n = n2; out->p = p2; out->z2 = in->z2; out->r = in->r;
    for (int l = 0; l < in->r; ++l) {
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < n; ++j) out->f[OR_U][l][i * n2 + j] = in->f[OR_U][l][i * n + j];
        for (int j = 0; j < n; ++j)
            for (int k = 0; k < p; ++k) out->f[OR_V][l][j * p2 + k] = in->f[OR_V][l][j * p + k];
        for (int k = 0; k < p; ++k)
            for (int i = 0; i < m; ++i) out->f[OR_W][l][k * m2 + i] = in->f[OR_W][l][k * m + i];
    }
    int l = in->r;
    if (axis == 2) {
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < n; ++j, ++l) {
                out->f[OR_U][l][i * n2 + j] = 1;
                out->f[OR_V][l][j * p2 + p] = 1;
                out->f[OR_W][l][p * m2 + i] = 1;
            }
    } else if (axis == 0) {
        for (int j = 0; j < n; ++j)
            for (int k = 0; k < p; ++k, ++l) {
                out->f[OR_U][l][m * n2 + j] = 1;
                out->f[OR_V][l][j * p2 + k] = 1;
                out->f[OR_W][l][k * m2 + m] = 1;
            }
    } else {
        for (int i = 0; i < m; ++i)
            for (int k = 0; k < p; ++k, ++l) {
                out->f[OR_U][l][i * n2 + n] = 1;
                out->f[OR_V][l][n * p2 + k] = 1;
                out->f[OR_W][l][k * m2 + i] = 1;
            }
    }
    out->r = l;
    return 0;
}

/* Swap sizes (Sec. 3.3.2): (m,n,p:r) -> (m,p,n:r).  C^T = B^T A^T turns a
 * scheme for (m,n,p) into one for (p,n,m) (u' = v^T, v' = u^T, w' = w^T as
 * matrices), and rotating the factors (u,v,w) -> (v,w,u) turns a scheme for
 * (m,n,p) into one for (n,p,m) (the C^T layout makes the Brent equations
 * cyclic); the transpose followed by two rotations gives (m,p,n) with
 * u'' = w^T (m x p), v'' = v^T (p x n), w'' = u^T (n x m).  Terms renormalised. */
int or_swap_sizes(const or_scheme *in, or_scheme *out)
{
    int m = in->m, n = in->n, p = in->p;
    memset(out, 0, sizeof(*out));
    out->m = m; out->n = p; out->p = n; out->z2 = in->z2; out->r = in->r;
    for (int l = 0; l < in->r; ++l) {
        for (int k = 0; k < p; ++k)          /* w: p x m, entry (k, i) */
            for (int i = 0; i < m; ++i) out->f[OR_U][l][i * p + k] = in->f[OR_W][l][k * m + i];
        for (int j = 0; j < n; ++j)          /* v: n x p, entry (j, k) */
            for (int k = 0; k < p; ++k) out->f[OR_V][l][k * n + j] = in->f[OR_V][l][j * p + k];
        for (int i = 0; i < m; ++i)          /* u: m x n, entry (i, j) */
            for (int j = 0; j < n; ++j) out->f[OR_W][l][j * m + i] = in->f[OR_U][l][i * n + j];
        or_normalise_term(out, l);
    }
    return 0;
}

/* Merge (Sec. 3.3.2) of (m,n,p1:r1) and (m,n,p2:r2) into (m,n,p1+p2:r1+r2)
 * (axis 2: C = A [B1 B2], the second scheme's b and c columns shifted by
 * p1); axis 0: (m1+m2,n,p) from [A1; A2] B; axis 1: (m,n1+n2,p) from
 * [A1 A2][B1; B2] = A1 B1 + A2 B2.  The terms of a come first.  Returns -1
 * when the other two dimensions differ or a factor would exceed 64 entries
 * or the rank OR_MAXT. */
int or_merge(const or_scheme *a, const or_scheme *b, int axis, or_scheme *out)
{
    if (axis < 0 || axis > 2 || a->z2 != b->z2) return -1;
    if (axis == 0 && (a->n != b->n || a->p != b->p)) return -1;
    if (axis == 1 && (a->m != b->m || a->p != b->p)) return -1;
    if (axis == 2 && (a->m != b->m || a->n != b->n)) return -1;
    int M = axis == 0 ? a->m + b->m : a->m, N = axis == 1 ? a->n + b->n : a->n,
        P = axis == 2 ? a->p + b->p : a->p;
    if (M * N > OR_MAXL || N * P > OR_MAXL || P * M > OR_MAXL || a->r + b->r > OR_MAXT) return -1;
    memset(out, 0, sizeof(*out));
    out->m = M; out->n = N; out->p = P; out->z2 = a->z2; out->r = a->r + b->r;
    for (int q = 0; q < 2; ++q) {
        const or_scheme *s = q ? b : a;
        int oi = (q && axis == 0) ? a->m : 0, oj = (q && axis == 1) ? a->n : 0,
            ok = (q && axis == 2) ? a->p : 0;
        for (int l = 0; l < s->r; ++l) {
            int L = (q ? a->r : 0) + l;
            for (int i = 0; i < s->m; ++i)
                for (int j = 0; j < s->n; ++j)
                    out->f[OR_U][L][(i + oi) * N + j + oj] = s->f[OR_U][l][i * s->n + j];
            for (int j = 0; j < s->n; ++j)
                for (int k = 0; k < s->p; ++k)
                    out->f[OR_V][L][(j + oj) * P + k + ok] = s->f[OR_V][l][j * s->p + k];
            for (int k = 0; k < s->p; ++k)
                for (int i = 0; i < s->m; ++i)
                    out->f[OR_W][L][(k + ok) * M + i + oi] = s->f[OR_W][l][k * s->m + i];
        }
    }
    for (int l = 0; l < out->r; ++l) or_normalise_term(out, l);
    return 0;
}

/* Product (Sec. 3.3.2): the tensor (Kronecker) product of (m1,n1,p1:r1) and
 * (m2,n2,p2:r2) is a scheme for (m1 m2, n1 n2, p1 p2 : r1 r2): term
 * l1*r2 + l2 has u = u1 (x) u2 with row i1*m2+i2, column j1*n2+j2 (likewise v,
 * w).  Returns -1 when a factor would exceed 64 entries or the rank OR_MAXT. */
int or_product(const or_scheme *a, const or_scheme *b, or_scheme *out)
{
    if (a->z2 != b->z2) return -1;
    int M = a->m * b->m, N = a->n * b->n, P = a->p * b->p;
    if (M * N > OR_MAXL || N * P > OR_MAXL || P * M > OR_MAXL || a->r * b->r > OR_MAXT) return -1;
    memset(out, 0, sizeof(*out));
    out->m = M; out->n = N; out->p = P; out->z2 = a->z2; out->r = a->r * b->r;
    for (int l1 = 0; l1 < a->r; ++l1)
        for (int l2 = 0; l2 < b->r; ++l2) {
            int L = l1 * b->r + l2;
            for (int i1 = 0; i1 < a->m; ++i1) for (int j1 = 0; j1 < a->n; ++j1)
                for (int i2 = 0; i2 < b->m; ++i2) for (int j2 = 0; j2 < b->n; ++j2)
                    out->f[OR_U][L][(i1 * b->m + i2) * N + j1 * b->n + j2] = (int8_t)(
                        a->f[OR_U][l1][i1 * a->n + j1] * b->f[OR_U][l2][i2 * b->n + j2]);
            for (int j1 = 0; j1 < a->n; ++j1) for (int k1 = 0; k1 < a->p; ++k1)
                for (int j2 = 0; j2 < b->n; ++j2) for (int k2 = 0; k2 < b->p; ++k2)
                    out->f[OR_V][L][(j1 * b->n + j2) * P + k1 * b->p + k2] = (int8_t)(
                        a->f[OR_V][l1][j1 * a->p + k1] * b->f[OR_V][l2][j2 * b->p + k2]);
            for (int k1 = 0; k1 < a->p; ++k1) for (int i1 = 0; i1 < a->m; ++i1)
                for (int k2 = 0; k2 < b->p; ++k2) for (int i2 = 0; i2 < b->m; ++i2)
                    out->f[OR_W][L][(k1 * b->p + k2) * M + i1 * b->m + i2] = (int8_t)(
                        a->f[OR_W][l1][k1 * a->m + i1] * b->f[OR_W][l2][k2 * b->m + i2]);
            or_normalise_term(out, L);
        }
    return 0;
}

/* Resize (Algorithm 2, Sec. 3.4.3) of one scheme s of a walk, given the
 * population's best schemes.  Reading of the random choices (the paper gives
 * the probabilities only): Philox blocks b0 = (round, 0, 3) and
 * b1 = (round, 1, 3) keyed by the walk seed.
 *   b0.w0 < 2^31: swap sizes.
 *   merge partner best[U(b0.w1, n_best)]; try the axes p, m, n in that order
 *   and keep the first merge that exists and fits (rank <= cap).
 *   No merge and b0.w2 < t_resize: q = b0.w3 picks project (q < 0.05 * 2^32),
 *   product with best[U(b1.w0, n_best)] (q < 0.55 * 2^32), double (merge
 *   with itself, q < 0.85 * 2^32) or extend; axis U(b1.w1, 3), project index
 *   U(b1.w2, dim).  An operator that does not exist or fit leaves the
 *   scheme unchanged.  Returns the operators applied: bit 0 swap, 1 merge,
 *   2 project, 3 product, 4 double, 5 extend. */
#define OR_T_PROJECT 214748365u   /* round(0.05 * 2^32) */
#define OR_T_PRODUCT 2362232013u  /* round(0.55 * 2^32) */
#define OR_T_DOUBLE 3650722202u   /* round(0.85 * 2^32) */
int or_resize(const or_scheme *s, const or_scheme *best, int n_best, uint64_t seed,
              int64_t round, uint64_t t_resize, int cap, or_scheme *out)
{
    or_scheme *tmp = (or_scheme *)malloc(2 * sizeof(or_scheme));  /* ~100 KB each */
    if (!tmp) return -1;
    or_scheme *self = tmp + 1;
    uint32_t b0[4], b1[4];
    int applied = 0;
    draw(seed, round, 0, 3, b0);
    draw(seed, round, 1, 3, b1);
    *out = *s;
    if (b0[0] < 0x80000000u) {
        or_swap_sizes(out, tmp);
        *out = *tmp;
        applied |= 1;
    }
    if (n_best > 0) {
        const or_scheme *partner = &best[uniform_below(b0[1], n_best)];
        static const int order[3] = { 2, 0, 1 };
        for (int q = 0; q < 3 && !(applied & 2); ++q)
            if (or_merge(out, partner, order[q], tmp) == 0 && tmp->r <= cap) {
                *out = *tmp;
                applied |= 2;
            }
    }
    if (!(applied & 2) && (uint64_t)b0[2] < t_resize) {
        int axis = uniform_below(b1[1], 3);
        int dims[3] = { out->m, out->n, out->p };
        int ok = -1, bit = 0;
        if (b0[3] < OR_T_PROJECT) {
            bit = 4;
            if (dims[axis] >= 2) ok = or_project(out, axis, uniform_below(b1[2], dims[axis]), tmp);
        } else if (b0[3] < OR_T_PRODUCT) {
            bit = 8;
            if (n_best > 0) ok = or_product(out, &best[uniform_below(b1[0], n_best)], tmp);
        } else if (b0[3] < OR_T_DOUBLE) {
            bit = 16;
            *self = *out;
            ok = or_merge(out, self, axis, tmp);
        } else {
            bit = 32;
            ok = or_extend(out, axis, tmp);
        }
        if (ok == 0 && tmp->r <= cap) {
            *out = *tmp;
            applied |= bit;
        }
    }
    free(tmp);
    return applied;
}

/* Ternary lifting (Sec. 3.10.1): signs for the non-zero coefficients of a
 * Z2 scheme such that the Brent equations hold over the integers.  Reading:
 * an exhaustive search that returns the first solution in a fixed order
 * (the paper uses a constraint solver; any solution is a valid lifting, the
 * order only makes the answer unique).  Per term, the first non-zero entry of
 * u and of v is +1 (any solution can be brought to this form, Sec. 3.6); the
 * other non-zero entries -- u ascending, then v, then w -- are the term's free
 * signs, bit i of the term's pattern x set meaning entry i is -1.  Terms are
 * assigned in order, patterns ascending; after each term, every equation it
 * touches must still be reachable: |target - partial sum| <= the number of
 * later terms that touch it (each adds +-1).  Returns 1 with the scheme in
 * *out, 0 when no lifting exists, -1 when max_nodes term assignments were
 * tried first; *nodes counts them. */
typedef struct {
    const or_scheme *s;
    int Lu, Lv, Lw;
    int *nz[3];          /* per term and kind: the non-zero entries, ascending */
    int cnt[OR_MAXT][3];
    long *res, *rem;     /* per equation: target - partial sum; later contributors */
    int8_t sign[OR_MAXT][3][OR_MAXL];
    int64_t nodes, max_nodes;
} lift_state;

static int lift_free(const lift_state *L, int l)
{
    return L->cnt[l][0] - 1 + L->cnt[l][1] - 1 + L->cnt[l][2];
}

/* the pattern's signs into sign[l] */
static void lift_pattern(lift_state *L, int l, long x)
{
    int bit = 0;
    for (int X = 0; X < 3; ++X)
        for (int q = 0; q < L->cnt[l][X]; ++q) {
            int e = L->nz[X][l * OR_MAXL + q];
            if (X < 2 && q == 0) {
                L->sign[l][X][e] = 1;
            } else {
                L->sign[l][X][e] = ((x >> bit) & 1) ? -1 : 1;
                ++bit;
            }
        }
}

/* add (dir = -1) or remove (+1) term l's products; returns 1 when every
 * touched equation stays reachable (checked when adding) */
static int lift_apply(lift_state *L, int l, int dir)
{
    int ok = 1;
    for (int qa = 0; qa < L->cnt[l][0]; ++qa) {
        int a = L->nz[0][l * OR_MAXL + qa];
        for (int qb = 0; qb < L->cnt[l][1]; ++qb) {
            int b = L->nz[1][l * OR_MAXL + qb];
            for (int qc = 0; qc < L->cnt[l][2]; ++qc) {
                int c = L->nz[2][l * OR_MAXL + qc];
                long e = ((long)a * L->Lv + b) * L->Lw + c;
                long prod = L->sign[l][0][a] * L->sign[l][1][b] * L->sign[l][2][c];
                L->res[e] += dir * prod;
                L->rem[e] += dir;
                if (dir < 0 && (L->res[e] > L->rem[e] || -L->res[e] > L->rem[e])) ok = 0;
            }
        }
    }
    return ok;
}

static int lift_dfs(lift_state *L, int l)
{
    if (l == L->s->r) return 1;
    long n_pat = 1L << lift_free(L, l);
    for (long x = 0; x < n_pat; ++x) {
        if (L->nodes >= L->max_nodes) return -1;
        L->nodes++;
        lift_pattern(L, l, x);
        int ok = lift_apply(L, l, -1);
        if (ok) {
            int r = lift_dfs(L, l + 1);
            if (r != 0) return r;   /* found (1) or out of budget (-1): keep the signs */
        }
        lift_apply(L, l, +1);
    }
    return 0;
}

int or_lift(const or_scheme *z2s, int64_t max_nodes, or_scheme *out, int64_t *nodes)
{
    const or_scheme *s = z2s;
    int m = s->m, n = s->n, p = s->p;
    lift_state *L = (lift_state *)calloc(1, sizeof(lift_state));
    if (!L) return -2;
    L->s = s;
    L->Lu = m * n; L->Lv = n * p; L->Lw = p * m;
    L->max_nodes = max_nodes;
    long E = (long)L->Lu * L->Lv * L->Lw;
    L->res = (long *)calloc((size_t)E, sizeof(long));
    L->rem = (long *)calloc((size_t)E, sizeof(long));
    for (int X = 0; X < 3; ++X) L->nz[X] = (int *)calloc((size_t)OR_MAXT * OR_MAXL, sizeof(int));
    int lens[3] = { L->Lu, L->Lv, L->Lw };
    int status = 0;
    for (int l = 0; l < s->r; ++l)
        for (int X = 0; X < 3; ++X) {
            int c = 0;
            for (int e = 0; e < lens[X]; ++e)
                if (s->f[X][l][e] != 0) L->nz[X][l * OR_MAXL + c++] = e;
            L->cnt[l][X] = c;
            if (c == 0) status = -3;      /* a zero factor: not a scheme term */
        }
    for (long e = 0; e < E; ++e) {
        long a = e / ((long)L->Lv * L->Lw), b = (e / L->Lw) % L->Lv, c = e % L->Lw;
        int a1 = (int)(a / n), a2 = (int)(a % n), b1 = (int)(b / p), b2 = (int)(b % p);
        int c1 = (int)(c / m), c2 = (int)(c % m);
        L->res[e] = (a2 == b1 && b2 == c1 && c2 == a1) ? 1 : 0;
    }
    for (int l = 0; l < s->r && status == 0; ++l)
        for (int qa = 0; qa < L->cnt[l][0]; ++qa)
            for (int qb = 0; qb < L->cnt[l][1]; ++qb)
                for (int qc = 0; qc < L->cnt[l][2]; ++qc) {
                    long e = ((long)L->nz[0][l * OR_MAXL + qa] * L->Lv + L->nz[1][l * OR_MAXL + qb]) *
                             L->Lw + L->nz[2][l * OR_MAXL + qc];
                    L->rem[e]++;
                }
    if (status == 0) {
        for (int l = 0; l < s->r; ++l)
            if (lift_free(L, l) > 40) status = -3;   /* beyond any search here */
    }
    if (status == 0) status = lift_dfs(L, 0);
    if (status == 1) {
        memset(out, 0, sizeof(*out));
        out->m = m; out->n = n; out->p = p; out->r = s->r; out->z2 = 0;
        for (int l = 0; l < s->r; ++l)
            for (int X = 0; X < 3; ++X)
                for (int e = 0; e < lens[X]; ++e)
                    out->f[X][l][e] = s->f[X][l][e] ? L->sign[l][X][e] : 0;
    }
    if (nodes) *nodes = L->nodes;
    for (int X = 0; X < 3; ++X) free(L->nz[X]);
    free(L->res);
    free(L->rem);
    free(L);
    return status;
}

/* ------------------------------------------------------------------------ */
/* The walk: Algorithm 1 (RandomWalk kernel, Sec. 3.4.2)                     */
/* ------------------------------------------------------------------------ */

void or_walk_init(or_walk *w, const or_scheme *start)
{
    memset(w, 0, sizeof(*w));
    w->start = *start;
    for (int l = 0; l < w->start.r; ++l) or_normalise_term(&w->start, l);
    w->cur = w->start;
    w->best = w->start;
    w->best_rank = w->start.r;
    w->best_nnz = (int32_t)or_nonzeros(&w->start);
}

/* best := current (the best scheme's non-zero count follows it) */
static void set_best(or_walk *w)
{
    w->best = w->cur;
    w->best_rank = w->cur.r;
    w->best_nnz = (int32_t)or_nonzeros(&w->cur);
}

/* Is (j, sigma, role) a valid flip partner of (i, X)?  keep_rank: also
 * require that neither modified factor becomes zero (a flip that zeroes a
 * factor removes a term, which the additions objective excludes). */
static int partner(const or_scheme *s, int i, int j, int X, int role, int keep_rank, int *sigma)
{
    if (j == i) return 0;
    int sg = shared_sign(s, i, j, X);
    if (sg == 0) return 0;
    if (!or_flip_valid(s, i, j, X, sg, role)) return 0;
    if (keep_rank) {
        int Y, Z;
        int8_t tmp[OR_MAXL];
        other_kinds(X, role, &Y, &Z);
        or_ternary_add(s->f[Y][i], s->f[Y][j], sg, or_len(s, Y), s->z2, tmp);
        if (vec_zero(tmp, or_len(s, Y))) return 0;
        or_ternary_add(s->f[Z][j], s->f[Z][i], -1, or_len(s, Z), s->z2, tmp);
        if (vec_zero(tmp, or_len(s, Z))) return 0;
    }
    *sigma = sg;
    return 1;
}

/* Candidates of the attempt (i, X): the valid (j, role), role 0 then 1, j
 * ascending.  Returns their number; when pick >= 0, the pick-th candidate is
 * written to *pj, *psg, *prole. */
static int attempt_candidates(const or_scheme *s, int i, int X, int keep_rank, long pick, int *pj,
                              int *psg, int *prole)
{
    int n = 0;
    for (int role = 0; role < 2; ++role)
        for (int j = 0; j < s->r; ++j) {
            int sg;
            if (!partner(s, i, j, X, role, keep_rank, &sg)) continue;
            if (n == pick) {
                *pj = j; *psg = sg; *prole = role;
            }
            ++n;
        }
    return n;
}

static int fallback_flip(or_walk *w, const or_params *prm, int64_t t, int *pi, int *pj, int *pX,
                         int *prole);

/* try_flip of Algorithm 1.  Reading (the paper does not fix how a flip is
 * sampled): attempt a = 0..flip_tries-1 draws block (t,a,0): term
 * i = U(w0, r), factor X = U(w1, 3); its candidates are the valid
 * (j, role) in order role 0 then 1, j ascending; a non-empty list yields
 * candidate U(w2, |list|).  If every attempt is empty, the unused fourth
 * words of blocks (t,0,0) and (t,1,0) give a starting pair p0 = U(w3, 3r)
 * (block (t,0,0)); the pairs p = 3i + X are visited cyclically from p0 and the
 * first one with candidates yields candidate U(w3, |list|) (block (t,1,0)).
 * Only when no pair has a candidate (no valid flip exists at all) does
 * try_flip fail.  On success *pi and *pj hold the modified terms. */
static int try_flip(or_walk *w, const or_params *prm, int64_t t, int *pi, int *pj, int *pX,
                    int *prole)
{
    or_scheme *s = &w->cur;
    int r = s->r;
    uint32_t rw[4];
    int j = -1, sg = 0, role = 0;
    const int keep = prm->objective == 1;
    if (r < 2) return 0;
    for (int a = 0; a < prm->flip_tries; ++a) {
        draw(prm->seed, t, (uint32_t)a, 0, rw);
        w->c.attempts++;
        int i = uniform_below(rw[0], r);
        int X = uniform_below(rw[1], 3);
        int n = attempt_candidates(s, i, X, keep, -1, &j, &sg, &role);
        if (n > 0) {
            attempt_candidates(s, i, X, keep, uniform_below(rw[2], n), &j, &sg, &role);
            *pi = i; *pj = j; *pX = X; *prole = role;
            return 1;
        }
    }
    return fallback_flip(w, prm, t, pi, pj, pX, prole);
}

/* every attempt was empty: cyclic search over the (i, X) pairs */
static int fallback_flip(or_walk *w, const or_params *prm, int64_t t, int *pi, int *pj, int *pX,
                         int *prole)
{
    or_scheme *s = &w->cur;
    int r = s->r;
    uint32_t b0[4], b1[4];
    int j = -1, sg = 0, role = 0;
    const int keep = prm->objective == 1;
    w->c.fallbacks++;
    draw(prm->seed, t, 0, 0, b0);
    draw(prm->seed, t, 1, 0, b1);
    int npairs = 3 * r;
    int p0 = uniform_below(b0[3], npairs);
    for (int q = 0; q < npairs; ++q) {
        int p = (p0 + q) % npairs;
        int i = p / 3, X = p % 3;
        int n = attempt_candidates(s, i, X, keep, -1, &j, &sg, &role);
        if (n == 0) continue;
        attempt_candidates(s, i, X, keep, uniform_below(b1[3], n), &j, &sg, &role);
        *pi = i; *pj = j; *pX = X; *prole = role;
        return 1;
    }
    return 0;
}

/* expand of Algorithm 1 (plus or split, 50/50, Sec. 3.3.1).  Reading: up to
 * eight attempts; attempt a draws block (t,a,2): i = U(w0, r),
 * j = U(w1, r-1) shifted past i, roles PERMS[U(w2, 6)], and the top bit of
 * w3 picks plus (0) or split (1).  Refused when the rank reached r_cap. */
static int expand(or_walk *w, const or_params *prm, int64_t t)
{
    or_scheme *s = &w->cur;
    int r = s->r;
    uint32_t rw[4];
    if (r >= prm->r_cap || r < 2 || r >= OR_MAXT) return 0;
    for (int a = 0; a < 8; ++a) {
        draw(prm->seed, t, (uint32_t)a, 2, rw);
        int i = uniform_below(rw[0], r);
        int j = uniform_below(rw[1], r - 1);
        if (j >= i) ++j;
        int perm = uniform_below(rw[2], 6);
        int ok = (rw[3] >> 31) ? or_split(s, i, j, perm) : or_plus(s, i, j, perm);
        if (ok) {
            w->c.expands++;
            return 1;
        }
    }
    w->c.expand_fails++;
    return 0;
}

static void restart_check(or_walk *w, const or_params *prm, int64_t t)
{
    if (prm->plateau > 0 && t - w->plateau_start >= prm->plateau) {
        w->cur = prm->restart_from_best ? w->best : w->start;
        w->plateau_start = t;
        w->c.restarts++;
    }
}

/* the two terms of a flip before it is applied, in role order, as masks */
static void log_factors(const or_scheme *s, int i, int j, int X, int role, or_log *lg)
{
    int Y, Z;
    other_kinds(X, role, &Y, &Z);
    const int8_t *fac[6] = { s->f[X][i], s->f[Y][i], s->f[Z][i], s->f[X][j], s->f[Y][j], s->f[Z][j] };
    const int kind[6] = { X, Y, Z, X, Y, Z };
    for (int q = 0; q < 6; ++q) {
        uint64_t d = 0, sg = 0;
        for (int e = 0; e < or_len(s, kind[q]); ++e) {
            if (fac[q][e] != 0) d |= 1ull << e;
            if (fac[q][e] < 0) sg |= 1ull << e;
        }
        lg->f[2 * q] = d;
        lg->f[2 * q + 1] = sg;
    }
}

/* The rest of an iteration of the additions objective, after try_flip found
 * (i, j, X, role) among the flips that keep every factor non-zero.  Reading
 * of the complexity-minimisation mode (Sec. 3.9: flips without reduction
 * edges): apply the flip; the rank never changes, there is no reduce and no
 * expand; Algorithm 1's best-scheme rule is applied to the number of
 * non-zero coefficients (equivalently to the naive additions of Sec. 4.5,
 * which differ from it by the constant 2r + mp): strictly fewer always, as
 * many with probability t_eq (word 0 of block (t,0,1)); a strict improvement
 * records (t, naive additions) and resets the plateau; then the plateau
 * restart. */
static void additions_step(or_walk *w, const or_params *prm, int64_t t, int i, int j, int X,
                           int role)
{
    or_scheme *s = &w->cur;
    or_flip(s, i, j, X, shared_sign(s, i, j, X), role);
    w->c.flips++;
    uint32_t g[4];
    draw(prm->seed, t, 0, 1, g);
    const long nnz = or_nonzeros(s);
    if (nnz < w->best_nnz) {
        set_best(w);
        w->plateau_start = t;
        if (w->n_rec < OR_MAXREC) {
            w->rec_iter[w->n_rec] = t;
            w->rec_rank[w->n_rec] = (int32_t)or_naive_additions(s);
        }
        w->n_rec++;
        w->c.improvements++;
    } else if (nnz == w->best_nnz && (uint64_t)g[0] < prm->t_eq) {
        set_best(w);
        w->c.eq_accepts++;
    }
    restart_check(w, prm, t);
}

/* the walk's stop rule: best rank (or, for the additions objective, best
 * naive additions) at most the target */
static int reached(const or_walk *w, const or_params *prm)
{
    if (prm->objective == 1)
        return w->best_nnz - 2L * w->best.r - (long)w->best.m * w->best.p <= prm->target_rank;
    return w->best_rank <= prm->target_rank;
}

/* One iteration of Algorithm 1.  choice < 0: uniform proposals (try_flip);
 * choice >= 0: the externally chosen attempt (255 = fallback), see
 * or_walk_run_choices.  Returns 0, or 1 when the choice was inconsistent. */
static int one_iteration(or_walk *w, const or_params *prm, int64_t t, int choice, or_log *lg)
{
    or_scheme *s = &w->cur;
    int i = -1, j = -1, X = 0, role = 0;
    int found;
    w->c.iters++;
    if (lg) {
        memset(lg, 0, sizeof(*lg));
        lg->iter = t;
        lg->rank_before = -1;
    }
    if (choice < 0) {
        found = try_flip(w, prm, t, &i, &j, &X, &role);
    } else {
        int K = prm->flip_tries, any = 0;
        w->c.attempts += K;
        for (int a = 0; a < K; ++a)
            if (or_attempt_candidate(s, prm->seed, t, a, &i, &j, &X, &role) > 0) any = 1;
        if (choice == 255) {
            if (any) return 1;
            found = s->r >= 2 && fallback_flip(w, prm, t, &i, &j, &X, &role);
        } else {
            if (choice >= K) return 1;
            if (or_attempt_candidate(s, prm->seed, t, choice, &i, &j, &X, &role) == 0) return 1;
            found = 1;
        }
    }
    if (!found) {
        /* Algorithm 1: no flip -> expand, continue (the additions objective
         * keeps the rank and does not expand) */
        w->c.dead_ends++;
        if (prm->objective != 1) expand(w, prm, t);
        restart_check(w, prm, t);
        if (lg) lg->rank_after = s->r;
        return 0;
    }
    if (prm->objective == 1) {
        if (lg) {
            log_factors(s, i, j, X, role, lg);
            lg->rank_before = s->r;
        }
        additions_step(w, prm, t, i, j, X, role);
        if (lg) lg->rank_after = s->r;
        return 0;
    }
    if (lg) {
        log_factors(s, i, j, X, role, lg);
        lg->rank_before = s->r;
    }
    or_flip(s, i, j, X, shared_sign(s, i, j, X), role);
    w->c.flips++;

    /* a flip that makes a factor zero is a reduction edge: the zero term
     * leaves the scheme at once (higher slot first, swap-remove) */
    int track[2] = { i, j };
    int zi = term_has_zero_factor(s, i), zj = term_has_zero_factor(s, j);
    if (zi && zj) {
        int hi = i > j ? i : j, lo = i > j ? j : i;
        swap_remove(s, hi, track, 2);
        swap_remove(s, lo, track, 2);
        w->c.zero_removed += 2;
    } else if (zi) {
        swap_remove(s, i, track, 2);
        w->c.zero_removed++;
    } else if (zj) {
        swap_remove(s, j, track, 2);
        w->c.zero_removed++;
    }

    uint32_t g[4];
    draw(prm->seed, t, 0, 1, g);
    /* best update: strictly better always, equal rank with probability 0.01 */
    if (s->r < w->best_rank) {
        set_best(w);
        w->plateau_start = t;
        if (w->n_rec < OR_MAXREC) {
            w->rec_iter[w->n_rec] = t;
            w->rec_rank[w->n_rec] = s->r;
        }
        w->n_rec++;
        w->c.improvements++;
    } else if (s->r == w->best_rank && (uint64_t)g[0] < prm->t_eq) {
        set_best(w);
        w->c.eq_accepts++;
    }
    /* reduce with probability p_reduce: merge the modified terms */
    if ((uint64_t)g[1] < prm->t_reduce) w->c.merges += reduce_tracked(s, track, 2);
    /* expand with probability p_expand, only near the best rank */
    if ((uint64_t)g[2] < prm->t_expand && s->r <= w->best_rank + 2 && s->r < prm->r_cap)
        expand(w, prm, t);
    restart_check(w, prm, t);
    if (lg) lg->rank_after = s->r;
    return 0;
}

int or_attempt_candidate(const or_scheme *s, uint64_t seed, int64_t t, int a, int *pi, int *pj,
                         int *pX, int *prole)
{
    uint32_t rw[4];
    int j = -1, sg = 0, role = 0;
    if (s->r < 2) return 0;
    draw(seed, t, (uint32_t)a, 0, rw);
    int i = uniform_below(rw[0], s->r);
    int X = uniform_below(rw[1], 3);
    int n = attempt_candidates(s, i, X, 0, -1, &j, &sg, &role);
    if (n == 0) return 0;
    attempt_candidates(s, i, X, 0, uniform_below(rw[2], n), &j, &sg, &role);
    *pi = i; *pj = j; *pX = X; *prole = role;
    return n;
}

void or_walk_run_logged(or_walk *w, const or_params *prm, int64_t n_iters, or_log *log,
                        int64_t log_cap, int32_t format_slot)
{
    for (int64_t step = 0; step < n_iters; ++step) {
        if (reached(w, prm)) w->done = 1;
        if (w->done || w->t >= prm->max_iters) return;
        int64_t t = w->t + 1;
        or_log *lg = (log && t <= log_cap) ? &log[t - 1] : NULL;
        one_iteration(w, prm, t, -1, lg);
        if (lg) lg->format_slot = format_slot;
        w->t = t;
    }
    if (reached(w, prm)) w->done = 1;
}

void or_walk_run_choices(or_walk *w, const or_params *prm, int64_t n_iters,
                         const uint8_t *choices, int64_t n_choices, int64_t *bad)
{
    for (int64_t step = 0; step < n_iters; ++step) {
        if (reached(w, prm)) w->done = 1;
        if (w->done || w->t >= prm->max_iters) return;
        int64_t t = w->t + 1;
        if (t > n_choices) return;
        if (one_iteration(w, prm, t, choices[t - 1], NULL)) {
            ++*bad;
            return;
        }
        w->t = t;
    }
    if (reached(w, prm)) w->done = 1;
}

void or_walk_run(or_walk *w, const or_params *prm, int64_t n_iters)
{
    for (int64_t step = 0; step < n_iters; ++step) {
        if (reached(w, prm)) w->done = 1;
        if (w->done || w->t >= prm->max_iters) return;
        int64_t t = w->t + 1;
        one_iteration(w, prm, t, -1, NULL);
        w->t = t;
    }
    if (reached(w, prm)) w->done = 1;
}

/* ------------------------------------------------------------------------ */
/* Many walks on host threads (used to time the oracle)                      */
/* ------------------------------------------------------------------------ */
typedef struct {
    const or_scheme *start;
    const or_params *prm;
    uint64_t base_seed;
    int64_t first_walk;
    int n_walks;
    int64_t n_iters;
    or_walk *out;
    int next;
    pthread_mutex_t lock;
} many_job;

static void *many_worker(void *arg)
{
    many_job *job = (many_job *)arg;
    for (;;) {
        pthread_mutex_lock(&job->lock);
        int k = job->next++;
        pthread_mutex_unlock(&job->lock);
        if (k >= job->n_walks) break;
        or_params prm = *job->prm;
        prm.seed = job->base_seed + (uint64_t)(job->first_walk + k);
        or_walk_init(&job->out[k], job->start);
        or_walk_run(&job->out[k], &prm, job->n_iters);
    }
    return NULL;
}

void or_run_many(const or_scheme *start, const or_params *prm, uint64_t base_seed,
                 int64_t first_walk, int n_walks, int64_t n_iters, int n_threads,
                 or_walk *out)
{
    many_job job;
    job.start = start; job.prm = prm; job.base_seed = base_seed;
    job.first_walk = first_walk; job.n_walks = n_walks; job.n_iters = n_iters;
    job.out = out; job.next = 0;
    pthread_mutex_init(&job.lock, NULL);
    if (n_threads < 1) n_threads = 1;
    if (n_threads > 256) n_threads = 256;
    pthread_t th[256];
    for (int q = 0; q < n_threads; ++q) pthread_create(&th[q], NULL, many_worker, &job);
    for (int q = 0; q < n_threads; ++q) pthread_join(th[q], NULL);
    pthread_mutex_destroy(&job.lock);
}
