// host.cpp -- host-side scheme operations of libtsf (see include/tsf.h):
// standard scheme, packing to the one-bit form, Brent verification,
// normalisation, reduction and the project/extend meta operators.
#include "../../include/tsf.h"
#include "tsf_bits.h"
#include "tsf_meta.h"
#include "tsf_internal.h"

#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

namespace {

thread_local std::string g_err;

#define fail tsf_fail

struct Lens {
    int u, v, w;
};

Lens lens_of(int m, int n, int p) { return Lens{m * n, n * p, p * m}; }

tsf_status check_dims(const tsf_dims &d, bool need_rank = true)
{
    if (d.m < 1 || d.n < 1 || d.p < 1)
        return fail(TSF_E_FORMAT, "format (%d,%d,%d): dimensions must be >= 1", d.m, d.n, d.p);
    Lens L = lens_of(d.m, d.n, d.p);
    if (L.u > 64 || L.v > 64 || L.w > 64)
        return fail(TSF_E_FORMAT, "format (%d,%d,%d): a factor has more than 64 entries", d.m,
                    d.n, d.p);
    if (d.mode != TSF_TERNARY && d.mode != TSF_Z2)
        return fail(TSF_E_ARG, "mode %d is neither ternary (0) nor Z2 (1)", d.mode);
    if (need_rank && (d.rank < 0 || d.rank > d.capacity))
        return fail(TSF_E_CAPACITY, "rank %d outside [0, capacity %d]", d.rank, d.capacity);
    return TSF_OK;
}

// A term in the one-bit form: factor X has digits f[2X], signs f[2X+1].
struct Term {
    uint64_t f[6];
};

tsf_status to_terms(const tsf_scheme *s, std::vector<Term> &out)
{
    const tsf_dims &d = s->d;
    Lens L = lens_of(d.m, d.n, d.p);
    const int len[3] = {L.u, L.v, L.w};
    const int8_t *mat[3] = {s->U, s->V, s->W};
    out.assign(d.rank, Term{});
    for (int l = 0; l < d.rank; ++l)
        for (int X = 0; X < 3; ++X) {
            uint64_t dg = 0, sg = 0;
            for (int e = 0; e < len[X]; ++e) {
                int c = mat[X][(size_t)l * len[X] + e];
                if (c == 0) continue;
                if (c == 1) {
                    dg |= 1ull << e;
                } else if (c == -1 && d.mode == TSF_TERNARY) {
                    dg |= 1ull << e;
                    sg |= 1ull << e;
                } else {
                    return fail(TSF_E_NOT_TERNARY, "term %d factor %c entry %d is %d", l,
                                "UVW"[X], e, c);
                }
            }
            out[l].f[2 * X] = dg;
            out[l].f[2 * X + 1] = sg;
        }
    return TSF_OK;
}

void from_terms(const std::vector<Term> &t, tsf_scheme *s)
{
    tsf_dims &d = s->d;
    Lens L = lens_of(d.m, d.n, d.p);
    const int len[3] = {L.u, L.v, L.w};
    int8_t *mat[3] = {s->U, s->V, s->W};
    d.rank = (int32_t)t.size();
    for (int X = 0; X < 3; ++X) std::memset(mat[X], 0, (size_t)d.capacity * len[X]);
    for (size_t l = 0; l < t.size(); ++l)
        for (int X = 0; X < 3; ++X)
            for (int e = 0; e < len[X]; ++e) {
                uint64_t bit = 1ull << e;
                if (t[l].f[2 * X] & bit)
                    mat[X][l * len[X] + e] = (t[l].f[2 * X + 1] & bit) ? -1 : 1;
            }
}

// Sign-symmetry normalisation (Sec. 3.6): lowest set digit of u, then of v,
// made positive; w absorbs each sign change.
void normalise_term(Term &t, bool z2)
{
    if (z2) return;
    for (int X = 0; X < 2; ++X) {
        uint64_t dg = t.f[2 * X];
        uint64_t low = dg & (~dg + 1);
        if (t.f[2 * X + 1] & low) {
            t.f[2 * X + 1] ^= dg;
            t.f[5] ^= t.f[4];
        }
    }
}

bool same(const Term &a, const Term &b, int X)
{
    return a.f[2 * X] == b.f[2 * X] && a.f[2 * X + 1] == b.f[2 * X + 1];
}

// +1 if factor X of b equals that of a, -1 if it is the negation (w only,
// ternary only), 0 otherwise
int rel_sign(const Term &a, const Term &b, int X, bool z2)
{
    if (same(a, b, X)) return 1;
    if (!z2 && X == 2 && tern_neg_eq(b.f[4], b.f[5], a.f[4], a.f[5])) return -1;
    return 0;
}

// Reduction (Sec. 3.3.1): try to merge terms a and b (sharing two factors).
// Returns the merged kind (0,1,2) or -1, and the merged factor in (md, ms).
int try_merge(const Term &a, const Term &b, bool z2, uint64_t &md, uint64_t &ms)
{
    const bool eu = same(a, b, 0), ev = same(a, b, 1);
    const int sw = rel_sign(a, b, 2, z2);
    if (eu && ev && tern_axpy(z2, 1, a.f[4], a.f[5], b.f[4], b.f[5], md, ms)) return 2;
    if (eu && sw && tern_axpy(z2, sw, a.f[2], a.f[3], b.f[2], b.f[3], md, ms)) return 1;
    if (ev && sw && tern_axpy(z2, sw, a.f[0], a.f[1], b.f[0], b.f[1], md, ms)) return 0;
    return -1;
}

bool has_zero_factor(const Term &t) { return t.f[0] == 0 || t.f[2] == 0 || t.f[4] == 0; }

}  // namespace

tsf_status tsf_fail(tsf_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

extern "C" {

const char *tsf_last_error(void) { return g_err.c_str(); }

tsf_status tsf_init_scheme(int32_t m, int32_t n, int32_t p, int32_t mode, tsf_scheme *out)
{
    if (!out || !out->U || !out->V || !out->W) return fail(TSF_E_ARG, "null scheme");
    tsf_dims d = out->d;
    d.m = m; d.n = n; d.p = p; d.mode = mode; d.rank = 0;
    tsf_status st = check_dims(d);
    if (st) return st;
    if ((int64_t)m * n * p > d.capacity)
        return fail(TSF_E_CAPACITY, "standard scheme needs %d rows, capacity %d", m * n * p,
                    d.capacity);
    std::vector<Term> t;
    t.reserve((size_t)m * n * p);
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < n; ++j)
            for (int k = 0; k < p; ++k) {
                Term x{};
                x.f[0] = 1ull << (i * n + j);
                x.f[2] = 1ull << (j * p + k);
                x.f[4] = 1ull << (k * m + i);
                t.push_back(x);
            }
    out->d = d;
    from_terms(t, out);
    return TSF_OK;
}

tsf_status tsf_verify(const tsf_scheme *s, int64_t *n_violated)
{
    if (!s || !n_violated || !s->U || !s->V || !s->W) return fail(TSF_E_ARG, "null argument");
    tsf_status st = check_dims(s->d);
    if (st) return st;
    std::vector<Term> t;
    if ((st = to_terms(s, t))) return st;
    const int m = s->d.m, n = s->d.n, p = s->d.p;
    Lens L = lens_of(m, n, p);
    // accumulate sum_l u_l (x) v_l (x) w_l over the non-zero entries only
    std::vector<int32_t> T((size_t)L.u * L.v * L.w, 0);
    for (const Term &x : t)
        for (uint64_t du = x.f[0]; du; du &= du - 1) {
            int a = __builtin_ctzll(du);
            int su = (x.f[1] >> a) & 1 ? -1 : 1;
            for (uint64_t dv = x.f[2]; dv; dv &= dv - 1) {
                int b = __builtin_ctzll(dv);
                int sv = (x.f[3] >> b) & 1 ? -su : su;
                int32_t *row = &T[((size_t)a * L.v + b) * L.w];
                for (uint64_t dw = x.f[4]; dw; dw &= dw - 1) {
                    int c = __builtin_ctzll(dw);
                    row[c] += (x.f[5] >> c) & 1 ? -sv : sv;
                }
            }
        }
    int64_t bad = 0;
    const bool z2 = s->d.mode == TSF_Z2;
    for (int a1 = 0; a1 < m; ++a1)
        for (int a2 = 0; a2 < n; ++a2)
            for (int b1 = 0; b1 < n; ++b1)
                for (int b2 = 0; b2 < p; ++b2)
                    for (int c1 = 0; c1 < p; ++c1)
                        for (int c2 = 0; c2 < m; ++c2) {
                            int32_t got = T[((size_t)(a1 * n + a2) * L.v + (b1 * p + b2)) * L.w +
                                            (c1 * m + c2)];
                            int32_t want = (a2 == b1 && b2 == c1 && c2 == a1) ? 1 : 0;
                            if (z2) got &= 1;
                            bad += got != want;
                        }
    *n_violated = bad;
    return TSF_OK;
}

tsf_status tsf_normalise(tsf_scheme *s)
{
    if (!s || !s->U || !s->V || !s->W) return fail(TSF_E_ARG, "null scheme");
    tsf_status st = check_dims(s->d);
    if (st) return st;
    std::vector<Term> t;
    if ((st = to_terms(s, t))) return st;
    for (Term &x : t) normalise_term(x, s->d.mode == TSF_Z2);
    from_terms(t, s);
    return TSF_OK;
}

tsf_status tsf_reduce(tsf_scheme *s, int32_t *n_reductions)
{
    if (!s || !s->U || !s->V || !s->W) return fail(TSF_E_ARG, "null scheme");
    tsf_status st = check_dims(s->d);
    if (st) return st;
    std::vector<Term> t;
    if ((st = to_terms(s, t))) return st;
    const bool z2 = s->d.mode == TSF_Z2;
    std::vector<Term> live;
    for (Term &x : t) {
        normalise_term(x, z2);
        if (!has_zero_factor(x)) live.push_back(x);
    }
    int32_t merges = 0;
    bool changed = true;
    while (changed) {
        changed = false;
        for (size_t a = 0; a < live.size() && !changed; ++a)
            for (size_t b = a + 1; b < live.size() && !changed; ++b) {
                uint64_t md, ms;
                int kind = try_merge(live[a], live[b], z2, md, ms);
                if (kind < 0) continue;
                ++merges;
                changed = true;
                if (md == 0) {
                    live.erase(live.begin() + b);
                    live.erase(live.begin() + a);
                } else {
                    live[a].f[2 * kind] = md;
                    live[a].f[2 * kind + 1] = ms;
                    normalise_term(live[a], z2);
                    live.erase(live.begin() + b);
                }
            }
    }
    if (n_reductions) *n_reductions = merges;
    from_terms(live, s);
    return TSF_OK;
}

tsf_status tsf_meta_project(const tsf_scheme *in, int32_t axis, int32_t index, tsf_scheme *out)
{
    if (!in || !out || !in->U || !out->U || !out->V || !out->W)
        return fail(TSF_E_ARG, "null scheme");
    tsf_status st = check_dims(in->d);
    if (st) return st;
    const int dims[3] = {in->d.m, in->d.n, in->d.p};
    if (axis < 0 || axis > 2) return fail(TSF_E_ARG, "axis %d not in 0..2", axis);
    if (dims[axis] < 2) return fail(TSF_E_ARG, "cannot project a dimension of size 1");
    if (index < 0 || index >= dims[axis])
        return fail(TSF_E_ARG, "index %d outside [0,%d)", index, dims[axis]);
    std::vector<Term> t;
    if ((st = to_terms(in, t))) return st;
    const int m = dims[0], n = dims[1], p = dims[2];
    const int m2 = m - (axis == 0), n2 = n - (axis == 1), p2 = p - (axis == 2);
    // new position of an index along each axis, or -1 where it is dropped
    auto keep = [&](int ax, int x) -> int {
        if (ax != axis) return x;
        return x == index ? -1 : x - (x > index);
    };
    // remap factor masks entry by entry: U over (i,j), V over (j,k), W over (k,i)
    auto remap = [&](uint64_t mask, int r_ax, int c_ax, int cols, int cols2) {
        uint64_t o = 0;
        for (; mask; mask &= mask - 1) {
            int e = __builtin_ctzll(mask);
            int rr = keep(r_ax, e / cols), cc = keep(c_ax, e % cols);
            if (rr >= 0 && cc >= 0) o |= 1ull << (rr * cols2 + cc);
        }
        return o;
    };
    std::vector<Term> o;
    const bool z2 = in->d.mode == TSF_Z2;
    for (const Term &x : t) {
        Term y;
        y.f[0] = remap(x.f[0], 0, 1, n, n2);
        y.f[1] = remap(x.f[1], 0, 1, n, n2);
        y.f[2] = remap(x.f[2], 1, 2, p, p2);
        y.f[3] = remap(x.f[3], 1, 2, p, p2);
        y.f[4] = remap(x.f[4], 2, 0, m, m2);
        y.f[5] = remap(x.f[5], 2, 0, m, m2);
        if (has_zero_factor(y)) continue;
        normalise_term(y, z2);
        o.push_back(y);
    }
    if ((int)o.size() > out->d.capacity)
        return fail(TSF_E_CAPACITY, "projected rank %zu exceeds capacity %d", o.size(),
                    out->d.capacity);
    out->d.m = m2; out->d.n = n2; out->d.p = p2; out->d.mode = in->d.mode;
    from_terms(o, out);
    return TSF_OK;
}

tsf_status tsf_meta_extend(const tsf_scheme *in, int32_t axis, tsf_scheme *out)
{
    if (!in || !out || !in->U || !out->U || !out->V || !out->W)
        return fail(TSF_E_ARG, "null scheme");
    tsf_status st = check_dims(in->d);
    if (st) return st;
    if (axis < 0 || axis > 2) return fail(TSF_E_ARG, "axis %d not in 0..2", axis);
    const int m = in->d.m, n = in->d.n, p = in->d.p;
    const int m2 = m + (axis == 0), n2 = n + (axis == 1), p2 = p + (axis == 2);
    tsf_dims nd = out->d;
    nd.m = m2; nd.n = n2; nd.p = p2; nd.mode = in->d.mode; nd.rank = 0;
    if ((st = check_dims(nd))) return st;
    std::vector<Term> t;
    if ((st = to_terms(in, t))) return st;
    // existing entries keep (row, col); only the flattening stride changes
    auto grow = [](uint64_t mask, int cols, int cols2) {
        uint64_t o = 0;
        for (; mask; mask &= mask - 1) {
            int e = __builtin_ctzll(mask);
            o |= 1ull << ((e / cols) * cols2 + e % cols);
        }
        return o;
    };
    for (Term &x : t) {
        x.f[0] = grow(x.f[0], n, n2); x.f[1] = grow(x.f[1], n, n2);
        x.f[2] = grow(x.f[2], p, p2); x.f[3] = grow(x.f[3], p, p2);
        x.f[4] = grow(x.f[4], m, m2); x.f[5] = grow(x.f[5], m, m2);
    }
    auto naive = [&](int i, int j, int k) {
        Term y{};
        y.f[0] = 1ull << (i * n2 + j);
        y.f[2] = 1ull << (j * p2 + k);
        y.f[4] = 1ull << (k * m2 + i);
        t.push_back(y);
    };
    if (axis == 2) {
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < n; ++j) naive(i, j, p);
    } else if (axis == 0) {
        for (int j = 0; j < n; ++j)
            for (int k = 0; k < p; ++k) naive(m, j, k);
    } else {
        for (int i = 0; i < m; ++i)
            for (int k = 0; k < p; ++k) naive(i, n, k);
    }
    if ((int)t.size() > out->d.capacity)
        return fail(TSF_E_CAPACITY, "extended rank %zu exceeds capacity %d", t.size(),
                    out->d.capacity);
    out->d = nd;
    from_terms(t, out);
    return TSF_OK;
}

tsf_status tsf_pack(const tsf_scheme *in, uint64_t *packed)
{
    if (!in || !packed || !in->U || !in->V || !in->W) return fail(TSF_E_ARG, "null argument");
    tsf_status st = check_dims(in->d);
    if (st) return st;
    std::vector<Term> t;
    if ((st = to_terms(in, t))) return st;
    std::memset(packed, 0, (size_t)in->d.capacity * 6 * sizeof(uint64_t));
    for (size_t l = 0; l < t.size(); ++l) std::memcpy(packed + 6 * l, t[l].f, sizeof(Term));
    return TSF_OK;
}

namespace {
tsf_status check_out(const tsf_scheme *out, int rank)
{
    if (!out || !out->U || !out->V || !out->W) return fail(TSF_E_ARG, "null output scheme");
    if (out->d.capacity < rank)
        return fail(TSF_E_CAPACITY, "output capacity %d < rank %d", out->d.capacity, rank);
    return TSF_OK;
}

void set_out(tsf_scheme *out, int m, int n, int p, int mode, std::vector<Term> &t)
{
    out->d.m = m;
    out->d.n = n;
    out->d.p = p;
    out->d.mode = mode;
    out->d.rank = (int32_t)t.size();
    from_terms(t, out);
}
}  // namespace

tsf_status tsf_meta_swap(const tsf_scheme *in, tsf_scheme *out)
{
    if (!in || !in->U || !in->V || !in->W) return fail(TSF_E_ARG, "null scheme");
    tsf_status st = check_dims(in->d);
    if (st) return st;
    std::vector<Term> t;
    if ((st = to_terms(in, t))) return st;
    if ((st = check_out(out, (int)t.size()))) return st;
    const int m = in->d.m, n = in->d.n, p = in->d.p;
    for (Term &x : t) {
        uint64_t o[6];
        term_swap(x.f, m, n, p, o);
        for (int e = 0; e < 6; ++e) x.f[e] = o[e];
    }
    set_out(out, m, p, n, in->d.mode, t);
    return TSF_OK;
}

tsf_status tsf_meta_merge(const tsf_scheme *a, const tsf_scheme *b, int32_t axis, tsf_scheme *out)
{
    if (!a || !b || !a->U || !b->U) return fail(TSF_E_ARG, "null scheme");
    tsf_status st = check_dims(a->d);
    if (st || (st = check_dims(b->d))) return st;
    if (a->d.mode != b->d.mode) return fail(TSF_E_ARG, "modes differ");
    if (axis < 0 || axis > 2) return fail(TSF_E_ARG, "axis %d not in 0..2", axis);
    const int m = a->d.m, n = a->d.n, p = a->d.p;
    const int bm = b->d.m, bn = b->d.n, bp = b->d.p;
    if ((axis == 0 && (n != bn || p != bp)) || (axis == 1 && (m != bm || p != bp)) ||
        (axis == 2 && (m != bm || n != bn)))
        return fail(TSF_E_ARG, "formats do not merge along axis %d", axis);
    const int M = axis == 0 ? m + bm : m, N = axis == 1 ? n + bn : n, P = axis == 2 ? p + bp : p;
    if (M * N > 64 || N * P > 64 || P * M > 64)
        return fail(TSF_E_FORMAT, "merged factors exceed 64 entries");
    std::vector<Term> ta, tb;
    if ((st = to_terms(a, ta)) || (st = to_terms(b, tb))) return st;
    if ((st = check_out(out, (int)(ta.size() + tb.size())))) return st;
    std::vector<Term> t;
    for (const Term &x : ta) {
        Term y;
        term_embed(x.f, m, n, p, M, N, P, 0, 0, 0, y.f);
        t.push_back(y);
    }
    for (const Term &x : tb) {
        Term y;
        term_embed(x.f, bm, bn, bp, M, N, P, axis == 0 ? m : 0, axis == 1 ? n : 0, axis == 2 ? p : 0,
                   y.f);
        t.push_back(y);
    }
    set_out(out, M, N, P, a->d.mode, t);
    return TSF_OK;
}

tsf_status tsf_meta_product(const tsf_scheme *a, const tsf_scheme *b, tsf_scheme *out)
{
    if (!a || !b || !a->U || !b->U) return fail(TSF_E_ARG, "null scheme");
    tsf_status st = check_dims(a->d);
    if (st || (st = check_dims(b->d))) return st;
    if (a->d.mode != b->d.mode) return fail(TSF_E_ARG, "modes differ");
    const int M = a->d.m * b->d.m, N = a->d.n * b->d.n, P = a->d.p * b->d.p;
    if (M * N > 64 || N * P > 64 || P * M > 64)
        return fail(TSF_E_FORMAT, "product factors exceed 64 entries");
    std::vector<Term> ta, tb;
    if ((st = to_terms(a, ta)) || (st = to_terms(b, tb))) return st;
    if ((st = check_out(out, (int)(ta.size() * tb.size())))) return st;
    std::vector<Term> t;
    for (const Term &x : ta)
        for (const Term &y : tb) {
            Term z;
            term_kron(x.f, a->d.m, a->d.n, a->d.p, y.f, b->d.m, b->d.n, b->d.p, z.f);
            t.push_back(z);
        }
    set_out(out, M, N, P, a->d.mode, t);
    return TSF_OK;
}

tsf_status tsf_scheme_invariants(const tsf_scheme *s, uint8_t *term_ranks, tsf_invariants *out)
{
    if (!s || !out || !s->U || !s->V || !s->W) return fail(TSF_E_ARG, "null argument");
    tsf_status st = check_dims(s->d);
    if (st) return st;
    std::vector<Term> t;
    if ((st = to_terms(s, t))) return st;
    const int m = s->d.m, n = s->d.n, p = s->d.p;
    const int rows[3] = {m, n, p}, cols[3] = {n, p, m};
    const bool z2 = s->d.mode == TSF_Z2;
    std::memset(out, 0, sizeof *out);
    int32_t M[64];
    static const int perm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    for (size_t l = 0; l < t.size(); ++l) {
        int rk[3];
        for (int X = 0; X < 3; ++X) {
            rk[X] = factor_rank(t[l].f[2 * X], t[l].f[2 * X + 1], rows[X], cols[X], z2, M);
            out->rank_sum[X] += rk[X];
            if (term_ranks) term_ranks[3 * l + X] = (uint8_t)rk[X];
        }
        out->type_poly[rk[0]][rk[1]][rk[2]]++;
        for (const int *q : perm) out->sym_poly[rk[q[0]]][rk[q[1]]][rk[q[2]]]++;
    }
    return TSF_OK;
}

tsf_status tsf_unpack(const uint64_t *packed, const tsf_dims *d, tsf_scheme *out)
{
    if (!packed || !d || !out || !out->U || !out->V || !out->W)
        return fail(TSF_E_ARG, "null argument");
    tsf_status st = check_dims(*d);
    if (st) return st;
    Lens L = lens_of(d->m, d->n, d->p);
    const int len[3] = {L.u, L.v, L.w};
    std::vector<Term> t(d->rank);
    for (int l = 0; l < d->rank; ++l)
        for (int X = 0; X < 3; ++X) {
            uint64_t dg = packed[6 * l + 2 * X], sg = packed[6 * l + 2 * X + 1];
            uint64_t lim = len[X] == 64 ? ~0ull : ((1ull << len[X]) - 1);
            if ((sg & ~dg) || (dg & ~lim) || (d->mode == TSF_Z2 && sg))
                return fail(TSF_E_NOT_TERNARY, "packed term %d factor %c is malformed", l,
                            "UVW"[X]);
            t[l].f[2 * X] = dg;
            t[l].f[2 * X + 1] = sg;
        }
    out->d = *d;
    from_terms(t, out);
    return TSF_OK;
}

}  // extern "C"

extern "C" int32_t tsf_format_slot(int32_t m, int32_t n, int32_t p) { return format_slot(m, n, p); }

namespace {
// FNV-1a over the little-endian bytes of one value
template <typename V>
void fnv1a(uint64_t &h, V v)
{
    uint64_t u = (uint64_t)v;
    for (size_t b = 0; b < sizeof(V); ++b) {
        h ^= (u >> (8 * b)) & 0xFF;
        h *= 0x100000001B3ull;
    }
}
}  // namespace

extern "C" uint64_t tsf_params_hash(const tsf_walk_params *prm)
{
    if (!prm) return 0;
    uint64_t h = 0xCBF29CE484222325ull;
    fnv1a(h, prm->base_seed);
    fnv1a(h, prm->first_walk_id);
    fnv1a(h, prm->max_iters);
    fnv1a(h, prm->plateau);
    fnv1a(h, prm->t_eq);
    fnv1a(h, prm->t_reduce);
    fnv1a(h, prm->t_expand);
    fnv1a(h, prm->flip_tries);
    fnv1a(h, prm->restart_from_best);
    fnv1a(h, prm->objective);
    return h ? h : 1;
}

extern "C" tsf_status tsf_state_check(const tsf_walk_header *hdr, const uint64_t *cur,
                                      const uint64_t *best, const uint64_t *start, int32_t n_walks,
                                      int32_t capacity, int32_t check_brent, int32_t *first_bad)
{
    if (first_bad) *first_bad = -1;
    if (n_walks < 0 || capacity < 1 || (n_walks > 0 && (!hdr || !cur || !best || !start)))
        return fail(TSF_E_ARG, "tsf_state_check: null buffer, n_walks < 0 or capacity < 1");
    std::vector<int8_t> U((size_t)capacity * 64), V((size_t)capacity * 64), W((size_t)capacity * 64);
    for (int32_t w = 0; w < n_walks; ++w) {
        const tsf_walk_header &h = hdr[w];
        if (h.done < 0) continue;  // flagged by a walk call; never advanced again
        auto bad = [&](tsf_status st) {
            if (first_bad) *first_bad = w;
            return st;
        };
        tsf_dims d{h.m, h.n, h.p, 0, capacity, h.mode};
        tsf_status st = check_dims(d, false);
        if (st) return bad(st);
        if (h.r_cap < 0 || h.r_cap > capacity || h.rank < 0 || h.rank > h.r_cap ||
            h.best_rank < 0 || h.best_rank > capacity || h.start_rank < 0 ||
            h.start_rank > capacity)
            return bad(fail(TSF_E_CAPACITY, "walk %d: ranks %d/%d/%d or r_cap %d outside the "
                            "capacity %d", (int)w, h.rank, h.best_rank, h.start_rank, h.r_cap,
                            (int)capacity));
        const uint64_t *bufs[3] = {cur, best, start};
        const int ranks[3] = {h.rank, h.best_rank, h.start_rank};
        for (int q = 0; q < 3; ++q) {
            d.rank = ranks[q];
            tsf_scheme sc{d, U.data(), V.data(), W.data()};
            // tsf_unpack checks the coding (TSF_E_NOT_TERNARY)
            if ((st = tsf_unpack(bufs[q] + (size_t)w * capacity * 6, &d, &sc)))
                return bad(fail(st, "walk %d: the %s scheme is malformed", (int)w,
                                q == 0 ? "current" : q == 1 ? "best" : "start"));
            if (!check_brent) continue;
            int64_t nv = 0;
            if ((st = tsf_verify(&sc, &nv))) return bad(st);
            if (nv)
                return bad(fail(TSF_E_INVALID_SCHEME, "walk %d: the %s scheme fails %lld Brent "
                                "equations", (int)w, q == 0 ? "current" : q == 1 ? "best" : "start",
                                (long long)nv));
        }
    }
    return TSF_OK;
}

extern "C" tsf_status tsf_walk_check(const tsf_walk_params *prm, const tsf_walk_header *hdr,
                                     int32_t n_walks, int32_t *n_mismatched)
{
    if (n_mismatched) *n_mismatched = 0;
    if (!prm || (n_walks > 0 && !hdr) || n_walks < 0)
        return fail(TSF_E_ARG, "tsf_walk_check: null argument or n_walks < 0");
    const uint64_t want = tsf_params_hash(prm);
    int32_t bad = 0;
    for (int32_t w = 0; w < n_walks; ++w)
        if ((hdr[w].params_hash != 0 && hdr[w].params_hash != want) || hdr[w].done == -3) ++bad;
    if (n_mismatched) *n_mismatched = bad;
    if (bad)
        return fail(TSF_E_STATE, "%d walks were run with other walk parameters", (int)bad);
    return TSF_OK;
}
