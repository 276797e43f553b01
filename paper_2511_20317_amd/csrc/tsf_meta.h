// tsf_meta.h -- the meta operators of Sec. 3.3.2 on one term in the packed
// one-bit form, shared by the host library and the resize kernel.  A factor
// is a rows x cols matrix, entry (r, c) at bit r*cols + c: u is m x n
// (a_ij), v is n x p (b_jk), w is p x m (c_ik at row k, column i: the C^T
// layout of Sec. 3.1).  A term is f[6] = (u.d, u.s, v.d, v.s, w.d, w.s).
#pragma once
#include "tsf_bits.h"

// bit (r, c) of a rows x cols matrix -> bit (c, r) of its transpose
TSF_HD uint64_t mask_transpose(uint64_t x, int rows, int cols)
{
    uint64_t o = 0;
    for (; x; x &= x - 1) {
        const int e = __builtin_ctzll(x);
        const int r = e / cols, c = e % cols;
        o |= 1ull << (c * rows + r);
    }
    return o;
}

// bit (r, c) of a matrix with `cols` columns -> bit (r + dr, c + dc) of one
// with `cols2` columns
TSF_HD uint64_t mask_embed(uint64_t x, int cols, int cols2, int dr, int dc)
{
    uint64_t o = 0;
    for (; x; x &= x - 1) {
        const int e = __builtin_ctzll(x);
        o |= 1ull << ((e / cols + dr) * cols2 + e % cols + dc);
    }
    return o;
}

// Kronecker product of a (r1 x c1) and b (r2 x c2): entry (a1*r2 + a2,
// b1*c2 + b2) = a(a1, b1) * b(a2, b2); signs multiply
TSF_HD void mask_kron(uint64_t da, uint64_t sa, int c1, uint64_t db, uint64_t sb, int r2, int c2,
                      uint64_t &d, uint64_t &s)
{
    d = s = 0;
    const int cols = c1 * c2;
    for (uint64_t x = da; x; x &= x - 1) {
        const int e = __builtin_ctzll(x);
        const int a1 = e / c1, b1 = e % c1;
        const uint64_t sg1 = (sa >> e) & 1;
        for (uint64_t y = db; y; y &= y - 1) {
            const int g = __builtin_ctzll(y);
            const int a2 = g / c2, b2 = g % c2;
            const int pos = (a1 * r2 + a2) * cols + b1 * c2 + b2;
            d |= 1ull << pos;
            s |= (sg1 ^ ((sb >> g) & 1)) << pos;
        }
    }
}

// Sec. 3.6 on a packed term: the first non-zero of u, then of v, positive;
// w absorbs each sign change.  No-op in Z2 (no signs).
TSF_HD void normalise_packed(uint64_t (&f)[6])
{
    for (int X = 0; X < 2; ++X) {
        const uint64_t low = f[2 * X] & (~f[2 * X] + 1);
        if (f[2 * X + 1] & low) {
            f[2 * X + 1] ^= f[2 * X];
            f[5] ^= f[4];
        }
    }
}

// Swap sizes: a term of an (m,n,p) scheme -> the term of the (m,p,n) scheme
// (u'' = w^T, v'' = v^T, w'' = u^T: C^T = B^T A^T, and the Brent equations of
// the C^T layout are invariant under the cyclic rotation of the three
// factors), normalised
TSF_HD void term_swap(const uint64_t (&f)[6], int m, int n, int p, uint64_t (&o)[6])
{
    o[0] = mask_transpose(f[4], p, m);
    o[1] = mask_transpose(f[5], p, m);
    o[2] = mask_transpose(f[2], n, p);
    o[3] = mask_transpose(f[3], n, p);
    o[4] = mask_transpose(f[0], m, n);
    o[5] = mask_transpose(f[1], m, n);
    normalise_packed(o);
}

// Merge: a term of a scheme of (m,n,p) placed into the merged format (M,N,P)
// with its indices shifted by (oi, oj, ok)
TSF_HD void term_embed(const uint64_t (&f)[6], int m, int n, int p, int M, int N, int P, int oi,
                       int oj, int ok, uint64_t (&o)[6])
{
    o[0] = mask_embed(f[0], n, N, oi, oj);
    o[1] = mask_embed(f[1], n, N, oi, oj);
    o[2] = mask_embed(f[2], p, P, oj, ok);
    o[3] = mask_embed(f[3], p, P, oj, ok);
    o[4] = mask_embed(f[4], m, M, ok, oi);
    o[5] = mask_embed(f[5], m, M, ok, oi);
    (void)p;
    normalise_packed(o);
}

// Product: term (l1, l2) of the product of an (m1,n1,p1) and an (m2,n2,p2)
// scheme
TSF_HD void term_kron(const uint64_t (&a)[6], int m1, int n1, int p1, const uint64_t (&b)[6],
                      int m2, int n2, int p2, uint64_t (&o)[6])
{
    mask_kron(a[0], a[1], n1, b[0], b[1], m2, n2, o[0], o[1]);
    mask_kron(a[2], a[3], p1, b[2], b[3], n2, p2, o[2], o[3]);
    mask_kron(a[4], a[5], m1, b[4], b[5], p2, m2, o[4], o[5]);
    (void)m1;
    normalise_packed(o);
}
