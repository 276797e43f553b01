// tsf_bits.h -- one-bit ternary vectors and the walk's counter-based random
// stream, shared by the host library and the gfx950 kernels.
//
// A ternary vector (Sec. 3.5.1 of the paper) is a pair of masks: `d` has bit e
// set iff entry e is non-zero, `s` has bit e set iff entry e is -1 (s is a
// subset of d).  Z2 vectors use d only.  The arithmetic follows the formulas
// of Sec. 3.5.2; each returns whether the result stays in {-1,0,1}.
#pragma once
#include <stdint.h>

#if defined(__HIP__)
#define TSF_HD __host__ __device__ __forceinline__
#else
#define TSF_HD static inline
#endif

// a + b: d = da ^ db, s = (sa&da | sb&db) & d; overflow where both entries
// are non-zero with equal signs.
template <typename T>
TSF_HD bool tern_add(T da, T sa, T db, T sb, T &d, T &s)
{
    d = da ^ db;
    s = ((sa & da) | (sb & db)) & d;
    return (da & db & ~(sa ^ sb)) == 0;
}

// a - b: d = da ^ db, s = (sa&da | ~sb&db) & d; overflow where both entries
// are non-zero with different signs.
template <typename T>
TSF_HD bool tern_sub(T da, T sa, T db, T sb, T &d, T &s)
{
    d = da ^ db;
    s = ((sa & da) | (~sb & db)) & d;
    return (da & db & (sa ^ sb)) == 0;
}

// a + sigma*b with sigma = +1 or -1; in Z2 plain XOR (always valid).
template <typename T>
TSF_HD bool tern_axpy(bool z2, int sigma, T da, T sa, T db, T sb, T &d, T &s)
{
    if (z2) {
        d = da ^ db;
        s = 0;
        return true;
    }
    return sigma > 0 ? tern_add(da, sa, db, sb, d, s) : tern_sub(da, sa, db, sb, d, s);
}

// a == -b: same support, signs opposite on it.
template <typename T>
TSF_HD bool tern_neg_eq(T da, T sa, T db, T sb)
{
    return da == db && sa == (sb ^ db);
}

// three-way xor: one v_bitop3_b32 (truth table 0x96, odd parity) on gfx950
#if defined(__HIP_DEVICE_COMPILE__)
#define TSF_XOR3(a, b, c) __builtin_amdgcn_bitop3_b32((a), (b), (c), 0x96)
#else
#define TSF_XOR3(a, b, c) ((a) ^ (b) ^ (c))
#endif

// Philox4x32-10 (Salmon et al., SC'11): 10 rounds, multipliers
// 0xD2511F53 / 0xCD9E8D57, key increments 0x9E3779B9 / 0xBB67AE85.
struct Philox4 {
    uint32_t x[4];
};

TSF_HD Philox4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                             uint32_t k1)
{
#if defined(__HIP__)
#pragma unroll
#endif
    for (int round = 0; round < 10; ++round) {
        const uint64_t prod0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t prod1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t y0 = TSF_XOR3((uint32_t)(prod1 >> 32), c1, k0);
        const uint32_t y2 = TSF_XOR3((uint32_t)(prod0 >> 32), c3, k1);
        c1 = (uint32_t)prod1;
        c3 = (uint32_t)prod0;
        c0 = y0;
        c2 = y2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    Philox4 out;
    out.x[0] = c0;
    out.x[1] = c1;
    out.x[2] = c2;
    out.x[3] = c3;
    return out;
}

// The walk's random block for (seed, iteration t, attempt a, domain dom):
// key = seed, counter = (t lo, t hi, a, dom).  Domains: 0 flip attempts,
// 1 per-iteration gates, 2 expand attempts.
TSF_HD Philox4 walk_block(uint64_t seed, int64_t t, uint32_t a, uint32_t dom)
{
    return philox4x32_10((uint32_t)(uint64_t)t, (uint32_t)((uint64_t)t >> 32), a, dom,
                         (uint32_t)seed, (uint32_t)(seed >> 32));
}

// uniform integer in [0, n) from one word: (word * n) >> 32
TSF_HD uint32_t below(uint32_t word, uint32_t n)
{
    return (uint32_t)(((uint64_t)word * n) >> 32);
}

// counters kept per walk, in tsf_walk_header.counters order
enum {
    C_ITERS = 0, C_FLIPS, C_ATTEMPTS, C_FALLBACKS, C_DEAD_ENDS, C_ZERO_REMOVED, C_MERGES,
    C_EXPANDS, C_EXPAND_FAILS, C_RESTARTS, C_EQ_ACCEPTS, C_IMPROVEMENTS, C_NUM
};

// Slot of a format in the proposal network's one-hot: fifteen small formats
// with their dimensions sorted, 15 for any other.
TSF_HD int format_slot(int m, int n, int p)
{
    int a = m, b = n, c = p, x;
    if (a > b) { x = a; a = b; b = x; }
    if (b > c) { x = b; b = c; c = x; }
    if (a > b) { x = a; a = b; b = x; }
    const int key = a * 100 + b * 10 + c;
    switch (key) {
    case 222: return 0;
    case 223: return 1;
    case 224: return 2;
    case 233: return 3;
    case 234: return 4;
    case 333: return 5;
    case 334: return 6;
    case 244: return 7;
    case 344: return 8;
    case 335: return 9;
    case 444: return 10;
    case 345: return 11;
    case 445: return 12;
    case 455: return 13;
    case 555: return 14;
    default: return 15;
    }
}

// Rank of one factor as a matrix (Sec. 3.7): entry (i, j) of the rows x cols
// matrix is bit i*cols + j of the one-bit masks (d, s) -- u as m x n, v as
// n x p, w as p x m (the C^T layout of Sec. 3.1).  Ternary factors are
// reduced over GF(65521): a non-zero minor of order k <= 8 of a {-1,0,1}
// matrix has |det| <= k^(k/2) <= 4096 (Hadamard's bound) < 65521, so this is
// the rank over Q; Z2 factors are reduced over GF(2).  Fraction-free row
// elimination (a row is replaced by pivot * row - row[c] * pivot_row, which
// keeps the row space's dimension).  M: rows * cols int32 of scratch.
TSF_HD int factor_rank(uint64_t d, uint64_t s, int rows, int cols, bool z2, int32_t *M)
{
    const uint32_t P = z2 ? 2u : 65521u;
    for (int e = 0; e < rows * cols; ++e)
        M[e] = ((d >> e) & 1) ? (((s >> e) & 1) ? (int32_t)(P - 1) : 1) : 0;
    int rank = 0;
    for (int c = 0; c < cols && rank < rows; ++c) {
        int piv = -1;
        for (int r = rank; r < rows; ++r)
            if (M[r * cols + c] != 0) {
                piv = r;
                break;
            }
        if (piv < 0) continue;
        if (piv != rank)
            for (int x = 0; x < cols; ++x) {
                const int32_t tmp = M[piv * cols + x];
                M[piv * cols + x] = M[rank * cols + x];
                M[rank * cols + x] = tmp;
            }
        const uint32_t pv = (uint32_t)M[rank * cols + c];
        for (int r = rank + 1; r < rows; ++r) {
            const uint32_t f = (uint32_t)M[r * cols + c];
            if (f == 0) continue;
            for (int x = c; x < cols; ++x) {
                const uint32_t a = (uint32_t)M[r * cols + x] * pv % P;
                const uint32_t b = (uint32_t)M[rank * cols + x] * f % P;
                M[r * cols + x] = (int32_t)((a + P - b) % P);
            }
        }
        ++rank;
    }
    return rank;
}
