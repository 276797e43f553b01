// walk_kernel.h -- batched ternary flip-graph random walks on gfx950 (MI355X).
//
// One walk is owned by a group of G lanes of a 64-lane wavefront (64/G walks
// per wavefront).  The walk's current scheme lives in LDS in the one-bit form
// of Sec. 3.5.1, factor-major: the (digits, signs) pair of factor X of term k
// sits at words 2*(X*cap2 + k), so the same factor of consecutive terms is
// contiguous (two terms per 128-bit LDS read with 32-bit masks).  Per-walk
// scalars (rank, counters, random words) are replicated in every lane of the
// group, which keeps control flow uniform inside a group; groups of one
// wavefront diverge freely because no instruction mixes lanes of different
// groups.  HBM is read and written only at the start and end of a call and
// when the best scheme changes.
//
// The iteration follows Algorithm 1 (RandomWalk kernel, Sec. 3.4.2): a flip
// (Sec. 3.3.1) with ternary-safe arithmetic (Sec. 3.5.2) and sign
// normalisation (Sec. 3.6), zero-term removal, the best-scheme update,
// reduction with probability p_reduce, expand with probability p_expand near
// the best rank, and a plateau restart.  Every random word comes from one
// Philox4x32-10 block per (iteration, attempt, domain): at the start of an
// iteration lane q < G-1 of the group draws the block of flip attempt q and
// lane G-1 the per-iteration gate block, so the draws run in parallel and a
// skipped draw never shifts the stream.
//
// Three strategies search for a flip; all take the first attempt (in attempt
// order) that has a valid partner, so their results are identical:
//  * attempt-parallel (AP, schemes of at most 64*S terms, S = 1 or 2 words
//    per partner set): each lane evaluates one random attempt (term i, factor
//    kind X) against all terms -- a match scan over the X factors (two terms
//    per LDS read), then the validity of the two roles for the few matches;
//  * term-parallel (TP, any size): attempts run one after another and the G
//    lanes split the terms (slot q of lane l is term q*G + l), with one group
//    ballot per slot and role;
//  * indexed attempt-parallel (IX, at most 64 terms): AP over a match index
//    kept in LDS after the terms of the workgroup -- for every term k and
//    factor kind X a 64-bit mask of the other live terms whose factor X
//    equals that of k (w up to sign).  A flip changes two factors, so the index is refreshed in
//    one lane-parallel pass over the terms, and both the partner scan of an
//    attempt and the two-shared-factors search of a reduction become mask
//    lookups.
//
// The searches only choose a flip; one call site applies it.  Every costly
// step of an iteration (apply, removal, best copy, merge, expand, restart)
// has a single call site, so the walks of a wavefront that take a step in the
// same iteration take it in one pass.
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/tsf.h"
#include "tsf_bits.h"

namespace tsfk {

struct KArgs {
    uint64_t base_seed;
    uint64_t params_hash;  // tsf_params_hash of the call's parameters
    int64_t first_walk_id;
    int64_t max_iters;
    int64_t plateau;
    int64_t n_iters;
    uint64_t t_eq, t_reduce, t_expand;
    int32_t flip_tries;
    int32_t restart_from_best;
    int32_t objective;  // TSF_OBJ_RANK or TSF_OBJ_ADDITIONS
    int32_t n_walks;
    int32_t cap;
    int32_t rec_cap;
    int32_t mode;
    int32_t max_len;
    int32_t cap2;  // LDS stride per factor kind: cap rounded up to even (IX: to 4)
    int32_t capm;  // IX: row stride of the match masks (the capacity)
    tsf_walk_header *hdr;
    uint64_t *cur;
    uint64_t *best;
    const uint64_t *start;
    tsf_record *rec;
    // training log (uniform proposals); null = off
    tsf_flip_log *log;
    int32_t log_cap;
    // learned proposal: attempts scored per iteration, and the buffers
    int32_t learn_k;
    uint32_t *cand;      // 8 per walk
    uint16_t *feat;      // 8 rows of 512 bf16 per walk
    const float *logit;  // 8 per walk
    uint8_t *choice;     // choice_cap per walk, optional
    int32_t choice_cap;
    int32_t phase;       // 0: n_iters uniform iterations; 1: propose; 2: apply
};

constexpr int kLearnRows = 8;  // candidate rows per walk in the learned workspace

// bf16 bit patterns of +1 and -1
constexpr uint16_t kBf16One = 0x3F80, kBf16MinusOne = 0xBF80;

// Feature row of the proposal network (512 bf16): six blocks of 64 entries
// (+1 / -1 / 0 of the factors x_i y_i z_i x_j y_j z_j), the format one-hot at
// 384 + slot, the rank one-hot at 400 + min(rank, 95), zeros elsewhere.
__device__ __forceinline__ void write_feature_row(uint16_t *row, const uint64_t (&f)[12], int slot,
                                                  int rank)
{
    uint32_t *w32 = reinterpret_cast<uint32_t *>(row);
    for (int b = 0; b < 6; ++b) {
        const uint64_t d = f[2 * b], s = f[2 * b + 1];
#pragma unroll 4
        for (int e = 0; e < 64; e += 2) {
            const uint32_t lo = ((d >> e) & 1) ? (((s >> e) & 1) ? kBf16MinusOne : kBf16One) : 0u;
            const uint32_t hi =
                ((d >> (e + 1)) & 1) ? (((s >> (e + 1)) & 1) ? kBf16MinusOne : kBf16One) : 0u;
            w32[(b * 64 + e) >> 1] = lo | (hi << 16);
        }
    }
    const int fs = 384 + slot;
    const int rs = 400 + (rank < 95 ? (rank < 0 ? 0 : rank) : 95);
    for (int e = 384; e < 512; e += 2) {
        const uint32_t lo = (e == fs || e == rs) ? kBf16One : 0u;
        const uint32_t hi = (e + 1 == fs || e + 1 == rs) ? kBf16One : 0u;
        w32[e >> 1] = lo | (hi << 16);
    }
}

// role permutations (X,Y,Z) of (U,V,W), lexicographic
static __constant__ int8_t kPerm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2},
                                          {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};

template <typename T>
struct TV {
    T d, s;
};

// (the comparisons below use & and | rather than && and ||: both words are
// in registers already, and short-circuit forms compile to branches that can
// delay or split the LDS reads feeding them)
template <typename T>
__device__ __forceinline__ bool eqv(TV<T> a, TV<T> b)
{
    return (a.d == b.d) & (a.s == b.s);
}

// Order LDS accesses of the lanes of one wavefront: LDS instructions of a
// wavefront complete in issue order; this keeps the compiler from moving
// accesses across the point where one lane's store must be seen by others.
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int popc64(uint64_t x) { return __builtin_popcountll(x); }

// x ^= v on a 64-bit LDS word, as an atomic that returns nothing
__device__ __forceinline__ void lds_xor(uint64_t *p, uint64_t v)
{
    __hip_atomic_fetch_xor((__attribute__((address_space(3))) uint64_t *)p, v, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_WAVEFRONT);
}

// index of the c-th (0-based) set bit of m (m has more than c bits set)
__device__ __forceinline__ int kth_bit(uint64_t m, int c)
{
    for (int q = 0; q < c; ++q) m &= m - 1;
    return __builtin_ctzll(m);
}

// A set of term indexes below 64*NW, one bit per term (word q holds terms
// 64q .. 64q+63); the attempt-parallel partner sets
template <int NW>
struct TermSet {
    uint64_t w[NW];
    __device__ __forceinline__ void clear()
    {
#pragma unroll
        for (int q = 0; q < NW; ++q) w[q] = 0;
    }
    __device__ __forceinline__ bool any() const
    {
        uint64_t o = 0;
#pragma unroll
        for (int q = 0; q < NW; ++q) o |= w[q];
        return o != 0;
    }
    __device__ __forceinline__ int count() const
    {
        int c = 0;
#pragma unroll
        for (int q = 0; q < NW; ++q) c += __builtin_popcountll(w[q]);
        return c;
    }
    // removes and returns the lowest member (the set is not empty)
    __device__ __forceinline__ int pop()
    {
        if constexpr (NW == 1) {
            const int k = __builtin_ctzll(w[0]);
            w[0] &= w[0] - 1;
            return k;
        } else {
            // the first non-empty word, chosen with selects (no indexed
            // register access)
            int k = -1;
#pragma unroll
            for (int q = 0; q < NW; ++q) {
                const bool take = k < 0 && w[q] != 0;
                k = take ? 64 * q + __builtin_ctzll(w[q]) : k;
                w[q] = take ? w[q] & (w[q] - 1) : w[q];
            }
            return k;
        }
    }
    // adds member k when `on`
    __device__ __forceinline__ void set_if(int k, bool on)
    {
#pragma unroll
        for (int q = 0; q < NW; ++q)
            w[q] |= (on && (k >> 6) == q) ? 1ull << (k & 63) : 0ull;
    }
    // the c-th (0-based) member in ascending order (the set has more than c)
    __device__ __forceinline__ int kth(int c) const
    {
        if constexpr (NW == 1) {
            return kth_bit(w[0], c);
        } else {
            int k = -1;
#pragma unroll
            for (int q = 0; q < NW; ++q) {
                const int pc = __builtin_popcountll(w[q]);
                if (k < 0) {
                    if (c < pc)
                        k = 64 * q + kth_bit(w[q], c);
                    else
                        c -= pc;
                }
            }
            return k;
        }
    }
};

template <int G, int S, typename T, bool Z2, bool AP, bool IX, bool PK, bool CHK = false>
struct Walker {
    static_assert(!IX || AP, "the match index extends the attempt-parallel strategy");
    // PK: a factor of at most 16 entries is one 32-bit LDS word, digits in
    // bits 0..15 and signs in bits 16..31 (indexed kernels only)
    static_assert(!PK || (IX && sizeof(T) == 4), "packed factors: indexed kernels, 32-bit words");
    static constexpr int kFW = PK ? 1 : 2;  // LDS words per factor
    // attempt-parallel kernels: S is the number of 64-bit words of a partner
    // set (capacity up to 64*S); the indexed strategy keeps one word
    static_assert(!AP || S == 1 || (S == 2 && !IX), "attempt-parallel partner sets of 1 or 2 words");
    static constexpr int NW = AP ? S : 1;
    using PSet = TermSet<NW>;
    // group geometry
    int gl;      // lane within the group
    int gshift;  // first lane of the group within the wavefront
    int cap2;
    T *lds;
    uint64_t *mk;  // IX: match masks, mk[X*capm + k]
    int capm;      // IX: row stride of the masks (the capacity)
    // walk scalars, identical in every lane of the group
    uint64_t seed;
    int r, r_cap, best_rank, start_rank, target, n_rec;
    // additions objective: flips must keep every factor non-zero, the best
    // scheme is the one with the fewest non-zero coefficients
    bool additions;
    int nnz, best_nnz, mp;
    int64_t t, plateau_start;
    uint32_t cnt[C_NUM];
    const KArgs *a;
    int64_t walk;
    // this iteration's Philox block of this lane (attempt gl, or the gate)
    Philox4 pb;
    // the gate words (block (t, 0, 1), drawn by lane G-1), broadcast to the
    // group as soon as they are drawn
    uint32_t gate[3];
    // zero-factor flags of the two terms of the last flip
    bool zfi, zfj;
    // this iteration is written to the training log
    bool logging;
    int fmt_slot;
    // largest rank of the walks of this wavefront, rounded up to even: the
    // wave-uniform bound of the attempt-parallel match scan
    int scan_end;

    __device__ __forceinline__ void update_scan_end()
    {
        if constexpr (IX) return;
        int m = 0;
#pragma unroll
        for (int g = 0; g < 64 / G; ++g) m = max(m, __builtin_amdgcn_readlane(r, g * G));
        m = min(m, a->cap2);
        scan_end = (m + 1) & ~1;
    }

    __device__ __forceinline__ uint64_t gballot(bool p) const
    {
        uint64_t m = __ballot(p);
        if constexpr (G == 64)
            return m;
        else
            return (m >> gshift) & ((1ull << G) - 1);
    }
    // `lane` is the same in every lane of the group; the term-parallel kernels
    // with register slot copies (one group per wavefront) read it with a
    // scalar readlane instead of a lane permute
    __device__ __forceinline__ uint32_t from_lane(uint32_t v, int lane) const
    {
        if constexpr (G == 64 && kRegSlots)
            return (uint32_t)__builtin_amdgcn_readlane((int)v, lane);
        else
            return (uint32_t)__shfl((int)v, gshift + lane);
    }

    // The Philox block (iteration t, attempt att, domain dom) of this walk.
    // The key passes through an empty asm statement, so the compiler cannot
    // hoist the ten round keys of each half out of the iteration loop: they
    // are recomputed (one add per round and half, which the three-way xor
    // absorbs) instead of occupying twenty registers for the whole kernel.
    __device__ __forceinline__ Philox4 draw(uint32_t att, uint32_t dom) const
    {
        uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
        asm volatile("" : "+v"(k0), "+v"(k1));
        return philox4x32_10((uint32_t)(uint64_t)t, (uint32_t)((uint64_t)t >> 32), att, dom, k0, k1);
    }

    __device__ __forceinline__ int idx(int k, int X) const { return (X * cap2 + k) * kFW; }
    __device__ __forceinline__ static TV<T> unpack(T w) { return TV<T>{w & 0xFFFFu, w >> 16}; }
    // PK: the word held by every slot at or above the rank: signs without
    // digits, which no factor (nor a factor with its signs flipped) is, so a
    // comparison over a block of slots needs no mask of the live ones
    static constexpr uint32_t kDead = 0xFFFF0000u;
    // PK: store a packed word (lane 0 of the group)
    __device__ __forceinline__ void stw(int k, int X, T w)
    {
        if (gl == 0) lds[idx(k, X)] = w;
    }
    __device__ __forceinline__ static T pack(TV<T> v) { return v.d | (v.s << 16); }
    __device__ __forceinline__ TV<T> ld(int k, int X) const
    {
        const T *q = lds + idx(k, X);
        if constexpr (PK) return unpack(q[0]);
        return TV<T>{q[0], q[1]};
    }
    __device__ __forceinline__ void st(int k, int X, TV<T> v)
    {
        if (gl == 0) {
            T *q = lds + idx(k, X);
            if constexpr (PK) {
                q[0] = pack(v);
            } else {
                q[0] = v.d;
                q[1] = v.s;
            }
        }
    }

    __device__ __forceinline__ static bool axpy(int sigma, TV<T> x, TV<T> y, TV<T> &o)
    {
        if constexpr (Z2) {
            o.d = x.d ^ y.d;
            o.s = 0;
            return true;
        } else {
            return sigma > 0 ? tern_add(x.d, x.s, y.d, y.s, o.d, o.s)
                             : tern_sub(x.d, x.s, y.d, y.s, o.d, o.s);
        }
    }
    // +1 if y == x, -1 if y == -x (w only, ternary only), else 0
    __device__ __forceinline__ static int rel(TV<T> x, TV<T> y, int X)
    {
        if (eqv(x, y)) return 1;
        if constexpr (!Z2)
            if (X == 2 && tern_neg_eq(y.d, y.s, x.d, x.s)) return -1;
        return 0;
    }

    // factor X of two terms equal (w also when negated, ternary only): the
    // relation of the match index
    __device__ __forceinline__ static bool equiv(TV<T> x, TV<T> y, int X)
    {
        if constexpr (Z2) return x.d == y.d;
        return (x.d == y.d) & ((x.s == y.s) | ((X == 2) & ((x.s ^ x.d) == y.s)));
    }

    // largest rank of the walks of this wavefront (a wave-uniform loop bound)
    __device__ __forceinline__ int wave_max_r() const
    {
        int m = 0;
#pragma unroll
        for (int g = 0; g < 64 / G; ++g) m = max(m, __builtin_amdgcn_readlane(r, g * G));
        return min(m, a->cap);  // lanes of groups that left early hold no rank
    }

    // ------------------------------------------------------------ index (IX)
    // mk[X*capm + k], k < r: bit j set iff j != k, j < r and equiv(factor X
    // of j, factor X of k).  Built from scratch after a scheme is loaded.
    __device__ void build_index()
    {
        for (int k = gl; k < r; k += G) {
#pragma unroll
            for (int X = 0; X < 3; ++X) {
                const TV<T> xk = ld(k, X);
                uint64_t m = 0;
                for (int j = 0; j < r; ++j)
                    m |= (j != k && equiv(ld(j, X), xk, X)) ? (1ull << j) : 0ull;
                mk[X * capm + k] = m;
            }
        }
        wave_lds_sync();
    }

    // factor X of the four consecutive terms jb..jb+3 (jb a multiple of 4;
    // the IX layout pads cap2 to a multiple of 4) with 16-byte LDS reads
    __device__ __forceinline__ void load4(int jb, int X, TV<T> (&f)[4]) const
    {
        const T *q = lds + idx(jb, X);
        if constexpr (sizeof(T) == 4) {
            const uint4 a = *reinterpret_cast<const uint4 *>(q);
            const uint4 b = *reinterpret_cast<const uint4 *>(q + 4);
            f[0] = TV<T>{a.x, a.y};
            f[1] = TV<T>{a.z, a.w};
            f[2] = TV<T>{b.x, b.y};
            f[3] = TV<T>{b.z, b.w};
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const ulonglong2 v = *reinterpret_cast<const ulonglong2 *>(q + 2 * e);
                f[e] = TV<T>{(T)v.x, (T)v.y};
            }
        }
    }

    // Factor X1 of term k1 and factor X2 != X1 of term k2 have been given the
    // new values n1 and n2 (the two factors a flip changes; o1 and o2 are
    // their masks before the change).  For every live term j whose
    // relation to one of them changed, bit k of j's mask and bit j of k's mask
    // are toggled (LDS atomics, so no lane waits for a read-modify-write).
    // Lane l handles the four consecutive terms 4l .. 4l+3 of each block of
    // 4G terms.
    __device__ void refresh(int k1, int X1, TV<T> n1, uint64_t o1, int k2, int X2, TV<T> n2,
                            uint64_t o2)
    {
        // PK: the factors are compared as packed words; p = the new value,
        // q = the other accepted word (w negated: the signs flip where the
        // digits are set), equal to p where no sign freedom applies
        const T p1 = PK ? pack(n1) : 0, p2 = PK ? pack(n2) : 0;
        const T q1 = (PK && !Z2 && X1 == 2) ? (p1 ^ (p1 << 16)) : p1;
        const T q2 = (PK && !Z2 && X2 == 2) ? (p2 ^ (p2 << 16)) : p2;
        const uint64_t b1 = 1ull << k1, b2 = 1ull << k2;
        // passes of 4G terms while some walk of the wavefront has terms left
        for (int j0 = 0;; j0 += 4 * G) {
            const int jb = j0 + 4 * gl;
            if (jb < r) {
                // nibbles of the four terms: relation now, then changed ones
                uint32_t c1 = 0, c2 = 0;
                if constexpr (PK) {
                    const uint4 a1 = *reinterpret_cast<const uint4 *>(lds + idx(jb, X1));
                    const uint4 a2 = *reinterpret_cast<const uint4 *>(lds + idx(jb, X2));
                    const auto hit = [](T w, T p, T q) { return (w == p) | (w == q); };
                    c1 = (hit(a1.x, p1, q1) ? 1u : 0u) | (hit(a1.y, p1, q1) ? 2u : 0u) |
                         (hit(a1.z, p1, q1) ? 4u : 0u) | (hit(a1.w, p1, q1) ? 8u : 0u);
                    c2 = (hit(a2.x, p2, q2) ? 1u : 0u) | (hit(a2.y, p2, q2) ? 2u : 0u) |
                         (hit(a2.z, p2, q2) ? 4u : 0u) | (hit(a2.w, p2, q2) ? 8u : 0u);
                } else {
                    TV<T> f1[4], f2[4];
                    load4(jb, X1, f1);
                    load4(jb, X2, f2);
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        c1 |= equiv(f1[e], n1, X1) ? 1u << e : 0u;
                        c2 |= equiv(f2[e], n2, X2) ? 1u << e : 0u;
                    }
                }
                if constexpr (!PK) {
                    // slots at or above the rank hold stale terms
                    const uint32_t live = (r - jb >= 4 ? 0xFu : (1u << (r - jb)) - 1u);
                    c1 &= live;
                    c2 &= live;
                }
                // changed relations; a term is never in its own mask
                c1 = (c1 ^ (uint32_t)(o1 >> jb)) & ~(uint32_t)(b1 >> jb) & 0xFu;
                c2 = (c2 ^ (uint32_t)(o2 >> jb)) & ~(uint32_t)(b2 >> jb) & 0xFu;
                for (; c1; c1 &= c1 - 1) {
                    const int j = jb + __builtin_ctz(c1);
                    lds_xor(mk + X1 * capm + j, b1);
                    lds_xor(mk + X1 * capm + k1, 1ull << j);
                }
                for (; c2; c2 &= c2 - 1) {
                    const int j = jb + __builtin_ctz(c2);
                    lds_xor(mk + X2 * capm + j, b2);
                    lds_xor(mk + X2 * capm + k2, 1ull << j);
                }
            }
            if (!__ballot(j0 + 4 * G < r)) break;
        }
        wave_lds_sync();
    }

    // refresh() for one factor, one term per lane and round: used on the rare
    // paths (merges, expands), where code size and registers matter more
    __device__ void refresh_one(int k, int X, bool fresh)
    {
        const TV<T> nk = ld(k, X);
        const uint64_t o = fresh ? 0ull : mk[X * capm + k];
        if (fresh) {
            if (gl == 0) mk[X * capm + k] = 0;
            wave_lds_sync();
        }
#pragma unroll 1
        for (int j = gl; j < r; j += G) {
            const bool e = j != k && equiv(ld(j, X), nk, X);
            if (e != (((o >> j) & 1ull) != 0)) {
                lds_xor(mk + X * capm + j, 1ull << k);
                lds_xor(mk + X * capm + k, 1ull << j);
            }
        }
        wave_lds_sync();
    }

    // Sec. 3.6 on a term held in registers: first non-zero of u, then of v,
    // made positive; w absorbs.
    __device__ __forceinline__ static void normalise_regs(TV<T> (&f)[3])
    {
        if constexpr (!Z2) {
            const T lu = f[0].d & (~f[0].d + 1);
            if (f[0].s & lu) {
                f[0].s ^= f[0].d;
                f[2].s ^= f[2].d;
            }
            const T lv = f[1].d & (~f[1].d + 1);
            if (f[1].s & lv) {
                f[1].s ^= f[1].d;
                f[2].s ^= f[2].d;
            }
        }
    }
    __device__ void normalise(int k)
    {
        if constexpr (Z2) return;
        TV<T> f[3] = {ld(k, 0), ld(k, 1), ld(k, 2)};
        const T s0 = f[0].s, s1 = f[1].s;
        normalise_regs(f);
        if (f[0].s != s0 || f[1].s != s1) {
            st(k, 0, f[0]);
            st(k, 1, f[1]);
            st(k, 2, f[2]);
        }
        wave_lds_sync();
    }

    // swap-remove slot h (the last term moves into it); tracked indices follow
    __device__ void swap_remove(int h, int &tr0, int &tr1)
    {
        const int last = r - 1;
        if (tr0 == h) tr0 = -1;
        if (tr1 == h) tr1 = -1;
        if constexpr (IX) {
            // drop bit h from every mask; bit `last` becomes bit h, and the
            // masks of term `last` move to slot h
            const uint64_t bh = 1ull << h, bl = 1ull << last;
            for (int q = 0; q * G < r; ++q) {
                const int j = q * G + gl;
                if (j < r && j != h) {
                    const int dst = j == last ? h : j;
#pragma unroll
                    for (int X = 0; X < 3; ++X) {
                        uint64_t m = mk[X * capm + j] & ~bh;
                        if (m & bl) m = (m & ~bl) | bh;
                        mk[X * capm + dst] = m;
                    }
                }
            }
        }
        if constexpr (PK) {
            // slot `last` becomes a dead slot
            if (gl < 3) {
                if (h != last) lds[idx(h, gl)] = lds[idx(last, gl)];
                lds[idx(last, gl)] = kDead;
            }
        } else if (h != last) {
            for (int q = gl; q < 3 * kFW; q += G) {
                const int X = q / kFW, w = q % kFW;
                lds[idx(h, X) + w] = lds[idx(last, X) + w];
            }
        }
        if (h != last) {
            if (tr0 == last) tr0 = h;
            if (tr1 == last) tr1 = h;
        }
        wave_lds_sync();
        r = last;
    }

    // factor X (runtime) of a term held in three named registers; written as
    // selects on scalars so that no register array is indexed at run time
    __device__ __forceinline__ static TV<T> sel3(TV<T> f0, TV<T> f1, TV<T> f2, int X)
    {
        TV<T> o;
        o.d = X == 0 ? f0.d : (X == 1 ? f1.d : f2.d);
        o.s = X == 0 ? f0.s : (X == 1 ? f1.s : f2.s);
        return o;
    }
    __device__ __forceinline__ static void set3(TV<T> &f0, TV<T> &f1, TV<T> &f2, int X, TV<T> v)
    {
        f0.d = X == 0 ? v.d : f0.d;
        f0.s = X == 0 ? v.s : f0.s;
        f1.d = X == 1 ? v.d : f1.d;
        f1.s = X == 1 ? v.s : f1.s;
        f2.d = X == 2 ? v.d : f2.d;
        f2.s = X == 2 ? v.s : f2.s;
    }
    __device__ __forceinline__ void load_term(int k, TV<T> (&f)[3]) const
    {
        f[0] = ld(k, 0);
        f[1] = ld(k, 1);
        f[2] = ld(k, 2);
    }
    __device__ __forceinline__ void store_term(int k, const TV<T> (&f)[3])
    {
        st(k, 0, f[0]);
        st(k, 1, f[1]);
        st(k, 2, f[2]);
    }
    __device__ __forceinline__ static bool zero_factor(const TV<T> (&f)[3])
    {
        return f[0].d == 0 || f[1].d == 0 || f[2].d == 0;
    }

    // Flip (Sec. 3.3.1): x_j = sigma x_i; y_i += sigma y_j; z_j -= z_i;
    // (Y,Z) = the other kinds in U<V<W order, swapped for role 1.  Every live
    // term is normalised and has non-zero factors (the start scheme is
    // validated and every write keeps it so), so only y_i and z_j can become
    // zero, and normalising term i (j) only needs y_i (z_j) and w.  Returns
    // which of the two terms now has a zero factor.
    __device__ void apply_flip(int i, int j, int X, int role, bool &zi, bool &zj)
    {
        const int A = X == 0 ? 1 : 0, B = X == 2 ? 1 : 2;
        const int Y = role ? B : A, Z = role ? A : B;
        // every factor the flip reads is read up front (one round of reads);
        // PK: the sign is a comparison of packed words, and a w whose signs
        // flip is flipped as a packed word
        TV<T> xi, yi, zi0, xj, yj, zj0;
        T wxi = 0, wzi = 0, wxj = 0, wyj = 0;
        int sg;
        if constexpr (PK) {
            wxi = lds[idx(i, X)];
            wzi = lds[idx(i, Z)];
            wxj = lds[idx(j, X)];
            wyj = lds[idx(j, Y)];
            const T wyi = lds[idx(i, Y)], wzj = lds[idx(j, Z)];
            xi = unpack(wxi);
            yi = unpack(wyi);
            zi0 = unpack(wzi);
            xj = unpack(wxj);
            yj = unpack(wyj);
            zj0 = unpack(wzj);
            sg = (Z2 || wxi == wxj) ? 1 : -1;
        } else {
            xi = ld(i, X);
            yi = ld(i, Y);
            zi0 = ld(i, Z);
            xj = ld(j, X);
            yj = ld(j, Y);
            zj0 = ld(j, Z);
            sg = rel(xi, xj, X);
        }
        if (logging && gl == 0) {
            tsf_flip_log *lg = a->log + (size_t)walk * a->log_cap + (t - 1);
            const TV<T> fv[6] = {xi, yi, zi0, xj, yj, zj0};
#pragma unroll
            for (int q = 0; q < 6; ++q) {
                lg->f[2 * q] = (uint64_t)fv[q].d;
                lg->f[2 * q + 1] = (uint64_t)fv[q].s;
            }
            lg->rank_before = r;
        }
        TV<T> ny, nz;
        axpy(sg, yi, yj, ny);
        axpy(-1, zj0, zi0, nz);
        zi = ny.d == 0;
        zj = nz.d == 0;
        if (additions)
            nnz += popc64((uint64_t)ny.d) - popc64((uint64_t)yi.d) + popc64((uint64_t)nz.d) -
                   popc64((uint64_t)zj0.d);
        if constexpr (!Z2) {
            // Sec. 3.6: a u or v factor whose first non-zero entry is -1 is
            // negated, and w absorbs the sign (w of term i is x_i or z_i when
            // y is not w; w of term j is x_j or y_j when z is not w)
            if (Y != 2 && (ny.s & ny.d & (~ny.d + 1))) {
                ny.s ^= ny.d;
                if constexpr (PK) {
                    const T w = X == 2 ? wxi : wzi;
                    stw(i, 2, w ^ (w << 16));
                } else {
                    TV<T> w = X == 2 ? xi : zi0;
                    w.s ^= w.d;
                    st(i, 2, w);
                }
            }
            if (Z != 2 && (nz.s & nz.d & (~nz.d + 1))) {
                nz.s ^= nz.d;
                if constexpr (PK) {
                    const T w = X == 2 ? wxj : wyj;
                    stw(j, 2, w ^ (w << 16));
                } else {
                    TV<T> w = X == 2 ? xj : yj;
                    w.s ^= w.d;
                    st(j, 2, w);
                }
            }
        }
        if constexpr (IX) {
            const uint64_t oy = mk[Y * capm + i], oz = mk[Z * capm + j];
            st(i, Y, ny);
            st(j, Z, nz);
            if (!zi && !zj) {
                // the refresh compares the new factors (in registers) with
                // factors of other terms only, which these stores do not
                // change (w only up to sign), so it needs no barrier first
                refresh(i, Y, ny, oy, j, Z, nz, oz);
                return;
            }
            wave_lds_sync();
            // a term with a zero factor is removed next, and its removal
            // clears its bit from every mask: only a survivor is refreshed
            if (!zi || !zj) refresh_one(!zi ? i : j, !zi ? Y : Z, false);
            return;
        }
        st(i, Y, ny);
        st(j, Z, nz);
        wave_lds_sync();
    }

    // random words of flip attempt `att`: from the lane that drew them in this
    // iteration's batch, or drawn now (uniformly by the whole group)
    __device__ __forceinline__ void attempt_words(int att, uint32_t &w0, uint32_t &w1,
                                                  uint32_t &w2)
    {
        if (att < G - 1) {
            w0 = from_lane(pb.x[0], att);
            w1 = from_lane(pb.x[1], att);
            w2 = from_lane(pb.x[2], att);
        } else {
            const Philox4 w = draw((uint32_t)att, 0);
            w0 = w.x[0];
            w1 = w.x[1];
            w2 = w.x[2];
        }
    }

    // ------------------------------------------------------------------ TP
    // With four to seven slots per lane the three factors of this lane's S
    // terms (k = q*G + lane, indexes clamped to the rows) are read in one
    // round: the attempts and the cyclic search of an iteration compare
    // against these registers, since no term changes before a flip is
    // chosen.  With fewer slots each attempt reads the factors it compares
    // (measured faster there); eight slots of copies would not fit in 256
    // VGPRs.
    static constexpr bool kRegSlots = !AP && S >= 4 && S <= 7;
    __device__ __forceinline__ void load_slots(TV<T> (&F)[S][3]) const
    {
        if constexpr (!kRegSlots) return;
#pragma unroll
        for (int q = 0; q < S; ++q) {
            const int k = q * G + gl;
            load_term(k < cap2 ? k : cap2 - 1, F[q]);
        }
    }

    // Candidate partners of (i, X): lane-parallel over the terms, one ballot
    // per slot and role.  m0/m1: role 0/1 masks (bit = lane of slot q).
    // Factor X of every slot is compared first (read back to back at indexes
    // clamped to the walk's rows, or taken from F); the validity of the two
    // roles is evaluated only when some lane of the group has a match.
    __device__ void candidates_tp(int i, int X, const TV<T> (&F)[S][3], uint64_t (&m0)[S],
                                  uint64_t (&m1)[S], int &n0, int &n1) const
    {
        if constexpr (kRegSlots) {
            // X is wave-uniform: one specialisation per kind, so the slot
            // factors are picked from F at compile time
            if (X == 0)
                candidates_tp_x<0>(i, F, m0, m1, n0, n1);
            else if (X == 1)
                candidates_tp_x<1>(i, F, m0, m1, n0, n1);
            else
                candidates_tp_x<2>(i, F, m0, m1, n0, n1);
        } else {
            candidates_tp_lds(i, X, m0, m1, n0, n1);
        }
    }

    // the same from LDS, one code path for the three kinds (the smaller code
    // measured faster with few slots)
    __device__ void candidates_tp_lds(int i, int X, uint64_t (&m0)[S], uint64_t (&m1)[S],
                                      int &n0, int &n1) const
    {
        const int A = X == 0 ? 1 : 0, B = X == 2 ? 1 : 2;
        const TV<T> xi = ld(i, X);
        int sg[S];
        bool any = false;
#pragma unroll
        for (int q = 0; q < S; ++q) {
            const int k = q * G + gl;
            const TV<T> xk = ld(k < cap2 ? k : cap2 - 1, X);
            sg[q] = (k < r && k != i) ? rel(xi, xk, X) : 0;
            any |= sg[q] != 0;
        }
        // m0/m1 are read by the caller only when n0 + n1 > 0
        n0 = n1 = 0;
        if (!gballot(any)) return;
        const TV<T> Ai = ld(i, A), Bi = ld(i, B);
        uint32_t c0 = 0, c1 = 0;
#pragma unroll
        for (int q = 0; q < S; ++q) {
            if (sg[q] != 0) {
                const int k = q * G + gl;
                const TV<T> Ak = ld(k, A), Bk = ld(k, B);
                TV<T> o1, o2;
                const bool a1 = axpy(sg[q], Ai, Ak, o1), b1 = axpy(-1, Bk, Bi, o2);
                const bool a2 = axpy(sg[q], Bi, Bk, o1), b2 = axpy(-1, Ak, Ai, o2);
                const bool keep = !additions || (Ai.d != Ak.d && Bi.d != Bk.d);
                c0 |= (a1 && b1 && keep) ? 1u << q : 0u;
                c1 |= (a2 && b2 && keep) ? 1u << q : 0u;
            }
        }
        if (!gballot((c0 | c1) != 0)) return;
#pragma unroll
        for (int q = 0; q < S; ++q) {
            m0[q] = gballot((c0 >> q) & 1u);
            m1[q] = gballot((c1 >> q) & 1u);
            n0 += popc64(m0[q]);
            n1 += popc64(m1[q]);
        }
    }

    template <int X>
    __device__ void candidates_tp_x(int i, const TV<T> (&F)[S][3], uint64_t (&m0)[S],
                                    uint64_t (&m1)[S], int &n0, int &n1) const
    {
        constexpr int A = X == 0 ? 1 : 0, B = X == 2 ? 1 : 2;
        // term i's factors (one broadcast round of reads; taking them from
        // the registers of the lane that holds term i measured slower)
        const TV<T> xi = ld(i, X), Ai = ld(i, A), Bi = ld(i, B);
        int sg[S];
        bool any = false;
#pragma unroll
        for (int q = 0; q < S; ++q) {
            const int k = q * G + gl;
            sg[q] = (k < r && k != i) ? rel(xi, F[q][X], X) : 0;
            any |= sg[q] != 0;
        }
        // m0/m1 are read by the caller only when n0 + n1 > 0
        n0 = n1 = 0;
        if (!gballot(any)) return;
        // the validity of the two roles per slot, as bits of this lane; the
        // group's sets are built only for an attempt with a valid partner
        uint32_t c0 = 0, c1 = 0;
#pragma unroll
        for (int q = 0; q < S; ++q) {
            if (sg[q] != 0) {
                const TV<T> Ak = F[q][A], Bk = F[q][B];
                TV<T> o1, o2;
                const bool a1 = axpy(sg[q], Ai, Ak, o1), b1 = axpy(-1, Bk, Bi, o2);
                const bool a2 = axpy(sg[q], Bi, Bk, o1), b2 = axpy(-1, Ak, Ai, o2);
                const bool keep = !additions || (Ai.d != Ak.d && Bi.d != Bk.d);
                c0 |= (a1 && b1 && keep) ? 1u << q : 0u;
                c1 |= (a2 && b2 && keep) ? 1u << q : 0u;
            }
        }
        if (!gballot((c0 | c1) != 0)) return;
#pragma unroll
        for (int q = 0; q < S; ++q) {
            m0[q] = gballot((c0 >> q) & 1u);
            m1[q] = gballot((c1 >> q) & 1u);
            n0 += popc64(m0[q]);
            n1 += popc64(m1[q]);
        }
    }

    __device__ __forceinline__ int select_tp(const uint64_t (&m)[S], int c) const
    {
        int j = -1;
#pragma unroll
        for (int q = 0; q < S; ++q) {
            const int pc = popc64(m[q]);
            if (j < 0) {
                if (c < pc)
                    j = q * G + kth_bit(m[q], c);
                else
                    c -= pc;
            }
        }
        return j;
    }

    // ------------------------------------------------------------------ AP
    // Partners of attempt (i, X) for this lane (when `active`), over all
    // r <= 64*NW terms: member k of m0/m1 when (k, role 0/1) is a valid flip
    // partner.  The match scan runs to the batch capacity (a wave-uniform
    // bound, so the loop counter and the bit constants stay scalar; 32 terms
    // per partial mask) and drops terms >= r.  Then the matches are tested
    // one at a time.  (Stopping the lanes after the first lane of the group
    // that has a partner measured slower: 10% with a group ballot after
    // every match, 2% with one ballot after the first.)
    __device__ void candidates_ap(bool active, int i, int X, PSet &m0, PSet &m1) const
    {
        m0.clear();
        m1.clear();
        PSet match;
        match.clear();
        TV<T> xi{0, 0};
        if (active) {
            xi = ld(i, X);
            if constexpr (IX) {
                match.w[0] = mk[X * capm + i];
            } else {
                const T nsi = (!Z2 && X == 2) ? (xi.s ^ xi.d) : xi.s;  // accepted signs besides xi.s
                const T *col = lds + idx(0, X);
                const int kend = scan_end;  // even, wave-uniform
                uint32_t part[2 * NW];
                int k = 0;
#pragma unroll
                for (int c = 0; c < 2 * NW; ++c) {
                    part[c] = 0;
                    const int kc = kend < 32 * (c + 1) ? kend : 32 * (c + 1);
                    // four terms per step while four remain, then two
                    for (; k + 2 < kc; k += 4) {
                        const T d0 = col[2 * k], s0 = col[2 * k + 1], d1 = col[2 * k + 2],
                                s1 = col[2 * k + 3], d2 = col[2 * k + 4], s2 = col[2 * k + 5],
                                d3 = col[2 * k + 6], s3 = col[2 * k + 7];
                        const int sh = k - 32 * c;
                        part[c] |= ((d0 == xi.d) & ((s0 == xi.s) | (s0 == nsi)) ? 1u : 0u) << sh;
                        part[c] |= ((d1 == xi.d) & ((s1 == xi.s) | (s1 == nsi)) ? 2u : 0u) << sh;
                        part[c] |= ((d2 == xi.d) & ((s2 == xi.s) | (s2 == nsi)) ? 4u : 0u) << sh;
                        part[c] |= ((d3 == xi.d) & ((s3 == xi.s) | (s3 == nsi)) ? 8u : 0u) << sh;
                    }
                    if (k < kc) {
                        const T d0 = col[2 * k], s0 = col[2 * k + 1], d1 = col[2 * k + 2],
                                s1 = col[2 * k + 3];
                        const uint32_t b0 = 1u << (k - 32 * c), b1 = 2u << (k - 32 * c);
                        part[c] |= (d0 == xi.d && (s0 == xi.s || s0 == nsi)) ? b0 : 0u;
                        part[c] |= (d1 == xi.d && (s1 == xi.s || s1 == nsi)) ? b1 : 0u;
                        k += 2;
                    }
                }
#pragma unroll
                for (int q = 0; q < NW; ++q) {
                    const int lo = 64 * q;
                    const uint64_t live = r - lo >= 64 ? ~0ull : (r > lo ? (1ull << (r - lo)) - 1 : 0ull);
                    const uint64_t self = (i >> 6) == q ? 1ull << (i & 63) : 0ull;
                    match.w[q] = (((uint64_t)part[2 * q + 1] << 32) | part[2 * q]) & live & ~self;
                }
            }
        }
        if (!match.any()) return;
        const int A = X == 0 ? 1 : 0, B = X == 2 ? 1 : 2;
        // the factors of term i that the tests read (packed words for PK)
        T wx = 0, wa = 0, wb = 0;
        TV<T> Ai{0, 0}, Bi{0, 0};
        if constexpr (PK) {
            wx = lds[idx(i, X)];
            wa = lds[idx(i, A)];
            wb = lds[idx(i, B)];
        } else {
            Ai = ld(i, A);
            Bi = ld(i, B);
        }
        // the two roles of the flip with term kk
        const auto roles = [&](int kk, bool &v0, bool &v1) {
            if constexpr (PK) {
                roles_packed(wx, wa, wb, lds[idx(kk, X)], lds[idx(kk, A)], lds[idx(kk, B)],
                             v0, v1);
            } else {
                const int sg = (Z2 || ld(kk, X).s == xi.s) ? 1 : -1;
                const TV<T> Ak = ld(kk, A), Bk = ld(kk, B);
                TV<T> o1, o2;
                const bool a1 = axpy(sg, Ai, Ak, o1), b1 = axpy(-1, Bk, Bi, o2);
                const bool a2 = axpy(sg, Bi, Bk, o1), b2 = axpy(-1, Ak, Ai, o2);
                // a valid sum or difference is zero exactly when the
                // supports agree; the additions objective admits no such
                // flip
                const bool keep = !additions || (Ai.d != Ak.d && Bi.d != Bk.d);
                v0 = a1 && b1 && keep;
                v1 = a2 && b2 && keep;
            }
        };
        if (NW == 2 && !__ballot(r > 64)) {
            // two-word sets, but no walk of the wavefront has more than 64
            // terms: one word holds every match
            uint64_t mm = match.w[0], s0 = 0, s1 = 0;
            do {
                const int kk = __builtin_ctzll(mm);
                mm &= mm - 1;
                bool v0, v1;
                roles(kk, v0, v1);
                s0 |= (v0 ? 1ull : 0ull) << kk;
                s1 |= (v1 ? 1ull : 0ull) << kk;
            } while (mm);
            m0.w[0] = s0;
            m1.w[0] = s1;
            return;
        }
        if (NW == 1 && !__ballot(r > 32)) {
            // every walk of the wavefront has at most 32 terms: the sets fit
            // in 32-bit words
            uint32_t mm = (uint32_t)match.w[0], s0 = 0, s1 = 0;
            do {
                const int kk = __builtin_ctz(mm);
                mm &= mm - 1;
                bool v0, v1;
                roles(kk, v0, v1);
                s0 |= (v0 ? 1u : 0u) << kk;
                s1 |= (v1 ? 1u : 0u) << kk;
            } while (mm);
            m0.w[0] = s0;
            m1.w[0] = s1;
            return;
        }
        do {
            const int kk = match.pop();
            bool v0, v1;
            roles(kk, v0, v1);
            m0.set_if(kk, v0);
            m1.set_if(kk, v1);
        } while (match.any());
    }

    // The validity tests of candidates_ap on packed words (digits in bits
    // 0..15, signs in 16..31): x, a, b = factors X, A, B of term i; xk, ak, bk
    // those of term k.  Where both factors are non-zero, equal signs make a
    // sum leave the set and different signs a difference (Sec. 3.5.2).
    // Role 0 needs a_i + sigma a_k and b_k - b_i, role 1 b_i + sigma b_k and
    // a_k - a_i; sigma = +1 unless w_k = -w_i.
    __device__ __forceinline__ void roles_packed(T x, T a, T b, T xk, T ak, T bk, bool &v0,
                                                 bool &v1) const
    {
        const T xa = a ^ ak, xb = b ^ bk;
        bool keep = true;
        if (additions) keep = ((xa & 0xFFFFu) != 0) & ((xb & 0xFFFFu) != 0);
        if constexpr (Z2) {
            v0 = v1 = keep;
        } else {
            const T ya = xa >> 16, yb = xb >> 16;
            const T ba = a & ak & 0xFFFFu, bb = b & bk & 0xFFFFu;
            const bool da = (ba & ya) == 0, db = (bb & yb) == 0;    // no opposite signs
            const bool sa = (ba & ~ya) == 0, sb = (bb & ~yb) == 0;  // no equal signs
            const bool pos = xk == x;
            v0 = (pos ? sa : da) & db & keep;
            v1 = (pos ? sb : db) & da & keep;
        }
    }

    // ------------------------------------------------------------------ flip
    // A chosen flip, packed: i | j << 10 | X << 20 | role << 22 (terms below
    // 1024; kNoFlip: none)
    static constexpr uint32_t kNoFlip = ~0u;
    __device__ __forceinline__ static uint32_t pack_flip(int i, int j, int X, int role)
    {
        return (uint32_t)i | ((uint32_t)j << 10) | ((uint32_t)X << 20) | ((uint32_t)role << 22);
    }
    __device__ __forceinline__ void apply_packed(uint32_t d, int &fi, int &fj)
    {
        fi = d & 0x3FF;
        fj = (d >> 10) & 0x3FF;
        apply_flip(fi, fj, (d >> 20) & 3, (d >> 22) & 1, zfi, zfj);
    }

    // The searches (attempts, then the cyclic fallback) only choose the flip;
    // it is applied at one point afterwards, so a wavefront whose walks took
    // different searches applies their flips together.
    __device__ bool try_flip(int &fi, int &fj)
    {
        if (r < 2) return false;
        const uint32_t pick = choose_flip();
        if (pick == kNoFlip) return false;
        apply_packed(pick, fi, fj);
        return true;
    }

    __device__ uint32_t choose_flip()
    {
        const int T_ = a->flip_tries;
        if constexpr (AP) {
            update_scan_end();
            constexpr int P = G - 1;  // attempts per batch
            for (int base = 0; base < T_; base += P) {
                const int att = base + gl;
                const bool active = gl < P && att < T_;
                uint32_t w0, w1, w2;
                if (base == 0) {
                    w0 = pb.x[0];
                    w1 = pb.x[1];
                    w2 = pb.x[2];
                } else {
                    const Philox4 w = draw((uint32_t)att, 0);
                    w0 = w.x[0];
                    w1 = w.x[1];
                    w2 = w.x[2];
                }
                const int i = (int)below(w0, (uint32_t)r);
                const int X = (int)below(w1, 3u);
                PSet m0, m1;
                m0.clear();
                m1.clear();
                candidates_ap(active, i, X, m0, m1);
                const int n0 = m0.count(), n = n0 + m1.count();
                const uint64_t ok = gballot(n > 0);
                if (ok) {
                    const int win = __builtin_ctzll(ok);
                    uint32_t pick = 0;
                    if (gl == win) {
                        int c = (int)below(w2, (uint32_t)n);
                        const int role = c >= n0;
                        if (role) c -= n0;
                        const int j = (role ? m1 : m0).kth(c);  // one search, on the chosen set
                        pick = pack_flip(i, j, X, role);
                    }
                    cnt[C_ATTEMPTS] += (uint32_t)(base + win + 1);
                    return from_lane(pick, win);
                }
            }
            cnt[C_ATTEMPTS] += (uint32_t)T_;
            return fallback_ap();
        } else {
            TV<T> F[S][3];
            load_slots(F);
            uint64_t m0[S], m1[S];
            int n0, n1;
            for (int att = 0; att < T_; ++att) {
                uint32_t w0, w1, w2;
                attempt_words(att, w0, w1, w2);
                cnt[C_ATTEMPTS]++;
                const int i = (int)below(w0, (uint32_t)r);
                const int X = (int)below(w1, 3u);
                candidates_tp(i, X, F, m0, m1, n0, n1);
                const int n = n0 + n1;
                if (n > 0) {
                    int c = (int)below(w2, (uint32_t)n);
                    const int role = c >= n0;
                    if (role) c -= n0;
                    const int j = role ? select_tp(m1, c) : select_tp(m0, c);
                    return pack_flip(i, j, X, role);
                }
            }
            return fallback_tp(F);
        }
    }

    // When every attempt failed: the unused fourth words of the blocks of
    // attempts 0 and 1 (drawn by lanes 0 and 1 of the group) give a starting
    // pair p0 = U(w3 of (t,0,0), 3r); the pairs p = 3i + X are visited
    // cyclically from p0 and the first pair with a valid partner yields
    // candidate U(w3 of (t,1,0), n).  None at all: a dead end.
    __device__ uint32_t fallback_tp(const TV<T> (&F)[S][3])
    {
        cnt[C_FALLBACKS]++;
        uint64_t m0[S], m1[S];
        int n0, n1;
        const uint32_t f0 = from_lane(pb.x[3], 0), f1 = from_lane(pb.x[3], 1);
        const int npairs = 3 * r;
        const int p0 = (int)below(f0, (uint32_t)npairs);
        for (int q = 0; q < npairs; ++q) {
            int p = p0 + q;
            if (p >= npairs) p -= npairs;
            const int i = p / 3, X = p - 3 * i;
            candidates_tp(i, X, F, m0, m1, n0, n1);
            const int n = n0 + n1;
            if (n == 0) continue;
            int c = (int)below(f1, (uint32_t)n);
            const int role = c >= n0;
            if (role) c -= n0;
            const int j = role ? select_tp(m1, c) : select_tp(m0, c);
            return pack_flip(i, j, X, role);
        }
        return kNoFlip;
    }

    // The same search with G consecutive pairs per round, one per lane; the
    // first lane (in pair order) with a partner wins.
    __device__ uint32_t fallback_ap()
    {
        cnt[C_FALLBACKS]++;
        const uint32_t f0 = from_lane(pb.x[3], 0), f1 = from_lane(pb.x[3], 1);
        const int npairs = 3 * r;
        const int p0 = (int)below(f0, (uint32_t)npairs);
        for (int base = 0; base < npairs; base += G) {
            const int q = base + gl;
            int p = p0 + q;
            if (p >= npairs) p -= npairs;
            const int i = p / 3, X = p - 3 * i;
            PSet m0, m1;
            m0.clear();
            m1.clear();
            candidates_ap(q < npairs, i, X, m0, m1);
            const int n0 = m0.count(), n = n0 + m1.count();
            const uint64_t ok = gballot(n > 0);
            if (ok) {
                const int win = __builtin_ctzll(ok);
                uint32_t packed = 0;
                if (gl == win) {
                    int c = (int)below(f1, (uint32_t)n);
                    const int role = c >= n0;
                    if (role) c -= n0;
                    const int j = (role ? m1 : m0).kth(c);  // one search, on the chosen set
                    packed = pack_flip(i, j, X, role);
                }
                return from_lane(packed, win);
            }
        }
        return kNoFlip;
    }

    // ------------------------------------------------------------------ reduce
    // Reduction (Sec. 3.3.1) between terms t and k: shared (u,v) merges w,
    // shared (u, +-w) merges v, shared (v, +-w) merges u; returns the kind
    // merged or -1 when no merge keeps the coefficients in the set.
    __device__ __forceinline__ static int merge_kind(const TV<T> (&tt)[3], const TV<T> (&tk)[3],
                                                     TV<T> &o)
    {
        const bool eu = eqv(tt[0], tk[0]), ev = eqv(tt[1], tk[1]);
        const int sw = rel(tt[2], tk[2], 2);
        if (eu && ev && axpy(1, tt[2], tk[2], o)) return 2;
        if (eu && sw != 0 && axpy(sw, tt[1], tk[1], o)) return 1;
        if (ev && sw != 0 && axpy(sw, tt[0], tk[0], o)) return 0;
        return -1;
    }

    // two or more shared factors (w up to sign): the precondition of a merge
    __device__ __forceinline__ static bool shares_two(const TV<T> (&tt)[3], const TV<T> (&tk)[3])
    {
        const bool eu = eqv(tt[0], tk[0]), ev = eqv(tt[1], tk[1]);
        const bool ew = tk[2].d == tt[2].d &&
                        (tk[2].s == tt[2].s || (!Z2 && tk[2].s == (tt[2].s ^ tt[2].d)));
        return (eu && ev) || (eu && ew) || (ev && ew);
    }

    // First term k (ascending) that merges with term ia (k != ia) and with
    // term ib (k != ib), in one pass over the terms; -1 where there is none
    // or the tracked index is -1.  The slot loop has a wave-uniform bound, and
    // the merge validity is evaluated only when some lane shares two factors.
    __device__ void find_merges(int ia, const TV<T> (&ta)[3], int ib, const TV<T> (&tb)[3],
                                int &ka, int &kb) const
    {
        ka = kb = -1;
        if constexpr (IX) {
            const uint64_t ca = ia >= 0 ? two_shared(ia) : 0ull;
            const uint64_t cb = ib >= 0 ? two_shared(ib) : 0ull;
            ka = first_merge(ca, ta);
            kb = first_merge(cb, tb);
            return;
        }
        // U slots per round, their terms read before any is compared (indexes
        // clamped to the walk's rows), so the reads of a round overlap; the
        // term-parallel kernels with four to seven slots read all at once
        constexpr int U = kRegSlots ? S : 2;
        const int qend = (wave_max_r() + G - 1) / G;
#pragma unroll 1
        for (int q0 = 0; q0 < qend; q0 += U) {
            TV<T> tk[U][3];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int kk = (q0 + u) * G + gl;
                load_term(kk < cap2 ? kk : cap2 - 1, tk[u]);
            }
            bool oka[U], okb[U], any = false;
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int kk = (q0 + u) * G + gl;
                const bool live = kk < r;
                oka[u] = live && ia >= 0 && kk != ia && shares_two(ta, tk[u]);
                okb[u] = live && ib >= 0 && kk != ib && shares_two(tb, tk[u]);
                any |= oka[u] || okb[u];
            }
            // usually no term of these slots shares two factors with either
            if (!__ballot(any)) continue;
#pragma unroll
            for (int u = 0; u < U; ++u) {
                TV<T> o;
                oka[u] = oka[u] && merge_kind(ta, tk[u], o) >= 0;
                okb[u] = okb[u] && merge_kind(tb, tk[u], o) >= 0;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint64_t ma = gballot(oka[u]), mb = gballot(okb[u]);
                if (ka < 0 && ma) ka = (q0 + u) * G + __builtin_ctzll(ma);
                if (kb < 0 && mb) kb = (q0 + u) * G + __builtin_ctzll(mb);
            }
        }
    }

    // IX: the terms sharing two factors with term ti are the pairwise
    // intersections of its three masks (two_shared); first_merge returns the
    // first of them (ascending) whose merge keeps the coefficients in the
    // set, or -1
    __device__ __forceinline__ uint64_t two_shared(int ti) const
    {
        const uint64_t mu = mk[ti], mv = mk[capm + ti], mw = mk[2 * capm + ti];
        return (mu & mv) | (mu & mw) | (mv & mw);
    }
    __device__ int first_merge(uint64_t c, const TV<T> (&tt)[3]) const
    {
        for (; c; c &= c - 1) {
            const int k = __builtin_ctzll(c);
            TV<T> tk[3], o;
            load_term(k, tk);
            if (merge_kind(tt, tk, o) >= 0) return k;
        }
        return -1;
    }

    // merge term k into tracked term qq (Sec. 3.3.1 reduction); the merged
    // term takes slot min(t,k) and slot max(t,k) is swap-removed; a merged
    // factor of zero removes both terms.
    __device__ void merge_into(int qq, int k, int &tr0, int &tr1)
    {
        const int tt_i = qq == 0 ? tr0 : tr1;
        TV<T> tt[3], tk[3];
        load_term(tt_i, tt);
        load_term(k, tk);
        TV<T> md;
        const int kind = merge_kind(tt, tk, md);
        const int lo = tt_i < k ? tt_i : k, hi = tt_i < k ? k : tt_i;
        // the partner is consumed
        if (qq == 0 && tr1 == k) tr1 = -1;
        if (qq == 1 && tr0 == k) tr0 = -1;
        const bool vanish = md.d == 0;
        if (!vanish) {
            TV<T> nt[3] = {kind == 0 ? md : tt[0], kind == 1 ? md : tt[1],
                           kind == 2 ? md : tt[2]};
            normalise_regs(nt);
            store_term(lo, nt);
            wave_lds_sync();
            if constexpr (IX) {
                // the merged factor is new at slot lo; the two shared factors
                // are those of the term that held lo (w possibly negated,
                // which the index ignores)
                refresh_one(lo, kind, false);
            }
        }
        // the merged term keeps slot lo, or (a zero merged factor) both go
        if (qq == 0)
            tr0 = vanish ? -1 : lo;
        else
            tr1 = vanish ? -1 : lo;
        swap_remove(hi, tr0, tr1);
        if (vanish) swap_remove(lo, tr0, tr1);
    }

    // Reduce the two terms modified by the flip, cascading: the first tracked
    // term merges until it has no partner left, then the second.  Both are
    // looked up in one pass; the second term's result of a pass is used once
    // the first one is finished (nothing changed in between).  Returns merges.
    __device__ int reduce(int &tr0, int &tr1)
    {
        int merges = 0;
        if constexpr (IX) {
            // the common case: neither modified term shares two factors with
            // another term (six mask reads, no term loads)
            const uint64_t ca = tr0 >= 0 ? two_shared(tr0) : 0ull;
            const uint64_t cb = tr1 >= 0 ? two_shared(tr1) : 0ull;
            if ((ca | cb) == 0) return 0;
        }
        bool done0 = tr0 < 0;
        for (;;) {
            const int ia = done0 ? -1 : tr0, ib = tr1;
            if (ia < 0 && ib < 0) break;
            TV<T> ta[3] = {}, tb[3] = {};
            if (ia >= 0) load_term(ia, ta);
            if (ib >= 0) load_term(ib, tb);
            int ka, kb;
            find_merges(ia, ta, ib, tb, ka, kb);
            // the first tracked term merges while it has a partner, then the
            // second (one merge_into call site)
            int qq = -1, k = -1;
            if (!done0) {
                if (ka >= 0) {
                    qq = 0;
                    k = ka;
                } else {
                    done0 = true;
                }
            }
            if (qq < 0) {
                if (ib < 0 || kb < 0) break;
                qq = 1;
                k = kb;
            }
            ++merges;
            merge_into(qq, k, tr0, tr1);
            if (qq == 0 && tr0 < 0) done0 = true;
        }
        return merges;
    }

    // ------------------------------------------------------------------ expand
    // plus or split (Sec. 3.3.1), up to eight random attempts
    __device__ bool expand()
    {
        if (r >= r_cap || r < 2) return false;
        for (int att = 0; att < 8; ++att) {
            const Philox4 w = draw((uint32_t)att, 2);
            const int i = (int)below(w.x[0], (uint32_t)r);
            int j = (int)below(w.x[1], (uint32_t)(r - 1));
            if (j >= i) ++j;
            const int perm = (int)below(w.x[2], 6u);
            const int X = kPerm[perm][0], Y = kPerm[perm][1], Z = kPerm[perm][2];
            const TV<T> xi = ld(i, X), yi = ld(i, Y), zi = ld(i, Z);
            const TV<T> xj = ld(j, X), yj = ld(j, Y), zj = ld(j, Z);
            const int nw = r;
            if ((w.x[3] >> 31) == 0) {
                // plus: x_i(x)(y_i+y_j)(x)z_i + x_i(x)y_j(x)(z_j-z_i) + (x_j-x_i)(x)y_j(x)z_j
                if (eqv(xi, xj) || eqv(yi, yj) || eqv(zi, zj)) continue;
                TV<T> sa, sb, sc;
                if (!axpy(1, yi, yj, sa) || sa.d == 0) continue;
                if (!axpy(-1, zj, zi, sb)) continue;
                if (!axpy(-1, xj, xi, sc)) continue;
                st(nw, X, sc);
                st(nw, Y, yj);
                st(nw, Z, zj);
                st(j, X, xi);
                st(j, Z, sb);
                st(i, Y, sa);
            } else {
                // split: x_j(x)y_i(x)z_i + x_j(x)y_j(x)z_j + (x_i-x_j)(x)y_i(x)z_i
                if (eqv(xi, xj)) continue;
                TV<T> sc;
                if (!axpy(-1, xi, xj, sc)) continue;
                st(nw, X, sc);
                st(nw, Y, yi);
                st(nw, Z, zi);
                st(i, X, xj);
            }
            wave_lds_sync();
            r = nw + 1;
            normalise(i);
            normalise(j);
            normalise(nw);
            if constexpr (IX) {
                // one factor at a time: each refresh starts from masks that
                // are exact for every factor already refreshed
#pragma unroll 1
                for (int x = 0; x < 3; ++x) refresh_one(nw, x, true);
#pragma unroll 1
                for (int x = 0; x < 3; ++x) refresh_one(i, x, false);
#pragma unroll 1
                for (int x = 0; x < 3; ++x) refresh_one(j, x, false);
            }
            cnt[C_EXPANDS]++;
            return true;
        }
        cnt[C_EXPAND_FAILS]++;
        return false;
    }

    // ------------------------------------------------------------------ HBM
    // HBM holds terms as 6 consecutive uint64 (u.d u.s v.d v.s w.d w.s); lane
    // l of the group moves terms l, l+G, ...
    __device__ void load_scheme(const uint64_t *src, int rr)
    {
        for (int k = gl; k < rr; k += G)
#pragma unroll
            for (int X = 0; X < 3; ++X) {
                const TV<T> v{(T)src[k * 6 + 2 * X], (T)src[k * 6 + 2 * X + 1]};
                T *q = lds + idx(k, X);
                if constexpr (PK) {
                    q[0] = pack(v);
                } else {
                    q[0] = v.d;
                    q[1] = v.s;
                }
            }
        if constexpr (PK)
            for (int k = rr + gl; k < cap2; k += G)
#pragma unroll
                for (int X = 0; X < 3; ++X) lds[idx(k, X)] = kDead;
        wave_lds_sync();
        if constexpr (IX) {
            const int keep = r;
            r = rr;
            build_index();
            r = keep;
        }
    }
    // writes the current scheme to HBM; returns its non-zero coefficients
    __device__ int store_scheme(uint64_t *dst) const
    {
        int c = 0;
        for (int k = gl; k < r; k += G)
#pragma unroll
            for (int X = 0; X < 3; ++X) {
                const TV<T> v = ld(k, X);
                dst[k * 6 + 2 * X] = (uint64_t)v.d;
                dst[k * 6 + 2 * X + 1] = (uint64_t)v.s;
                c += popc64((uint64_t)v.d);
            }
        return group_sum(c);
    }
    __device__ int count_nnz() const
    {
        int c = 0;
        for (int k = gl; k < r; k += G)
#pragma unroll
            for (int X = 0; X < 3; ++X) c += popc64((uint64_t)ld(k, X).d);
        return group_sum(c);
    }
    __device__ __forceinline__ int group_sum(int c) const
    {
#pragma unroll
        for (int off = G / 2; off > 0; off >>= 1) c += __shfl_xor(c, off, G);
        return c;
    }
    // the stop rule: best rank (additions objective: best naive additions,
    // non-zero coefficients - 2r - mp, Sec. 4.5) at most the target
    __device__ __forceinline__ bool reached() const
    {
        return additions ? best_nnz - 2 * best_rank - mp <= target : best_rank <= target;
    }

    __device__ void restart_check()
    {
        if (a->plateau > 0 && t - plateau_start >= a->plateau) {
            const bool from_best = a->restart_from_best != 0;
            const uint64_t *src = (from_best ? (const uint64_t *)a->best : a->start) +
                                  (size_t)walk * a->cap * 6;
            const int rr = from_best ? best_rank : start_rank;
            load_scheme(src, rr);
            r = rr;
            if (additions) nnz = count_nnz();
            plateau_start = t;
            cnt[C_RESTARTS]++;
        }
    }

    __device__ void begin_iteration()
    {
        // this iteration's draws: lane q < G-1 -> flip attempt q, lane G-1 -> gates
        const bool gate_lane = gl == G - 1;
        pb = draw(gate_lane ? 0u : (uint32_t)gl, gate_lane ? 1u : 0u);
#pragma unroll
        for (int q = 0; q < 3; ++q) gate[q] = from_lane(pb.x[q], G - 1);
        logging = a->log != nullptr && t <= a->log_cap;
    }

    // everything of Algorithm 1 after try_flip
    __device__ void finish_iteration(bool found, int fi, int fj)
    {
        // each costly step (best copy, removal, expand, restart) has one call
        // site, so that the walks of a wavefront that take it do so together
        bool improved = false, accepted = false, grow = false;
        if (!found) {
            // Algorithm 1: no flip -> expand, continue (the additions
            // objective keeps the rank and does not expand)
            cnt[C_DEAD_ENDS]++;
            grow = !additions;
        } else {
            int tr0 = fi, tr1 = fj;
            // gates: block (t, 0, 1), drawn by the last lane of the group
            const uint32_t g0 = gate[0];
            if (additions) {
                // the rank is unchanged: best by non-zero count, no reduce or
                // expand
                improved = nnz < best_nnz;
                accepted = !improved && nnz == best_nnz && (uint64_t)g0 < a->t_eq;
            } else {
                // terms with a zero factor go, the higher index first
                const bool zi = zfi, zj = zfj;
                const int h1 = zi && zj ? (fi > fj ? fi : fj) : (zi ? fi : (zj ? fj : -1));
                const int h2 = zi && zj ? (fi > fj ? fj : fi) : -1;
                if (h1 >= 0) {
                    swap_remove(h1, tr0, tr1);
                    cnt[C_ZERO_REMOVED]++;
                }
                if (h2 >= 0) {
                    swap_remove(h2, tr0, tr1);
                    cnt[C_ZERO_REMOVED]++;
                }
                improved = r < best_rank;
                accepted = !improved && r == best_rank && (uint64_t)g0 < a->t_eq;
            }
            if (improved || accepted) {
                const int c = store_scheme(a->best + (size_t)walk * a->cap * 6);
                best_nnz = additions ? nnz : c;
                best_rank = r;
            }
            if (improved) {
                plateau_start = t;
                if (gl == 0 && n_rec < a->rec_cap) {
                    tsf_record *rc = a->rec + (size_t)walk * a->rec_cap + n_rec;
                    rc->iter = t;
                    rc->rank = additions ? nnz - 2 * r - mp : r;
                    rc->reserved = 0;
                }
                n_rec++;
                cnt[C_IMPROVEMENTS]++;
            } else if (accepted) {
                cnt[C_EQ_ACCEPTS]++;
            }
            if (!additions) {
                const uint32_t g1 = gate[1];
                const uint32_t g2 = gate[2];
                if ((uint64_t)g1 < a->t_reduce) cnt[C_MERGES] += (uint32_t)reduce(tr0, tr1);
                grow = (uint64_t)g2 < a->t_expand && r <= best_rank + 2 && r < r_cap;
            }
        }
        if (grow) expand();
        restart_check();
        write_log(found);
    }

    __device__ void write_log(bool flipped)
    {
        if (logging && gl == 0) {
            tsf_flip_log *lg = a->log + (size_t)walk * a->log_cap + (t - 1);
            lg->iter = t;
            if (!flipped) {
                lg->rank_before = -1;
                for (int q = 0; q < 12; ++q) lg->f[q] = 0;
            }
            lg->rank_after = r;
            lg->format_slot = fmt_slot;
            lg->reserved = 0;
            lg->pad = 0;
        }
    }

    // CHK: the invariants of the walk state that every step keeps, over the
    // terms of the group (lanes in parallel): the rank within [1, r_cap] and
    // the best rank at most the start rank (TSF_CHECK_RANK); every live
    // factor non-zero (TSF_CHECK_ZERO_FACTOR), signs only where digits are
    // (and none in Z2) and no entry beyond the factor's length
    // (TSF_CHECK_CODING); u and v of every live term normalised, Sec. 3.6
    // (TSF_CHECK_NORMALISED); IX: every mask equal to the relation it
    // indexes (TSF_CHECK_INDEX); PK: slots at or above the rank dead
    // (TSF_CHECK_DEAD_SLOTS).  Returns the OR of the failed checks.
    __device__ uint32_t check_state(const int (&len)[3]) const
    {
        uint32_t bad = 0;
        if (r < 1 || r > r_cap || best_rank > start_rank) bad |= TSF_CHECK_RANK;
        // terms below the rank, never beyond the capacity (the mask rows)
        const int rr = r < 0 ? 0 : (r > a->cap ? a->cap : r);
        for (int k = gl; k < rr; k += G) {
#pragma unroll
            for (int X = 0; X < 3; ++X) {
                const TV<T> v = ld(k, X);
                if (v.d == 0) bad |= TSF_CHECK_ZERO_FACTOR;
                if ((v.s & ~v.d) != 0 || (Z2 && v.s != 0)) bad |= TSF_CHECK_CODING;
                if (len[X] < (int)(8 * sizeof(T)) && (v.d >> len[X]) != 0) bad |= TSF_CHECK_CODING;
                if (!Z2 && X < 2 && (v.s & v.d & (~v.d + 1)) != 0) bad |= TSF_CHECK_NORMALISED;
                if constexpr (IX) {
                    uint64_t want = 0;
                    for (int j = 0; j < rr; ++j)
                        want |= (j != k && equiv(ld(j, X), v, X)) ? 1ull << j : 0ull;
                    if (mk[X * capm + k] != want) bad |= TSF_CHECK_INDEX;
                }
            }
        }
        if constexpr (PK) {
            for (int k = rr + gl; k < cap2; k += G)
#pragma unroll
                for (int X = 0; X < 3; ++X)
                    if (lds[idx(k, X)] != kDead) bad |= TSF_CHECK_DEAD_SLOTS;
        }
        uint32_t all = 0;
#pragma unroll
        for (int b = 0; b < 8; ++b)
            all |= gballot((bad >> b) & 1u) ? 1u << b : 0u;
        return all;
    }

    __device__ void iteration()
    {
        begin_iteration();
        int fi = -1, fj = -1;
        const bool found = try_flip(fi, fj);
        finish_iteration(found, fi, fj);
    }

    // ---------------------------------------------------------- learned
    // Phase 1 of a learned iteration: attempt q < K (one per lane) yields
    // its candidate exactly as with uniform proposals; lane q writes the
    // candidate (i | j<<8 | X<<16 | role<<18, or ~0 without one) and its
    // feature row.  The walk state is not changed.
    __device__ void propose()
    {
        const bool gate_lane = gl == G - 1;
        pb = draw(gate_lane ? 0u : (uint32_t)gl, gate_lane ? 1u : 0u);
        const int K = a->learn_k;
        uint32_t desc = ~0u;
        if (r >= 2) {
            update_scan_end();
            const int i = (int)below(pb.x[0], (uint32_t)r);
            const int X = (int)below(pb.x[1], 3u);
            PSet m0, m1;
            m0.clear();
            m1.clear();
            candidates_ap(gl < K, i, X, m0, m1);
            const int n0 = m0.count(), n = n0 + m1.count();
            if (n > 0) {
                int c = (int)below(pb.x[2], (uint32_t)n);
                const int role = c >= n0;
                if (role) c -= n0;
                const int j = (role ? m1 : m0).kth(c);  // one search, on the chosen set
                desc = (uint32_t)i | ((uint32_t)j << 8) | ((uint32_t)X << 16) |
                       ((uint32_t)role << 18);
                const int A = X == 0 ? 1 : 0, B = X == 2 ? 1 : 2;
                const int Y = role ? B : A, Z = role ? A : B;
                const TV<T> fv[6] = {ld(i, X), ld(i, Y), ld(i, Z), ld(j, X), ld(j, Y), ld(j, Z)};
                uint64_t f[12];
#pragma unroll
                for (int q = 0; q < 6; ++q) {
                    f[2 * q] = (uint64_t)fv[q].d;
                    f[2 * q + 1] = (uint64_t)fv[q].s;
                }
                write_feature_row(a->feat + ((size_t)walk * kLearnRows + gl) * 512, f, fmt_slot, r);
            }
        }
        if (gl < kLearnRows) a->cand[(size_t)walk * kLearnRows + gl] = desc;
    }

    // Phase 2: apply the best-scored candidate (ties: the lower attempt), or
    // run the uniform fallback search when no attempt had a candidate.
    __device__ void apply_learned()
    {
        begin_iteration();
        const int K = a->learn_k;
        uint32_t desc = ~0u;
        float score = -__builtin_inff();
        if (gl < K) {
            desc = a->cand[(size_t)walk * kLearnRows + gl];
            const float l = a->logit[(size_t)walk * kLearnRows + gl];
            if (desc != ~0u) score = (l == l) ? l : -__builtin_inff();
        }
        const bool valid = desc != ~0u;
        float best = score;
        for (int off = 1; off < G; off <<= 1) best = fmaxf(best, __shfl_xor(best, off, G));
        const uint64_t win_mask = gballot(valid && score == best);
        cnt[C_ATTEMPTS] += (uint32_t)K;
        int fi = -1, fj = -1;
        uint32_t d = kNoFlip;
        uint8_t choice = 255;
        if (win_mask) {
            const int win = __builtin_ctzll(win_mask);
            const uint32_t c = from_lane(desc, win);  // the candidate layout of propose()
            d = pack_flip(c & 0xFF, (c >> 8) & 0xFF, (c >> 16) & 3, (c >> 18) & 1);
            choice = (uint8_t)win;
        } else if (r >= 2) {
            update_scan_end();
            d = fallback_ap();
        }
        const bool found = d != kNoFlip;
        if (found) apply_packed(d, fi, fj);
        if (a->choice && gl == 0 && t <= a->choice_cap)
            a->choice[(size_t)walk * a->choice_cap + (t - 1)] = choice;
        finish_iteration(found, fi, fj);
    }
};

__device__ __forceinline__ int flen(int m, int n, int p, int X)
{
    return X == 0 ? m * n : X == 1 ? n * p : p * m;
}

// The walk kernel's body; CHK adds the invariant checks of
// tsf_walk_checked (after the scheme is loaded and after every iteration; a
// walk that fails one stops with done = -4 and the error word
// (iteration << 8) | failed checks in the header's `reserved`).
// Issue priority of a wavefront by its progress through the call: the fewer
// of the call's iterations it has done, the higher its priority (s_setprio;
// between equal priorities a SIMD issues the oldest wavefront first).  The
// wavefronts that share a SIMD would otherwise finish at staggered times, and
// the last of them would run on a SIMD that is partly empty; with it they end
// close together, and the next wavefronts take over whole SIMDs.  Band edges
// at 3/8, 5/8 and 13/16 of the call.  Only the order in which the SIMD issues
// instructions changes, never a result.
__device__ __forceinline__ void progress_priority(int64_t it, int64_t n)
{
    const uint64_t q = (uint64_t)it * 64u / (uint64_t)n;  // progress in 64ths
    if (q < 24) __builtin_amdgcn_s_setprio(3);
    else if (q < 40) __builtin_amdgcn_s_setprio(2);
    else if (q < 52) __builtin_amdgcn_s_setprio(1);
    else __builtin_amdgcn_s_setprio(0);
}

template <int G, int S, typename T, bool Z2, bool AP, bool IX, bool PK, bool CHK>
__device__ __forceinline__ void walk_body(const KArgs &a)
{
    extern __shared__ uint64_t smem_u64[];
    T *smem = reinterpret_cast<T *>(smem_u64);
    constexpr int W = 64 / G;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int grp = lane / G;
    const int wpb = blockDim.x >> 6;
    const int64_t walk = ((int64_t)blockIdx.x * wpb + wave) * W + grp;
    if (walk >= a.n_walks) return;  // the whole group leaves together

    using Wk = Walker<G, S, T, Z2, AP, IX, PK, CHK>;
    Wk wk;
    wk.gl = lane % G;
    wk.gshift = grp * G;
    wk.cap2 = a.cap2;
    wk.capm = a.capm;
    // the terms of every walk of the workgroup (6*cap2 words each), then for
    // IX the masks of every walk (3*capm u64 each); the masks are not padded
    // like the term rows, which keeps a wavefront's LDS small enough for one
    // more wavefront per CU at (3,3,3)
    const int slot = wave * W + grp;
    wk.lds = smem + (size_t)slot * a.cap2 * 3 * Wk::kFW;
    wk.mk = reinterpret_cast<uint64_t *>(smem + (size_t)wpb * W * a.cap2 * 3 * Wk::kFW) +
            (size_t)slot * a.capm * 3;
    wk.a = &a;
    wk.walk = walk;
    tsf_walk_header *h = a.hdr + walk;
    const int m = h->m, n = h->n, p = h->p;
    int done = h->done;
    // a header that does not fit this kernel is never advanced
    const int lmax = max(flen(m, n, p, 0), max(flen(m, n, p, 1), flen(m, n, p, 2)));
    const bool sane = m >= 1 && n >= 1 && p >= 1 && lmax <= a.max_len &&
                      lmax <= (PK ? 16 : (int)(8 * sizeof(T))) && h->mode == (Z2 ? 1 : 0) &&
                      h->r_cap <= a.cap && h->rank >= 0 && h->rank <= h->r_cap &&
                      h->best_rank >= 0 && h->best_rank <= a.cap && h->start_rank >= 0 &&
                      h->start_rank <= a.cap && (!AP || a.cap <= 64 * S) && (!IX || a.cap <= 64);
    if (!sane || done != 0) {
        if (!sane && wk.gl == 0 && done == 0) h->done = -1;
        return;
    }
    // a walk resumed with other parameters than it was run with is not
    // advanced (tsf_walk_check reports it)
    if (h->params_hash != 0 && h->params_hash != a.params_hash) {
        if (wk.gl == 0) h->done = -3;
        return;
    }
    wk.seed = a.base_seed + (uint64_t)(a.first_walk_id + walk);
    wk.r = h->rank;
    wk.r_cap = h->r_cap;
    wk.best_rank = h->best_rank;
    wk.best_nnz = h->best_nnz;
    wk.mp = m * p;
    wk.additions = a.objective == TSF_OBJ_ADDITIONS;
    wk.nnz = 0;
    wk.start_rank = h->start_rank;
    wk.target = h->target_rank;
    wk.n_rec = h->n_rec;
    wk.t = h->t;
    const int64_t t_first = wk.t;
    wk.plateau_start = h->plateau_start;
#pragma unroll
    for (int c = 0; c < C_NUM; ++c) wk.cnt[c] = 0;
    wk.logging = false;
    wk.fmt_slot = format_slot(m, n, p);
    wk.load_scheme(a.cur + (size_t)walk * a.cap * 6, wk.r);
    if (wk.additions) wk.nnz = wk.count_nnz();
    uint64_t err = 0;
    const int len[3] = {flen(m, n, p, 0), flen(m, n, p, 1), flen(m, n, p, 2)};
    if constexpr (CHK) {
        const uint32_t bad = wk.check_state(len);
        if (bad) {
            // the loaded state is left as it is
            if (wk.gl == 0) {
                h->done = -4;
                h->reserved = ((uint64_t)wk.t << 8) | bad;
            }
            return;
        }
    }

    if constexpr (AP && !IX) {
        if (a.phase == 1) {
            // learned proposal, phase 1: candidates and feature rows only
            if (wk.reached() || wk.t >= a.max_iters) return;
            wk.t += 1;
            wk.propose();
            return;
        }
    }
    if (AP && !IX && a.phase == 2) {
        if (wk.reached()) done = 1;
        if (!done && wk.t < a.max_iters) {
            wk.t += 1;
            if constexpr (AP && !IX) wk.apply_learned();
        }
    } else {
        for (int64_t it = 0; it < a.n_iters; ++it) {
            if (wk.reached()) done = 1;
            if (done || wk.t >= a.max_iters) break;
            if ((it & 63) == 0) progress_priority(it, a.n_iters);
            wk.t += 1;
            wk.iteration();
            if constexpr (CHK) {
                const uint32_t bad = wk.check_state(len);
                if (bad) {
                    done = -4;
                    err = ((uint64_t)wk.t << 8) | bad;
                    break;
                }
            }
        }
    }
    if ((!CHK || done != -4) && wk.reached()) done = 1;

    wk.store_scheme(a.cur + (size_t)walk * a.cap * 6);
    if (wk.gl == 0) {
        h->rank = wk.r;
        h->best_rank = wk.best_rank;
        h->best_nnz = wk.best_nnz;
        h->done = done;
        h->n_rec = wk.n_rec;
        h->t = wk.t;
        h->plateau_start = wk.plateau_start;
        h->params_hash = a.params_hash;
        if (CHK && done == -4) h->reserved = err;
        // every iteration of this call is a flip or a dead end
        wk.cnt[C_ITERS] = (uint32_t)(wk.t - t_first);
        wk.cnt[C_FLIPS] = wk.cnt[C_ITERS] - wk.cnt[C_DEAD_ENDS];
        for (int c = 0; c < C_NUM; ++c) h->counters[c] += wk.cnt[c];
    }
}

// Register budgets: the packed indexed kernels (8 or more lanes per walk)
// are held to 128 VGPRs, four wavefronts per SIMD, which their LDS also
// allows at (3,3,3) (10,176 bytes per 8-walk wavefront, sixteen per CU); the
// other indexed kernels with 32-bit masks to 168 VGPRs (three per SIMD, as
// many as their LDS allows); the term-parallel kernels with 64 lanes and four
// slots per walk (capacities 193-256, e.g. (4,5,12)) also to 168 VGPRs, three
// per SIMD, which their LDS allows; the rest are not constrained.
template <int G, int S, typename T, bool Z2, bool AP, bool IX, bool PK = false>
__global__ void __launch_bounds__(256) __attribute__((
    amdgpu_waves_per_eu(PK && G >= 8 ? 4 : (IX && G >= 8 && sizeof(T) == 4) ? 3 :
                        (!AP && G == 64 && S == 4) ? 3 : 1))) walk_kernel(KArgs a)
{
    walk_body<G, S, T, Z2, AP, IX, PK, false>(a);
}

// the same walk with the invariant checks (tsf_walk_checked)
template <int G, int S, typename T, bool Z2, bool AP, bool IX, bool PK = false>
__global__ void __launch_bounds__(256) walk_kernel_checked(KArgs a)
{
    walk_body<G, S, T, Z2, AP, IX, PK, true>(a);
}

using KernelFn = void (*)(KArgs);

}  // namespace tsfk
