// walk.hip -- host side of the batched walks: walk-state initialisation,
// batch Brent verification on the GPU, and the launch of the walk kernels
// (walk_kernel.h, instantiated in walk_inst.hip).
#include "walk_kernel.h"
#include "tsf_internal.h"
#include "tsf_meta.h"

#include <cstring>
#include <mutex>
#include <vector>

namespace tsfk {
KernelFn pick_kernel_w0_z0(int g, int s, int strategy, bool chk);
KernelFn pick_kernel_w0_z1(int g, int s, int strategy, bool chk);
KernelFn pick_kernel_w1_z0(int g, int s, int strategy, bool chk);
KernelFn pick_kernel_w1_z1(int g, int s, int strategy, bool chk);
}  // namespace tsfk

namespace {
using namespace tsfk;

// One wavefront per walk: validate the start scheme, then cur := best :=
// start and clear the walk's state.
__global__ void __launch_bounds__(64) init_kernel(tsf_walk_header *hdr, uint64_t *cur,
                                                  uint64_t *best, const uint64_t *start,
                                                  int32_t n_walks, int32_t cap)
{
    const int64_t walk = blockIdx.x;
    const int lane = threadIdx.x;
    if (walk >= n_walks) return;
    tsf_walk_header *h = hdr + walk;
    const int m = h->m, n = h->n, p = h->p, r0 = h->start_rank;
    const bool z2 = h->mode == 1;
    bool ok = m >= 1 && n >= 1 && p >= 1 && (h->mode == 0 || h->mode == 1) && r0 >= 0 &&
              r0 <= h->r_cap && h->r_cap <= cap;
    const int len[3] = {m * n, n * p, p * m};
    ok = ok && len[0] <= 64 && len[1] <= 64 && len[2] <= 64;
    const size_t base = (size_t)walk * cap * 6;
    bool bad = false;
    if (ok) {
        for (int k = lane; k < r0; k += 64) {
            for (int X = 0; X < 3; ++X) {
                const uint64_t d = start[base + k * 6 + 2 * X], s = start[base + k * 6 + 2 * X + 1];
                const uint64_t lim = len[X] == 64 ? ~0ull : ((1ull << len[X]) - 1);
                if (d == 0 || (s & ~d) || (d & ~lim) || (z2 && s)) bad = true;
                if (!z2 && X < 2 && (s & (d & (~d + 1)))) bad = true;  // not normalised
            }
            for (int x = 0; x < 6; ++x) {
                cur[base + k * 6 + x] = start[base + k * 6 + x];
                best[base + k * 6 + x] = start[base + k * 6 + x];
            }
        }
    }
    const bool any_bad = __ballot(bad) != 0;
    // non-zero coefficients of the start scheme
    int nnz = 0;
    if (ok)
        for (int k = lane; k < r0; k += 64)
            for (int X = 0; X < 3; ++X) nnz += __builtin_popcountll(start[base + k * 6 + 2 * X]);
    for (int off = 32; off > 0; off >>= 1) nnz += __shfl_xor(nnz, off);
    if (lane == 0) {
        h->done = (!ok || any_bad) ? -2 : 0;
        h->rank = r0;
        h->best_rank = r0;
        h->n_rec = 0;
        h->best_nnz = nnz;
        h->t = 0;
        h->plateau_start = 0;
        for (int c = 0; c < 12; ++c) h->counters[c] = 0;
        h->params_hash = 0;
        h->reserved = 0;
    }
}

// Brent verification (Eq. 1, C^T form of Sec. 3.1) of one scheme per
// workgroup: the tensor sum_l u_l (x) v_l (x) w_l is built one u-entry slice
// at a time in LDS (int32 atomics over the non-zero products), then compared
// with the matrix multiplication tensor.  A mask bit that encodes no
// coefficient (a digit at or beyond the factor's length, a sign without its
// digit, any sign of a Z2 scheme) counts as one violation of its own and
// takes no part in the tensor.
__global__ void __launch_bounds__(256) verify_kernel(const tsf_walk_header *hdr,
                                                     const uint64_t *schemes, int32_t cap,
                                                     int32_t n_walks, int32_t which,
                                                     int64_t *n_violated)
{
    __shared__ int32_t slice[64 * 64];
    __shared__ int32_t bad_sh;
    const int64_t q = blockIdx.x;
    if (q >= n_walks) return;
    const tsf_walk_header *h = hdr + q;
    const int m = h->m, n = h->n, p = h->p;
    const int rank = which == 0 ? h->rank : which == 1 ? h->best_rank : h->start_rank;
    const bool z2 = h->mode == 1;
    const int Lu = m * n, Lv = n * p, Lw = p * m;
    if (m < 1 || n < 1 || p < 1 || Lu > 64 || Lv > 64 || Lw > 64 || rank < 0 || rank > cap) {
        if (threadIdx.x == 0) n_violated[q] = -1;
        return;
    }
    const uint64_t *sc = schemes + (size_t)q * cap * 6;
    if (threadIdx.x == 0) bad_sh = 0;
    int32_t bad = 0;
    const uint64_t lim[3] = {Lu == 64 ? ~0ull : (1ull << Lu) - 1, Lv == 64 ? ~0ull : (1ull << Lv) - 1,
                             Lw == 64 ? ~0ull : (1ull << Lw) - 1};
    for (int l = threadIdx.x; l < rank; l += blockDim.x)
        for (int X = 0; X < 3; ++X) {
            const uint64_t d = sc[l * 6 + 2 * X], sg = sc[l * 6 + 2 * X + 1];
            bad += __builtin_popcountll(d & ~lim[X]) +
                   __builtin_popcountll(z2 ? sg : (sg & ~(d & lim[X])));
        }
    for (int av = 0; av < Lu; ++av) {
        for (int e = threadIdx.x; e < Lv * Lw; e += blockDim.x) slice[e] = 0;
        __syncthreads();
        const int a1 = av / n, a2 = av % n;
        for (int l = threadIdx.x; l < rank; l += blockDim.x) {
            const uint64_t ud = sc[l * 6 + 0], us = sc[l * 6 + 1];
            if (!((ud >> av) & 1)) continue;
            const int su = ((us >> av) & 1) ? -1 : 1;
            for (uint64_t dv = sc[l * 6 + 2] & lim[1]; dv; dv &= dv - 1) {
                const int b = __builtin_ctzll(dv);
                const int sv = ((sc[l * 6 + 3] >> b) & 1) ? -su : su;
                for (uint64_t dw = sc[l * 6 + 4] & lim[2]; dw; dw &= dw - 1) {
                    const int c = __builtin_ctzll(dw);
                    atomicAdd(&slice[b * Lw + c], ((sc[l * 6 + 5] >> c) & 1) ? -sv : sv);
                }
            }
        }
        __syncthreads();
        for (int e = threadIdx.x; e < Lv * Lw; e += blockDim.x) {
            const int b = e / Lw, c = e % Lw;
            const int b1 = b / p, b2 = b % p, c1 = c / m, c2 = c % m;
            const int want = (a2 == b1 && b2 == c1 && c2 == a1) ? 1 : 0;
            int got = slice[e];
            if (z2) got &= 1;
            bad += got != want;
        }
        __syncthreads();
    }
    atomicAdd(&bad_sh, bad);
    __syncthreads();
    if (threadIdx.x == 0) n_violated[q] = bad_sh;
}

// (r, c) of a row-major rows x cols factor -> the new position, or -1 when
// its row or column is dropped (drop_r / drop_c, -1 for none); cols2 is the
// new row length
__device__ __forceinline__ uint64_t remap_mask(uint64_t mask, int cols, int cols2, int drop_r,
                                               int drop_c)
{
    uint64_t o = 0;
    for (; mask; mask &= mask - 1) {
        const int e = __builtin_ctzll(mask);
        const int rr = e / cols, cc = e % cols;
        if (rr == drop_r || cc == drop_c) continue;
        const int r2 = rr - (drop_r >= 0 && rr > drop_r), c2 = cc - (drop_c >= 0 && cc > drop_c);
        o |= 1ull << (r2 * cols2 + c2);
    }
    return o;
}

// One wavefront per walk: project / extend / copy a scheme into a new start.
__global__ void __launch_bounds__(64) meta_kernel(tsf_walk_batch in, int32_t which,
                                                  const int32_t *op, const int32_t *axis,
                                                  const int32_t *index, int32_t r_cap_extra,
                                                  tsf_walk_batch out)
{
    const int64_t walk = blockIdx.x;
    const int lane = threadIdx.x;
    if (walk >= in.n_walks) return;
    const tsf_walk_header *h = in.hdr + walk;
    tsf_walk_header *ho = out.hdr + walk;
    const int m = h->m, n = h->n, p = h->p, mode = h->mode;
    const int rank = which ? h->best_rank : h->rank;
    const int o = op[walk], ax = axis[walk], ix = index[walk];
    const int dims[3] = {m, n, p};
    bool ok = m >= 1 && n >= 1 && p >= 1 && rank >= 0 && rank <= in.capacity && o >= 0 &&
              o <= 2 && (o == 0 || (ax >= 0 && ax <= 2));
    if (ok && o == 1) ok = dims[ax] >= 2 && ix >= 0 && ix < dims[ax];
    const int m2 = m + (ok && ax == 0 ? (o == 1 ? -1 : o == 2 ? 1 : 0) : 0);
    const int n2 = n + (ok && ax == 1 ? (o == 1 ? -1 : o == 2 ? 1 : 0) : 0);
    const int p2 = p + (ok && ax == 2 ? (o == 1 ? -1 : o == 2 ? 1 : 0) : 0);
    ok = ok && m2 * n2 <= 64 && n2 * p2 <= 64 && p2 * m2 <= 64;
    const int extra = (ok && o == 2) ? (ax == 0 ? n * p : ax == 1 ? m * p : m * n) : 0;
    // per factor: columns before/after and the dropped row/column (axis order:
    // U rows i (m) cols j (n); V rows j (n) cols k (p); W rows k (p) cols i (m))
    const int colsU = n, colsV = p, colsW = m;
    const int colsU2 = n2, colsV2 = p2, colsW2 = m2;
    const int dr_u = (o == 1 && ax == 0) ? ix : -1, dc_u = (o == 1 && ax == 1) ? ix : -1;
    const int dr_v = (o == 1 && ax == 1) ? ix : -1, dc_v = (o == 1 && ax == 2) ? ix : -1;
    const int dr_w = (o == 1 && ax == 2) ? ix : -1, dc_w = (o == 1 && ax == 0) ? ix : -1;
    const uint64_t *src = (which ? in.best : in.cur) + (size_t)walk * in.capacity * 6;
    uint64_t *dst = const_cast<uint64_t *>(out.start) + (size_t)walk * out.capacity * 6;
    int count = 0;
    if (ok) {
        for (int base = 0; base < rank; base += 64) {
            const int k = base + lane;
            uint64_t f[6] = {0, 0, 0, 0, 0, 0};
            bool keep = false;
            if (k < rank) {
                f[0] = remap_mask(src[k * 6 + 0], colsU, colsU2, dr_u, dc_u);
                f[1] = remap_mask(src[k * 6 + 1], colsU, colsU2, dr_u, dc_u);
                f[2] = remap_mask(src[k * 6 + 2], colsV, colsV2, dr_v, dc_v);
                f[3] = remap_mask(src[k * 6 + 3], colsV, colsV2, dr_v, dc_v);
                f[4] = remap_mask(src[k * 6 + 4], colsW, colsW2, dr_w, dc_w);
                f[5] = remap_mask(src[k * 6 + 5], colsW, colsW2, dr_w, dc_w);
                keep = f[0] != 0 && f[2] != 0 && f[4] != 0;
                if (mode == 0) {
                    // Sec. 3.6: first non-zero of u, then of v, positive; w absorbs
                    for (int X = 0; X < 2; ++X) {
                        const uint64_t low = f[2 * X] & (~f[2 * X] + 1);
                        if (f[2 * X + 1] & low) {
                            f[2 * X + 1] ^= f[2 * X];
                            f[5] ^= f[4];
                        }
                    }
                }
            }
            const uint64_t mk = __ballot(keep);
            const int pos = count + __builtin_amdgcn_mbcnt_hi((uint32_t)(mk >> 32),
                                                            __builtin_amdgcn_mbcnt_lo((uint32_t)mk, 0));
            if (keep && pos < out.capacity)
                for (int x = 0; x < 6; ++x) dst[pos * 6 + x] = f[x];
            count += __builtin_popcountll(mk);
        }
        // extend: the naive scheme of the new index
        for (int q = lane; q < extra; q += 64) {
            int i, j, k;
            if (ax == 2) { i = q / n; j = q % n; k = p; }
            else if (ax == 0) { i = m; j = q / p; k = q % p; }
            else { i = q / p; j = n; k = q % p; }
            const int pos = count + q;
            if (pos < out.capacity) {
                dst[pos * 6 + 0] = 1ull << (i * n2 + j);
                dst[pos * 6 + 1] = 0;
                dst[pos * 6 + 2] = 1ull << (j * p2 + k);
                dst[pos * 6 + 3] = 0;
                dst[pos * 6 + 4] = 1ull << (k * m2 + i);
                dst[pos * 6 + 5] = 0;
            }
        }
        count += extra;
    }
    if (lane == 0) {
        const bool fits = ok && count <= out.capacity;
        ho->m = fits ? m2 : m;
        ho->n = fits ? n2 : n;
        ho->p = fits ? p2 : p;
        ho->mode = mode;
        ho->target_rank = h->target_rank;
        ho->start_rank = fits ? count : -1;
        const int rc = count + r_cap_extra;
        ho->r_cap = fits ? (rc < out.capacity ? rc : out.capacity) : 0;
    }
}

// feature rows of the proposal network from log records, one row per thread
__global__ void __launch_bounds__(256) features_kernel(const tsf_flip_log *log, int64_t n,
                                                       uint16_t *X)
{
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= n) return;
    const tsf_flip_log &lg = log[q];
    uint64_t f[12];
    for (int e = 0; e < 12; ++e) f[e] = lg.f[e];
    const int slot = lg.format_slot < 0 || lg.format_slot > 15 ? 15 : lg.format_slot;
    write_feature_row(X + q * 512, f, slot, lg.rank_before);
}

// Isotropy invariants (Sec. 3.7) of one scheme per wavefront: lane l takes
// terms l, l+64, ...; the rank of each factor comes from elimination in the
// lane's own 64-word slice of LDS (factor_rank, shared with the host).
__global__ void __launch_bounds__(64) invariants_kernel(const tsf_walk_header *hdr,
                                                       const uint64_t *schemes, int32_t cap,
                                                       int32_t n_walks, int32_t which,
                                                       uint8_t *term_ranks, int32_t *rank_sums)
{
    __shared__ int32_t scratch[64 * 64];
    const int64_t walk = blockIdx.x;
    const int lane = threadIdx.x;
    if (walk >= n_walks) return;
    const tsf_walk_header *h = hdr + walk;
    const int m = h->m, n = h->n, p = h->p;
    const int rank = which == 0 ? h->rank : which == 1 ? h->best_rank : h->start_rank;
    const bool ok = m >= 1 && n >= 1 && p >= 1 && m * n <= 64 && n * p <= 64 && p * m <= 64 &&
                    (h->mode == 0 || h->mode == 1) && rank >= 0 && rank <= cap;
    if (!ok) {
        if (lane < 3) rank_sums[walk * 3 + lane] = -1;
        return;
    }
    const bool z2 = h->mode == 1;
    int32_t *M = scratch + lane * 64;
    int s0 = 0, s1 = 0, s2 = 0;
    const uint64_t *sc = schemes + (size_t)walk * cap * 6;
    uint8_t *out = term_ranks + (size_t)walk * cap * 3;
    for (int k = lane; k < rank; k += 64) {
        const int a = factor_rank(sc[k * 6 + 0], sc[k * 6 + 1], m, n, z2, M);
        const int b = factor_rank(sc[k * 6 + 2], sc[k * 6 + 3], n, p, z2, M);
        const int c = factor_rank(sc[k * 6 + 4], sc[k * 6 + 5], p, m, z2, M);
        out[k * 3 + 0] = (uint8_t)a;
        out[k * 3 + 1] = (uint8_t)b;
        out[k * 3 + 2] = (uint8_t)c;
        s0 += a;
        s1 += b;
        s2 += c;
    }
    for (int off = 32; off > 0; off >>= 1) {
        s0 += __shfl_xor(s0, off);
        s1 += __shfl_xor(s1, off);
        s2 += __shfl_xor(s2, off);
    }
    if (lane == 0) {
        rank_sums[walk * 3 + 0] = s0;
        rank_sums[walk * 3 + 1] = s1;
        rank_sums[walk * 3 + 2] = s2;
    }
}

// ---------------------------------------------------------------------------
// Population synchronisation and the Resize kernel (Sec. 3.4.1, Algorithm 2)
// ---------------------------------------------------------------------------
__global__ void clear_table_kernel(unsigned long long *keys, unsigned long long *vals, int slots,
                                   int32_t *overflow)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < slots) {
        keys[q] = 0;
        vals[q] = ~0ull;
    }
    if (q == 0) *overflow = 0;
}

// One thread per walk: insert the walk's format into an open-addressing
// table (key = 1 | m << 8 | n << 16 | p << 24) and keep, per format, the
// smallest (best rank << 32 | walk id).
__global__ void best_insert_kernel(const tsf_walk_header *hdr, int32_t n_walks,
                                   unsigned long long *keys, unsigned long long *vals, int slots,
                                   int32_t *overflow)
{
    const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= n_walks) return;
    const tsf_walk_header *h = hdr + w;
    if (h->done < 0 || h->m < 1 || h->m > 64 || h->n < 1 || h->n > 64 || h->p < 1 || h->p > 64)
        return;
    const unsigned long long key = 1ull | ((unsigned long long)h->m << 8) |
                                   ((unsigned long long)h->n << 16) | ((unsigned long long)h->p << 24);
    const unsigned long long val = ((unsigned long long)(uint32_t)h->best_rank << 32) | (uint64_t)w;
    int q = (int)((key * 0x9E3779B97F4A7C15ull) >> 40) % slots;
    for (int probe = 0; probe < slots; ++probe) {
        const unsigned long long prev = atomicCAS(&keys[q], 0ull, key);
        if (prev == 0 || prev == key) {
            atomicMin(&vals[q], val);
            return;
        }
        q = q + 1 == slots ? 0 : q + 1;
    }
    atomicAdd(overflow, 1);
}

// One workgroup: the occupied slots in ascending (m, n, p) order -> table
// (each slot's position = the number of smaller formats, counted over a copy
// of the format keys in LDS; empty slots hold the largest key).
constexpr int kMaxSlots = 4096;
__global__ void __launch_bounds__(256) best_compact_kernel(const unsigned long long *keys,
                                                           const unsigned long long *vals,
                                                           int slots, tsf_best_entry *table,
                                                           int32_t *n_entries,
                                                           const int32_t *overflow,
                                                           int32_t *dropped)
{
    __shared__ uint32_t ord[kMaxSlots];
    __shared__ int32_t used;
    if (threadIdx.x == 0) used = 0;
    __syncthreads();
    int mine = 0;
    for (int q = threadIdx.x; q < slots; q += blockDim.x) {
        const unsigned long long k = keys[q];
        ord[q] = k ? (uint32_t)(((k >> 8) & 0xFF) << 16 | ((k >> 16) & 0xFF) << 8 |
                                ((k >> 24) & 0xFF))
                   : 0xFFFFFFFFu;
        mine += k != 0;
    }
    atomicAdd(&used, mine);
    __syncthreads();
    for (int q = threadIdx.x; q < slots; q += blockDim.x) {
        const uint32_t o = ord[q];
        if (o == 0xFFFFFFFFu) continue;
        int pos = 0;
        for (int x = 0; x < slots; ++x) pos += ord[x] < o;
        const unsigned long long k = keys[q];
        tsf_best_entry e;
        e.m = (int32_t)((k >> 8) & 0xFF);
        e.n = (int32_t)((k >> 16) & 0xFF);
        e.p = (int32_t)((k >> 24) & 0xFF);
        e.rank = (int32_t)(vals[q] >> 32);
        e.walk = (int64_t)(vals[q] & 0xFFFFFFFFull);
        table[pos] = e;
    }
    if (threadIdx.x == 0) {
        *n_entries = used;
        if (dropped) *dropped = *overflow;
    }
}

// Algorithm 2 on every walk (one wavefront per walk): the walk's current or
// best scheme, after the operators drawn from Philox blocks (round, 0, 3)
// and (round, 1, 3) of its seed, becomes its start scheme in `out`.
// Partners are the best schemes of the table, read from in.best.  Lanes
// handle output terms.
__global__ void __launch_bounds__(64) resize_kernel(tsf_walk_batch in, int32_t which,
                                                    const tsf_best_entry *table,
                                                    const int32_t *n_entries, uint64_t base_seed,
                                                    int64_t first_walk_id, int64_t round,
                                                    uint64_t t_resize, int32_t r_cap_extra,
                                                    tsf_walk_batch out, int32_t *applied_out)
{
    const int64_t walk = blockIdx.x;
    const int lane = threadIdx.x;
    if (walk >= in.n_walks) return;
    const tsf_walk_header *h = in.hdr + walk;
    tsf_walk_header *ho = out.hdr + walk;
    const int m0 = h->m, n0 = h->n, p0 = h->p;
    const int r0 = which ? h->best_rank : h->rank;
    const int nb = *n_entries;
    const bool sane = h->done >= 0 && m0 >= 1 && n0 >= 1 && p0 >= 1 && m0 * n0 <= 64 &&
                      n0 * p0 <= 64 && p0 * m0 <= 64 && r0 >= 1 && r0 <= in.capacity &&
                      r0 <= out.capacity;
    const uint64_t seed = base_seed + (uint64_t)(first_walk_id + walk);
    const Philox4 b0 = walk_block(seed, round, 0, 3), b1 = walk_block(seed, round, 1, 3);
    const uint64_t *src = (which ? in.best : in.cur) + (size_t)walk * in.capacity * 6;
    uint64_t *dst = const_cast<uint64_t *>(out.start) + (size_t)walk * out.capacity * 6;
    const bool swp = sane && b0.x[0] < 0x80000000u;
    // format after the optional swap
    const int m = m0, n = swp ? p0 : n0, p = swp ? n0 : p0;
    auto term = [&](int k, uint64_t (&f)[6]) {
        uint64_t g[6];
        for (int x = 0; x < 6; ++x) g[x] = src[k * 6 + x];
        if (swp)
            term_swap(g, m0, n0, p0, f);
        else
            for (int x = 0; x < 6; ++x) f[x] = g[x];
    };
    int applied = swp ? 1 : 0;
    int op = 0;  // 0 keep, 2 merge, 4 project, 8 product, 16 double, 32 extend
    int axis = 0, pidx = 0, M = m, N = n, P = p, R = r0;
    int64_t partner = -1;
    int pm = 0, pn = 0, pp = 0, pr = 0;
    if (sane && nb > 0) {
        const tsf_best_entry e = table[below(b0.x[1], (uint32_t)nb)];
        const int order[3] = {2, 0, 1};
        for (int q = 0; q < 3 && op == 0; ++q) {
            const int ax = order[q];
            const bool compat = ax == 2 ? (e.m == m && e.n == n) : ax == 0 ? (e.n == n && e.p == p)
                                                                            : (e.m == m && e.p == p);
            const int M2 = ax == 0 ? m + e.m : m, N2 = ax == 1 ? n + e.n : n,
                      P2 = ax == 2 ? p + e.p : p;
            if (compat && M2 * N2 <= 64 && N2 * P2 <= 64 && P2 * M2 <= 64 &&
                r0 + e.rank <= out.capacity) {
                op = 2;
                axis = ax;
                M = M2; N = N2; P = P2; R = r0 + e.rank;
                partner = e.walk;
                pm = e.m; pn = e.n; pp = e.p; pr = e.rank;
            }
        }
    }
    if (sane && op == 0 && (uint64_t)b0.x[2] < t_resize) {
        axis = (int)below(b1.x[1], 3u);
        const int dim = axis == 0 ? m : axis == 1 ? n : p;
        const uint32_t q = b0.x[3];
        if (q < 214748365u) {  // round(0.05 * 2^32): project
            if (dim >= 2) {
                op = 4;
                pidx = (int)below(b1.x[2], (uint32_t)dim);
                M = m - (axis == 0); N = n - (axis == 1); P = p - (axis == 2);
            }
        } else if (q < 2362232013u) {  // round(0.55 * 2^32): product
            if (nb > 0) {
                const tsf_best_entry e = table[below(b1.x[0], (uint32_t)nb)];
                const int M2 = m * e.m, N2 = n * e.n, P2 = p * e.p;
                if (M2 * N2 <= 64 && N2 * P2 <= 64 && P2 * M2 <= 64 &&
                    (int64_t)r0 * e.rank <= out.capacity) {
                    op = 8;
                    M = M2; N = N2; P = P2; R = r0 * e.rank;
                    partner = e.walk;
                    pm = e.m; pn = e.n; pp = e.p; pr = e.rank;
                }
            }
        } else if (q < 3650722202u) {  // round(0.85 * 2^32): double
            const int M2 = axis == 0 ? 2 * m : m, N2 = axis == 1 ? 2 * n : n,
                      P2 = axis == 2 ? 2 * p : p;
            if (M2 * N2 <= 64 && N2 * P2 <= 64 && P2 * M2 <= 64 && 2 * r0 <= out.capacity) {
                op = 16;
                M = M2; N = N2; P = P2; R = 2 * r0;
            }
        } else {  // extend
            const int M2 = m + (axis == 0), N2 = n + (axis == 1), P2 = p + (axis == 2);
            const int extra = axis == 0 ? n * p : axis == 1 ? m * p : m * n;
            if (M2 * N2 <= 64 && N2 * P2 <= 64 && P2 * M2 <= 64 && r0 + extra <= out.capacity) {
                op = 32;
                M = M2; N = N2; P = P2; R = r0 + extra;
            }
        }
    }
    applied |= op;
    const uint64_t *psrc = partner >= 0 ? in.best + (size_t)partner * in.capacity * 6 : nullptr;
    int count = 0;
    if (sane) {
        if (op == 0 || op == 2 || op == 16 || op == 32) {
            // the walk's own terms, embedded (offset 0)
            for (int k = lane; k < r0; k += 64) {
                uint64_t f[6], o[6];
                term(k, f);
                term_embed(f, m, n, p, M, N, P, 0, 0, 0, o);
                for (int x = 0; x < 6; ++x) dst[k * 6 + x] = o[x];
            }
            count = r0;
        }
        if (op == 2) {
            const int oi = axis == 0 ? m : 0, oj = axis == 1 ? n : 0, ok = axis == 2 ? p : 0;
            for (int k = lane; k < pr; k += 64) {
                uint64_t f[6], o[6];
                for (int x = 0; x < 6; ++x) f[x] = psrc[k * 6 + x];
                term_embed(f, pm, pn, pp, M, N, P, oi, oj, ok, o);
                for (int x = 0; x < 6; ++x) dst[(r0 + k) * 6 + x] = o[x];
            }
            count = R;
        } else if (op == 16) {
            const int oi = axis == 0 ? m : 0, oj = axis == 1 ? n : 0, ok = axis == 2 ? p : 0;
            for (int k = lane; k < r0; k += 64) {
                uint64_t f[6], o[6];
                term(k, f);
                term_embed(f, m, n, p, M, N, P, oi, oj, ok, o);
                for (int x = 0; x < 6; ++x) dst[(r0 + k) * 6 + x] = o[x];
            }
            count = R;
        } else if (op == 32) {
            const int extra = R - r0;
            for (int q = lane; q < extra; q += 64) {
                int i, j, k;
                if (axis == 2) { i = q / n; j = q % n; k = p; }
                else if (axis == 0) { i = m; j = q / p; k = q % p; }
                else { i = q / p; j = n; k = q % p; }
                uint64_t *d = dst + (size_t)(r0 + q) * 6;
                d[0] = 1ull << (i * N + j);
                d[1] = 0;
                d[2] = 1ull << (j * P + k);
                d[3] = 0;
                d[4] = 1ull << (k * M + i);
                d[5] = 0;
            }
            count = R;
        } else if (op == 8) {
            for (int q = lane; q < R; q += 64) {
                const int l1 = q / pr, l2 = q % pr;
                uint64_t f[6], g[6], o[6];
                term(l1, f);
                for (int x = 0; x < 6; ++x) g[x] = psrc[l2 * 6 + x];
                term_kron(f, m, n, p, g, pm, pn, pp, o);
                for (int x = 0; x < 6; ++x) dst[q * 6 + x] = o[x];
            }
            count = R;
        } else if (op == 4) {
            // project: drop index pidx of `axis`, keep the non-zero terms in order
            const int cu = n, cv = p, cw = m;
            const int dr_u = axis == 0 ? pidx : -1, dc_u = axis == 1 ? pidx : -1;
            const int dr_v = axis == 1 ? pidx : -1, dc_v = axis == 2 ? pidx : -1;
            const int dr_w = axis == 2 ? pidx : -1, dc_w = axis == 0 ? pidx : -1;
            for (int base = 0; base < r0; base += 64) {
                const int k = base + lane;
                uint64_t f[6], o[6] = {0, 0, 0, 0, 0, 0};
                bool keep = false;
                if (k < r0) {
                    term(k, f);
                    o[0] = remap_mask(f[0], cu, N, dr_u, dc_u);
                    o[1] = remap_mask(f[1], cu, N, dr_u, dc_u);
                    o[2] = remap_mask(f[2], cv, P, dr_v, dc_v);
                    o[3] = remap_mask(f[3], cv, P, dr_v, dc_v);
                    o[4] = remap_mask(f[4], cw, M, dr_w, dc_w);
                    o[5] = remap_mask(f[5], cw, M, dr_w, dc_w);
                    keep = o[0] != 0 && o[2] != 0 && o[4] != 0;
                    normalise_packed(o);
                }
                const uint64_t mk = __ballot(keep);
                const int pos = count + __builtin_amdgcn_mbcnt_hi(
                                            (uint32_t)(mk >> 32),
                                            __builtin_amdgcn_mbcnt_lo((uint32_t)mk, 0));
                if (keep)
                    for (int x = 0; x < 6; ++x) dst[pos * 6 + x] = o[x];
                count += __builtin_popcountll(mk);
            }
            R = count;
        }
    }
    if (lane == 0) {
        ho->m = sane ? M : m0;
        ho->n = sane ? N : n0;
        ho->p = sane ? P : p0;
        ho->mode = h->mode;
        ho->target_rank = h->target_rank;
        ho->start_rank = sane ? count : -1;
        const int rc = count + r_cap_extra;
        ho->r_cap = rc < out.capacity ? rc : out.capacity;
        if (applied_out) applied_out[walk] = sane ? applied : -1;
    }
}

// ---------------------------------------------------------------------------
// host side: kernel table and launch
// ---------------------------------------------------------------------------
KernelFn pick_kernel(int g, int s, bool wide, bool z2, int strategy, bool chk)
{
    if (wide) return z2 ? pick_kernel_w1_z1(g, s, strategy, chk) : pick_kernel_w1_z0(g, s, strategy, chk);
    return z2 ? pick_kernel_w0_z1(g, s, strategy, chk) : pick_kernel_w0_z0(g, s, strategy, chk);
}

int slots_for(int cap, int g)
{
    for (int s : {1, 2, 4, 5, 6, 7, 8})
        if (s * g >= cap && (g == 64 || (s & (s - 1)) == 0)) return s;
    return -1;
}

tsf_status check_batch(const tsf_walk_batch *b)
{
    if (!b) return tsf_fail(TSF_E_ARG, "null batch");
    if (b->n_walks < 0) return tsf_fail(TSF_E_ARG, "n_walks %d < 0", b->n_walks);
    if (b->capacity < 1 || b->capacity > 512)
        return tsf_fail(TSF_E_CAPACITY, "capacity %d outside [1, 512]", b->capacity);
    if (b->rec_cap < 0) return tsf_fail(TSF_E_ARG, "rec_cap %d < 0", b->rec_cap);
    if (b->mode != TSF_TERNARY && b->mode != TSF_Z2)
        return tsf_fail(TSF_E_ARG, "batch mode %d", b->mode);
    if (b->max_len < 1 || b->max_len > 64)
        return tsf_fail(TSF_E_FORMAT, "max_len %d outside [1, 64]", b->max_len);
    if (b->n_walks > 0 && (!b->hdr || !b->cur || !b->best || !b->start ||
                           (b->rec_cap > 0 && !b->rec)))
        return tsf_fail(TSF_E_ARG, "null device buffer");
    return TSF_OK;
}

}  // namespace

// A captured sequence of learned iterations, replayed with hipGraphLaunch.
struct GraphEntry {
    unsigned char key[sizeof(KArgs) + 8 * sizeof(void *)];
    hipGraph_t graph;
    hipGraphExec_t exec;
    int64_t chunk;
    bool used;
};

// A tuned launch configuration for batches of one shape.
struct TuneEntry {
    int32_t capacity, max_len, mode, size_class;
    tsf_launch launch;
    bool used;
};

struct tsf_ctx {
    int device;
    int cu_count;
    hipStream_t capture;      // private stream used only to capture graphs
    GraphEntry graphs[8];
    int next_graph;
    TuneEntry tuned[16];
    int next_tuned;
    void *scratch;            // autotuner's copy of a batch
    size_t scratch_bytes;
};

namespace {
int size_class(int n_walks)
{
    int c = 0;
    while (n_walks > 1 && c < 30) {
        n_walks >>= 1;
        ++c;
    }
    return c;
}

const tsf_launch *tuned_launch(const tsf_ctx *ctx, const tsf_walk_batch *b)
{
    if (!ctx) return nullptr;
    const int sc = size_class(b->n_walks);
    for (const TuneEntry &e : ctx->tuned)
        if (e.used && e.capacity == b->capacity && e.max_len == b->max_len && e.mode == b->mode &&
            e.size_class == sc)
            return &e.launch;
    return nullptr;
}

bool launch_is_default(const tsf_launch *l)
{
    return !l || (l->lanes_per_walk == 0 && l->waves_per_block == 0 && l->strategy == 0);
}

// The three launches of the population synchronisation over a table of
// `slots` keys and values and an overflow counter in `work` (2*slots + 1
// words); the clear kernel writes every word the others read, so the table
// may hold anything before.
tsf_status launch_population(const tsf_walk_batch *b, tsf_best_entry *table, int32_t *n_entries,
                             uint64_t *work, int32_t slots, int32_t *dropped, hipStream_t s)
{
    unsigned long long *keys = (unsigned long long *)work, *vals = keys + slots;
    int32_t *overflow = (int32_t *)(vals + slots);
    hipLaunchKernelGGL(clear_table_kernel, dim3((slots + 255) / 256), dim3(256), 0, s, keys, vals,
                       slots, overflow);
    if (b->n_walks > 0)
        hipLaunchKernelGGL(best_insert_kernel, dim3((b->n_walks + 255) / 256), dim3(256), 0, s,
                           b->hdr, b->n_walks, keys, vals, slots, overflow);
    hipLaunchKernelGGL(best_compact_kernel, dim3(1), dim3(256), 0, s, keys, vals, slots, table,
                       n_entries, (const int32_t *)overflow, dropped);
    if (hipGetLastError() != hipSuccess) return tsf_fail(TSF_E_DEVICE, "population launch failed");
    return TSF_OK;
}

// Working memory of tsf_population_best_noalloc: the table at its largest
// size (kMaxSlots keys, kMaxSlots values, the overflow counter), one copy on
// every device the library runs on, for the life of the process.  Host code
// never passes the array's name to a kernel (on the host it only stands for
// the symbol): it uses the device address hipGetSymbolAddress returns, looked
// up once per device.
__device__ __align__(256) uint64_t scratch[2 * kMaxSlots + 1];

constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
uint64_t *scratch_ptr[kMaxDevices];

// the current device's copy of `scratch`
tsf_status population_scratch(uint64_t **out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return tsf_fail(TSF_E_DEVICE, "hipGetDevice failed");
    if (dev < 0 || dev >= kMaxDevices)
        return tsf_fail(TSF_E_DEVICE, "device %d beyond the %d the library supports", dev,
                        kMaxDevices);
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return tsf_fail(TSF_E_DEVICE, "hipGetSymbolAddress(scratch) failed: %s",
                            hipGetErrorString(e));
        scratch_ptr[dev] = (uint64_t *)p;
    }
    *out = scratch_ptr[dev];
    return TSF_OK;
}
}  // namespace

extern "C" {

tsf_status tsf_ctx_create(tsf_ctx **ctx)
{
    if (!ctx) return tsf_fail(TSF_E_ARG, "null ctx pointer");
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return tsf_fail(TSF_E_DEVICE, "hipGetDevice failed");
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return tsf_fail(TSF_E_DEVICE, "hipDeviceGetAttribute failed");
    tsf_ctx *c = new tsf_ctx;
    std::memset(c, 0, sizeof *c);
    c->device = dev;
    c->cu_count = cus;
    if (hipStreamCreateWithFlags(&c->capture, hipStreamNonBlocking) != hipSuccess) {
        delete c;
        return tsf_fail(TSF_E_DEVICE, "cannot create the capture stream");
    }
    *ctx = c;
    return TSF_OK;
}

tsf_status tsf_ctx_destroy(tsf_ctx *ctx)
{
    if (!ctx) return TSF_OK;
    for (GraphEntry &g : ctx->graphs)
        if (g.used) {
            hipGraphExecDestroy(g.exec);
            hipGraphDestroy(g.graph);
        }
    if (ctx->capture) hipStreamDestroy(ctx->capture);
    if (ctx->scratch) hipFree(ctx->scratch);
    delete ctx;
    return TSF_OK;
}

tsf_status tsf_walk_init(tsf_ctx *ctx, const tsf_walk_batch *b, void *hip_stream)
{
    (void)ctx;
    tsf_status st = check_batch(b);
    if (st) return st;
    if (b->n_walks == 0) return TSF_OK;
    hipStream_t s = (hipStream_t)hip_stream;
    hipLaunchKernelGGL(init_kernel, dim3(b->n_walks), dim3(64), 0, s, b->hdr, b->cur, b->best,
                       b->start, b->n_walks, b->capacity);
    if (hipGetLastError() != hipSuccess) return tsf_fail(TSF_E_DEVICE, "init launch failed");
    return TSF_OK;
}

}  // extern "C"

namespace {

struct Launch {
    KernelFn fn;
    dim3 grid, block;
    size_t lds;
    int g;
    bool ap, ix;
};

// validate a walk call and build its kernel arguments and launch shape
tsf_status prepare_walk(const tsf_walk_params *prm, const tsf_walk_batch *b, int64_t n_iters,
                        const tsf_launch *launch, KArgs &a, Launch &L, bool checked = false)
{
    tsf_status st = check_batch(b);
    if (st) return st;
    if (!prm) return tsf_fail(TSF_E_ARG, "null params");
    if (prm->flip_tries < 1 || prm->flip_tries > 64)
        return tsf_fail(TSF_E_ARG, "flip_tries %d outside [1, 64]", prm->flip_tries);
    if (prm->t_eq > (1ull << 32) || prm->t_reduce > (1ull << 32) || prm->t_expand > (1ull << 32))
        return tsf_fail(TSF_E_ARG, "a probability threshold exceeds 2^32");
    if (n_iters < 0) return tsf_fail(TSF_E_ARG, "n_iters < 0");
    if (prm->objective != TSF_OBJ_RANK && prm->objective != TSF_OBJ_ADDITIONS)
        return tsf_fail(TSF_E_ARG, "objective %d", prm->objective);
    if (b->log && b->log_cap < 0) return tsf_fail(TSF_E_ARG, "log_cap < 0");
    int strategy = launch ? launch->strategy : 0;
    if (strategy < 0 || strategy > 3) return tsf_fail(TSF_E_ARG, "strategy %d not in 0..3", strategy);
    // default: the indexed strategy up to 64 terms; the plain attempt-parallel
    // one up to 128 terms of 32-bit factors; the term-parallel one beyond and
    // for 64-bit factors (measured on the exploratory workload, capacity 128:
    // its LDS per walk keeps the attempt-parallel kernels at few wavefronts
    // per CU once the schemes grow)
    const bool wide = b->max_len > 32;
    if (strategy == 0) strategy = b->capacity <= 64 ? 3 : (b->capacity <= 128 && !wide ? 1 : 2);
    const bool ap = strategy == 1 || strategy == 3;
    const bool ix = strategy == 3;
    if (ix && b->capacity > 64)
        return tsf_fail(TSF_E_CAPACITY, "the indexed strategy needs capacity <= 64");
    if (ap && b->capacity > 128)
        return tsf_fail(TSF_E_CAPACITY, "the attempt-parallel strategy needs capacity <= 128");
    int g = launch && launch->lanes_per_walk ? launch->lanes_per_walk : (ap ? 8 : 64);
    int wpb = launch && launch->waves_per_block ? launch->waves_per_block : 1;
    if (g != 4 && g != 8 && g != 16 && g != 32 && g != 64)
        return tsf_fail(TSF_E_ARG, "lanes_per_walk %d not in {4,8,16,32,64}", g);
    if (g == 4 && !ap)
        return tsf_fail(TSF_E_ARG, "4 lanes per walk only with the attempt-parallel strategies");
    if (ap && g == 64)
        return tsf_fail(TSF_E_ARG, "the attempt-parallel strategies use 4 to 32 lanes per walk");
    if (wpb < 1 || wpb > 4) return tsf_fail(TSF_E_ARG, "waves_per_block %d not in 1..4", wpb);
    // term slots per lane (term-parallel kernels), or 64-bit words of a
    // partner set (attempt-parallel kernels)
    const int s = ap ? (b->capacity > 64 ? 2 : 1) : slots_for(b->capacity, g);
    if (s < 0)
        return tsf_fail(TSF_E_CAPACITY, "capacity %d needs more than 8 slots at %d lanes/walk",
                        b->capacity, g);
    // factors of at most 16 entries: the indexed kernels keep each factor's
    // digits and signs in one 32-bit LDS word
    const bool pk = ix && !wide && b->max_len <= 16;
    if (checked && g != (ap ? 8 : 64))
        return tsf_fail(TSF_E_ARG, "checked walks use %d lanes per walk with this strategy",
                        ap ? 8 : 64);
    L.fn = pick_kernel(g, s, wide, b->mode == TSF_Z2, pk ? 4 : strategy, checked);
    if (!L.fn) return tsf_fail(TSF_E_ARG, "no kernel for this configuration");
    const size_t word = wide ? 8 : 4;
    const size_t factor_bytes = pk ? 4 : 2 * word;
    const int walks_per_wave = 64 / g;
    // LDS stride per factor kind: capacity rounded up to even (to a multiple
    // of 4 for the indexed strategy, which reads four terms at a time)
    const int cap2 = ix ? (b->capacity + 3) & ~3 : b->capacity + (b->capacity & 1);
    // per walk: the terms, and for the indexed strategy 3 match masks per term
    // (rows of `capacity` masks, not padded)
    const size_t per_walk = (size_t)cap2 * 3 * factor_bytes + (ix ? (size_t)b->capacity * 3 * 8 : 0);
    L.lds = (size_t)wpb * walks_per_wave * per_walk;
    if (L.lds > 160 * 1024)
        return tsf_fail(TSF_E_CAPACITY, "%zu bytes of LDS per workgroup exceed 160 KiB", L.lds);
    std::memset(&a, 0, sizeof a);
    a.base_seed = prm->base_seed;
    a.params_hash = tsf_params_hash(prm);
    a.first_walk_id = prm->first_walk_id;
    a.max_iters = prm->max_iters;
    a.plateau = prm->plateau;
    a.n_iters = n_iters;
    a.t_eq = prm->t_eq;
    a.t_reduce = prm->t_reduce;
    a.t_expand = prm->t_expand;
    a.flip_tries = prm->flip_tries;
    a.restart_from_best = prm->restart_from_best;
    a.objective = prm->objective;
    a.n_walks = b->n_walks;
    a.cap = b->capacity;
    a.rec_cap = b->rec_cap;
    a.mode = b->mode;
    a.max_len = b->max_len;
    a.cap2 = cap2;
    a.capm = b->capacity;
    a.log = b->log;
    a.log_cap = b->log ? b->log_cap : 0;
    a.hdr = b->hdr;
    a.cur = b->cur;
    a.best = b->best;
    a.start = b->start;
    a.rec = b->rec;
    const int64_t walks_per_block = (int64_t)wpb * walks_per_wave;
    const int64_t blocks = (b->n_walks + walks_per_block - 1) / walks_per_block;
    L.grid = dim3((unsigned)blocks);
    L.block = dim3(64 * wpb);
    L.g = g;
    L.ap = ap;
    L.ix = ix;
    if (L.lds > 64 * 1024 &&
        hipFuncSetAttribute((const void *)L.fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)L.lds) != hipSuccess)
        return tsf_fail(TSF_E_DEVICE, "cannot raise the LDS limit to %zu bytes", L.lds);
    return TSF_OK;
}

tsf_status run(const Launch &L, const KArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(L.fn, L.grid, L.block, L.lds, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return tsf_fail(TSF_E_DEVICE, "walk launch failed: %s", hipGetErrorString(e));
    return TSF_OK;
}

}  // namespace

extern "C" {

tsf_status tsf_walk(tsf_ctx *ctx, const tsf_walk_params *prm, const tsf_walk_batch *b,
                    int64_t n_iters, const tsf_launch *launch, void *hip_stream)
{
    if (launch_is_default(launch) && b) {
        const tsf_launch *t = tuned_launch(ctx, b);
        if (t) launch = t;
    }
    KArgs a;
    Launch L;
    tsf_status st = prepare_walk(prm, b, n_iters, launch, a, L);
    if (st) return st;
    if (b->n_walks == 0 || n_iters == 0) return TSF_OK;
    return run(L, a, (hipStream_t)hip_stream);
}

tsf_status tsf_walk_checked(tsf_ctx *ctx, const tsf_walk_params *prm, const tsf_walk_batch *b,
                            int64_t n_iters, const tsf_launch *launch, void *hip_stream)
{
    (void)ctx;  // the autotuner's choices are not used: they may name other shapes
    KArgs a;
    Launch L;
    tsf_status st = prepare_walk(prm, b, n_iters, launch, a, L, true);
    if (st) return st;
    if (b->n_walks == 0 || n_iters == 0) return TSF_OK;
    return run(L, a, (hipStream_t)hip_stream);
}

tsf_status tsf_autotune(tsf_ctx *ctx, const tsf_walk_params *prm, const tsf_walk_batch *b,
                        int64_t trial_iters, tsf_launch *chosen, void *hip_stream)
{
    if (!ctx) return tsf_fail(TSF_E_ARG, "null context");
    tsf_status st = check_batch(b);
    if (st) return st;
    if (!prm || trial_iters < 1) return tsf_fail(TSF_E_ARG, "bad params or trial_iters");
    if (b->n_walks == 0) return tsf_fail(TSF_E_ARG, "empty batch");
    const size_t n = (size_t)b->n_walks;
    const size_t sz_hdr = n * sizeof(tsf_walk_header);
    const size_t sz_sch = n * (size_t)b->capacity * 6 * sizeof(uint64_t);
    const size_t sz_rec = n * (size_t)(b->rec_cap > 0 ? b->rec_cap : 1) * sizeof(tsf_record);
    const size_t need = 2 * (sz_hdr + 2 * sz_sch + sz_rec);
    if (ctx->scratch_bytes < need) {
        if (ctx->scratch) hipFree(ctx->scratch);
        ctx->scratch = nullptr;
        ctx->scratch_bytes = 0;
        if (hipMalloc(&ctx->scratch, need) != hipSuccess)
            return tsf_fail(TSF_E_DEVICE, "cannot allocate %zu bytes for the autotuner", need);
        ctx->scratch_bytes = need;
    }
    hipStream_t s = (hipStream_t)hip_stream;
    // snapshot of the batch (first half of the scratch) and the trial copy
    unsigned char *base = (unsigned char *)ctx->scratch;
    unsigned char *snap = base, *trial = base + need / 2;
    auto lay = [&](unsigned char *p, tsf_walk_batch &c) {
        c = *b;
        c.hdr = (tsf_walk_header *)p;
        c.cur = (uint64_t *)(p + sz_hdr);
        c.best = (uint64_t *)(p + sz_hdr + sz_sch);
        c.rec = (tsf_record *)(p + sz_hdr + 2 * sz_sch);
        c.log = nullptr;
        c.log_cap = 0;
    };
    tsf_walk_batch bs, bt;
    lay(snap, bs);
    lay(trial, bt);
    bool ok = hipMemcpyAsync(bs.hdr, b->hdr, sz_hdr, hipMemcpyDeviceToDevice, s) == hipSuccess &&
              hipMemcpyAsync(bs.cur, b->cur, sz_sch, hipMemcpyDeviceToDevice, s) == hipSuccess &&
              hipMemcpyAsync(bs.best, b->best, sz_sch, hipMemcpyDeviceToDevice, s) == hipSuccess;
    if (!ok) return tsf_fail(TSF_E_DEVICE, "autotuner snapshot failed");
    std::vector<tsf_launch> cands;
    for (int wpb : {1, 2, 4}) {
        for (int st : {3, 1})
            if (b->capacity <= (st == 3 ? 64 : 128))
                for (int g : {4, 8, 16}) cands.push_back(tsf_launch{g, wpb, st});
        for (int g : {16, 32, 64}) cands.push_back(tsf_launch{g, wpb, 2});
    }
    hipEvent_t e0, e1;
    hipEventCreate(&e0);
    hipEventCreate(&e1);
    float best_ms = -1.0f;
    tsf_launch best{0, 0, 0};
    for (const tsf_launch &c : cands) {
        KArgs a;
        Launch L;
        if (prepare_walk(prm, &bt, trial_iters, &c, a, L) != TSF_OK) continue;
        hipMemcpyAsync(bt.hdr, bs.hdr, sz_hdr, hipMemcpyDeviceToDevice, s);
        hipMemcpyAsync(bt.cur, bs.cur, sz_sch, hipMemcpyDeviceToDevice, s);
        hipMemcpyAsync(bt.best, bs.best, sz_sch, hipMemcpyDeviceToDevice, s);
        hipEventRecord(e0, s);
        if (run(L, a, s) != TSF_OK) continue;
        hipEventRecord(e1, s);
        if (hipEventSynchronize(e1) != hipSuccess) break;
        float ms = 0.0f;
        hipEventElapsedTime(&ms, e0, e1);
        if (best_ms < 0.0f || ms < best_ms) {
            best_ms = ms;
            best = c;
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (best_ms < 0.0f) return tsf_fail(TSF_E_CAPACITY, "no launch configuration fits the batch");
    TuneEntry *slot = nullptr;
    const int sc = size_class(b->n_walks);
    for (TuneEntry &e : ctx->tuned)
        if (e.used && e.capacity == b->capacity && e.max_len == b->max_len && e.mode == b->mode &&
            e.size_class == sc)
            slot = &e;
    if (!slot) {
        slot = &ctx->tuned[ctx->next_tuned];
        ctx->next_tuned = (ctx->next_tuned + 1) % 16;
    }
    *slot = TuneEntry{b->capacity, b->max_len, b->mode, sc, best, true};
    if (chosen) *chosen = best;
    return TSF_OK;
}

tsf_status tsf_walk_learned(tsf_ctx *ctx, const tsf_walk_params *prm, const tsf_walk_batch *b,
                            const tsf_mlp *net, const tsf_learn_ws *ws, int64_t n_iters,
                            const tsf_launch *launch, void *hip_stream)
{
    KArgs a;
    Launch L;
    // the propose and apply phases are kernels of the plain attempt-parallel
    // strategy (the scheme is reloaded by every launch, so an index would be
    // rebuilt each time)
    tsf_launch la = launch ? *launch : tsf_launch{0, 0, 0};
    if (la.strategy == 0) la.strategy = 1;
    if (la.strategy != 1)
        return tsf_fail(TSF_E_ARG, "learned proposals use the attempt-parallel strategy 1");
    if (prm && prm->objective != TSF_OBJ_RANK)
        return tsf_fail(TSF_E_ARG, "learned proposals serve the rank objective only");
    tsf_status st = prepare_walk(prm, b, n_iters, &la, a, L);
    if (st) return st;
    if (!L.ap)
        return tsf_fail(TSF_E_CAPACITY,
                        "learned proposals use the attempt-parallel strategy (capacity <= 64)");
    const int K = prm->flip_tries;
    if (K > L.g - 1 || K > kLearnRows)
        return tsf_fail(TSF_E_ARG, "flip_tries %d exceeds the %d attempts scored at %d lanes/walk",
                        K, L.g - 1 < kLearnRows ? L.g - 1 : kLearnRows, L.g);
    if (!net || !ws || !ws->cand || !ws->feat || !ws->h1 || !ws->h2 || !ws->logit)
        return tsf_fail(TSF_E_ARG, "null learned-proposal buffer");
    if (ws->choice && ws->choice_cap < 0) return tsf_fail(TSF_E_ARG, "choice_cap < 0");
    if (b->n_walks == 0 || n_iters == 0) return TSF_OK;
    const int64_t rows = (int64_t)b->n_walks * kLearnRows;
    if (rows > 0x7FFFFFFF) return tsf_fail(TSF_E_CAPACITY, "too many candidate rows");
    a.learn_k = K;
    a.cand = ws->cand;
    a.feat = ws->feat;
    a.logit = ws->logit;
    a.choice = ws->choice;
    a.choice_cap = ws->choice ? ws->choice_cap : 0;
    a.n_iters = 1;
    hipStream_t s = (hipStream_t)hip_stream;
    // one learned iteration: propose, score, apply
    auto iteration = [&](hipStream_t on) -> tsf_status {
        tsf_status e;
        a.phase = 1;
        if ((e = run(L, a, on))) return e;
        if ((e = tsf_mlp_fwd(net, ws->feat, (int32_t)rows, ws->h1, ws->h2, ws->logit, on)))
            return e;
        a.phase = 2;
        return run(L, a, on);
    };
    // Every iteration launches the same kernels with the same arguments (the
    // walk state lives in device memory), so a chunk of iterations is
    // captured once into a HIP graph and replayed.
    const int64_t chunk = 16;
    if (!ctx || n_iters < chunk) {
        for (int64_t it = 0; it < n_iters; ++it)
            if ((st = iteration(s))) return st;
        return TSF_OK;
    }
    unsigned char key[sizeof(GraphEntry::key)];
    std::memset(key, 0, sizeof key);
    a.phase = 0;
    std::memcpy(key, &a, sizeof a);
    const void *ptrs[8] = {net->param, net->wbf, ws->cand, ws->feat, ws->h1, ws->h2, ws->logit,
                           (const void *)L.fn};
    std::memcpy(key + sizeof a, ptrs, sizeof ptrs);
    GraphEntry *ge = nullptr;
    for (GraphEntry &g : ctx->graphs)
        if (g.used && g.chunk == chunk && std::memcmp(g.key, key, sizeof key) == 0) ge = &g;
    if (!ge) {
        ge = &ctx->graphs[ctx->next_graph];
        ctx->next_graph = (ctx->next_graph + 1) % 8;
        if (ge->used) {
            hipGraphExecDestroy(ge->exec);
            hipGraphDestroy(ge->graph);
            ge->used = false;
        }
        if (hipStreamBeginCapture(ctx->capture, hipStreamCaptureModeThreadLocal) != hipSuccess)
            return tsf_fail(TSF_E_DEVICE, "stream capture failed to start");
        for (int64_t it = 0; it < chunk; ++it)
            if ((st = iteration(ctx->capture))) {
                hipGraph_t dummy;
                hipStreamEndCapture(ctx->capture, &dummy);
                if (dummy) hipGraphDestroy(dummy);
                return st;
            }
        if (hipStreamEndCapture(ctx->capture, &ge->graph) != hipSuccess)
            return tsf_fail(TSF_E_DEVICE, "stream capture failed");
        if (hipGraphInstantiate(&ge->exec, ge->graph, nullptr, nullptr, 0) != hipSuccess) {
            hipGraphDestroy(ge->graph);
            return tsf_fail(TSF_E_DEVICE, "graph instantiation failed");
        }
        std::memcpy(ge->key, key, sizeof key);
        ge->chunk = chunk;
        ge->used = true;
    }
    int64_t done = 0;
    for (; done + chunk <= n_iters; done += chunk)
        if (hipGraphLaunch(ge->exec, s) != hipSuccess)
            return tsf_fail(TSF_E_DEVICE, "graph launch failed");
    for (; done < n_iters; ++done)
        if ((st = iteration(s))) return st;
    return TSF_OK;
}

tsf_status tsf_meta_batch(const tsf_walk_batch *in, int32_t which, const int32_t *op,
                          const int32_t *axis, const int32_t *index, int32_t r_cap_extra,
                          const tsf_walk_batch *out, void *hip_stream)
{
    tsf_status st = check_batch(in);
    if (st) return st;
    if ((st = check_batch(out))) return st;
    if (in->n_walks != out->n_walks) return tsf_fail(TSF_E_ARG, "batches differ in n_walks");
    if (which < 0 || which > 1) return tsf_fail(TSF_E_ARG, "which %d not in 0..1", which);
    if (r_cap_extra < 0) return tsf_fail(TSF_E_ARG, "r_cap_extra < 0");
    if (in->n_walks == 0) return TSF_OK;
    if (!op || !axis || !index) return tsf_fail(TSF_E_ARG, "null op/axis/index");
    if ((const void *)in->start == (const void *)out->start || in->cur == out->start ||
        in->best == out->start)
        return tsf_fail(TSF_E_ARG, "in and out must not share scheme buffers");
    hipLaunchKernelGGL(meta_kernel, dim3(in->n_walks), dim3(64), 0, (hipStream_t)hip_stream, *in,
                       which, op, axis, index, r_cap_extra, *out);
    if (hipGetLastError() != hipSuccess) return tsf_fail(TSF_E_DEVICE, "meta launch failed");
    return TSF_OK;
}

tsf_status tsf_features_from_log(const tsf_flip_log *log, int64_t n, uint16_t *X, void *hip_stream)
{
    if (n < 0 || (n > 0 && (!log || !X))) return tsf_fail(TSF_E_ARG, "bad feature arguments");
    if (n == 0) return TSF_OK;
    hipLaunchKernelGGL(features_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                       (hipStream_t)hip_stream, log, n, X);
    if (hipGetLastError() != hipSuccess) return tsf_fail(TSF_E_DEVICE, "feature launch failed");
    return TSF_OK;
}

tsf_status tsf_population_best(const tsf_walk_batch *b, tsf_best_entry *table, int32_t *n_entries,
                               uint64_t *work, int32_t slots, void *hip_stream)
{
    tsf_status st = check_batch(b);
    if (st) return st;
    if (slots < 1 || slots > kMaxSlots)
        return tsf_fail(TSF_E_ARG, "slots %d outside [1, %d]", slots, kMaxSlots);
    if (!table || !n_entries || !work) return tsf_fail(TSF_E_ARG, "null table or workspace");
    return launch_population(b, table, n_entries, work, slots, nullptr, (hipStream_t)hip_stream);
}

tsf_status tsf_population_best_noalloc(const tsf_walk_batch *b, tsf_best_entry *table,
                                       int32_t *n_entries, int32_t slots, int32_t *dropped,
                                       void *hip_stream)
{
    tsf_status st = check_batch(b);
    if (st) return st;
    if (slots < 1 || slots > kMaxSlots)
        return tsf_fail(TSF_E_ARG, "slots %d outside [1, %d] (the size of the library's table)",
                        slots, kMaxSlots);
    if (!table || !n_entries) return tsf_fail(TSF_E_ARG, "null table or count");
    uint64_t *work = nullptr;
    if ((st = population_scratch(&work))) return st;
    return launch_population(b, table, n_entries, work, slots, dropped, (hipStream_t)hip_stream);
}

tsf_status tsf_resize_batch(const tsf_walk_batch *in, int32_t which, const tsf_best_entry *table,
                            const int32_t *n_entries, const tsf_resize_params *prm,
                            const tsf_walk_batch *out, int32_t *applied, void *hip_stream)
{
    tsf_status st = check_batch(in);
    if (st) return st;
    if ((st = check_batch(out))) return st;
    if (in->n_walks != out->n_walks) return tsf_fail(TSF_E_ARG, "batches differ in n_walks");
    if (which < 0 || which > 1) return tsf_fail(TSF_E_ARG, "which %d not in 0..1", which);
    if (!prm || !table || !n_entries) return tsf_fail(TSF_E_ARG, "null argument");
    if (prm->r_cap_extra < 0 || prm->t_resize > (1ull << 32))
        return tsf_fail(TSF_E_ARG, "bad resize parameters");
    if (in->mode != out->mode) return tsf_fail(TSF_E_ARG, "batches differ in mode");
    if ((const void *)in->start == (const void *)out->start || in->cur == out->start ||
        in->best == out->start)
        return tsf_fail(TSF_E_ARG, "in and out must not share scheme buffers");
    if (in->n_walks == 0) return TSF_OK;
    hipLaunchKernelGGL(resize_kernel, dim3(in->n_walks), dim3(64), 0, (hipStream_t)hip_stream, *in,
                       which, table, n_entries, prm->base_seed, prm->first_walk_id, prm->round,
                       prm->t_resize, prm->r_cap_extra, *out, applied);
    if (hipGetLastError() != hipSuccess) return tsf_fail(TSF_E_DEVICE, "resize launch failed");
    return TSF_OK;
}

tsf_status tsf_invariants_batch(const tsf_walk_batch *b, int32_t which, uint8_t *term_ranks,
                                int32_t *rank_sums, void *hip_stream)
{
    tsf_status st = check_batch(b);
    if (st) return st;
    if (which < 0 || which > 2) return tsf_fail(TSF_E_ARG, "which %d not in 0..2", which);
    if (b->n_walks == 0) return TSF_OK;
    if (!term_ranks || !rank_sums) return tsf_fail(TSF_E_ARG, "null output");
    const uint64_t *src = which == 0 ? b->cur : which == 1 ? b->best : b->start;
    hipLaunchKernelGGL(invariants_kernel, dim3(b->n_walks), dim3(64), 0, (hipStream_t)hip_stream,
                       b->hdr, src, b->capacity, b->n_walks, which, term_ranks, rank_sums);
    if (hipGetLastError() != hipSuccess) return tsf_fail(TSF_E_DEVICE, "invariants launch failed");
    return TSF_OK;
}

tsf_status tsf_verify_batch(const tsf_walk_batch *b, int32_t which, int64_t *n_violated,
                            void *hip_stream)
{
    tsf_status st = check_batch(b);
    if (st) return st;
    if (which < 0 || which > 2) return tsf_fail(TSF_E_ARG, "which %d not in 0..2", which);
    if (!n_violated && b->n_walks) return tsf_fail(TSF_E_ARG, "null output");
    if (b->n_walks == 0) return TSF_OK;
    const uint64_t *src = which == 0 ? b->cur : which == 1 ? b->best : b->start;
    hipLaunchKernelGGL(verify_kernel, dim3(b->n_walks), dim3(256), 0, (hipStream_t)hip_stream,
                       b->hdr, src, b->capacity, b->n_walks, which, n_violated);
    if (hipGetLastError() != hipSuccess) return tsf_fail(TSF_E_DEVICE, "verify launch failed");
    return TSF_OK;
}

}  // extern "C"
