// lift.hip -- ternary lifting of a Z2 scheme (Sec. 3.10.1) as a parallel
// exhaustive search on the GPU.
//
// The search space and order (a fixed convention, so that the first lifting
// found is unique): per term the first non-zero entry of u and of v is +1 and the other non-zero entries --
// u ascending, then v, then w -- are the term's free signs, bit i of the
// term's pattern x meaning entry i is -1; terms in order, patterns
// ascending; after a term every equation it touches must stay reachable,
// |target - partial sum| <= the number of later terms touching it.  The
// patterns of the first P terms, read as one mixed-radix number (term 0 most
// significant), name a subtree; one wavefront searches one subtree depth
// first with the residuals of all equations in LDS, the lanes sharing the
// products of a term.  The first solution in the global order is the one in
// the smallest subtree that has a solution, provided every smaller subtree
// was searched to the end.
#include <hip/hip_runtime.h>

#include "../../include/tsf.h"
#include "tsf_bits.h"
#include "tsf_internal.h"

#include <cstdint>
#include <cstring>
#include <vector>

namespace {

constexpr int kLiftMaxEq = 8192;     // equations (mn)(np)(pm) searched on the GPU
constexpr int kLiftMaxTerms = 512;

struct LiftArgs {
    const uint64_t *d;      // r x 3 supports (u, v, w)
    int m, n, p, r, P;      // format, rank, prefix terms
    int64_t n_sub;          // subtrees
    int64_t max_nodes;      // per subtree
    int32_t *status;        // per subtree: 0 none, 1 found, 2 budget, 3 skipped
    unsigned long long *first;  // smallest subtree id with a solution
    uint64_t *signs;        // r x 3 sign masks of the solution (replay pass)
    int64_t replay;         // >= 0: search this subtree only and write its signs
};

__device__ __forceinline__ int nth_bit(uint64_t m, int k)
{
    for (int q = 0; q < k; ++q) m &= m - 1;
    return __builtin_ctzll(m);
}

struct LiftWave {
    const LiftArgs *a;
    int lane;
    int Lv, Lw;
    int16_t *res, *rem;
    int64_t *pat;           // pattern per term
    uint8_t *nfree;         // free signs per term

    __device__ uint64_t du(int l) const { return a->d[l * 3 + 0]; }
    __device__ uint64_t dv(int l) const { return a->d[l * 3 + 1]; }
    __device__ uint64_t dw(int l) const { return a->d[l * 3 + 2]; }

    // sign masks of term l under pattern x
    __device__ void sign_masks(int l, int64_t x, uint64_t &su, uint64_t &sv, uint64_t &sw) const
    {
        const uint64_t u = du(l), v = dv(l), w = dw(l);
        const int cu = __builtin_popcountll(u), cv = __builtin_popcountll(v);
        su = sv = sw = 0;
        int bit = 0;
        uint64_t q = u & (u - 1);   // u without its first entry
        for (; q; q &= q - 1, ++bit)
            if ((x >> bit) & 1) su |= q & (~q + 1);
        q = v & (v - 1);
        for (; q; q &= q - 1, ++bit)
            if ((x >> bit) & 1) sv |= q & (~q + 1);
        for (q = w; q; q &= q - 1, ++bit)
            if ((x >> bit) & 1) sw |= q & (~q + 1);
        (void)cu;
        (void)cv;
    }

    // add (dir -1) or remove (+1) term l's products under pattern x; returns
    // whether every touched equation stays reachable (when adding)
    __device__ bool apply(int l, int64_t x, int dir)
    {
        uint64_t su, sv, sw;
        sign_masks(l, x, su, sv, sw);
        const uint64_t u = du(l), v = dv(l), w = dw(l);
        const int cu = __builtin_popcountll(u), cv = __builtin_popcountll(v),
                  cw = __builtin_popcountll(w);
        const int total = cu * cv * cw;
        bool ok = true;
        for (int c = lane; c < total; c += 64) {
            const int qa = c / (cv * cw), qb = (c / cw) % cv, qc = c % cw;
            const int ea = nth_bit(u, qa), eb = nth_bit(v, qb), ec = nth_bit(w, qc);
            const int neg = (int)(((su >> ea) ^ (sv >> eb) ^ (sw >> ec)) & 1);
            const int e = (ea * Lv + eb) * Lw + ec;
            const int r2 = res[e] + dir * (neg ? -1 : 1);
            const int m2 = rem[e] + dir;
            res[e] = (int16_t)r2;
            rem[e] = (int16_t)m2;
            if (dir < 0 && (r2 > m2 || -r2 > m2)) ok = false;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        return __ballot(!ok) == 0;
    }
};

__global__ void __launch_bounds__(64) lift_kernel(LiftArgs a)
{
    __shared__ int16_t res[kLiftMaxEq], rem[kLiftMaxEq];
    __shared__ int64_t pat[kLiftMaxTerms];
    __shared__ uint8_t nfree[kLiftMaxTerms];
    const int64_t sub = a.replay >= 0 ? a.replay : (int64_t)blockIdx.x;
    const int lane = threadIdx.x;
    if (sub >= a.n_sub) return;
    int32_t *st = a.status + (a.replay >= 0 ? 0 : sub);
    LiftWave W{&a, lane, a.n * a.p, a.p * a.m, res, rem, pat, nfree};
    const int Lu = a.m * a.n, E = Lu * W.Lv * W.Lw;
    // targets and contributor counts
    for (int e = lane; e < E; e += 64) {
        const int ea = e / (W.Lv * W.Lw), eb = (e / W.Lw) % W.Lv, ec = e % W.Lw;
        const int a1 = ea / a.n, a2 = ea % a.n, b1 = eb / a.p, b2 = eb % a.p, c1 = ec / a.m,
                  c2 = ec % a.m;
        res[e] = (a2 == b1 && b2 == c1 && c2 == a1) ? 1 : 0;
        rem[e] = 0;
    }
    for (int l = lane; l < a.r; l += 64)
        nfree[l] = (uint8_t)(__builtin_popcountll(W.du(l)) - 1 + __builtin_popcountll(W.dv(l)) - 1 +
                             __builtin_popcountll(W.dw(l)));
    __syncthreads();
    for (int l = 0; l < a.r; ++l) {
        const uint64_t u = W.du(l), v = W.dv(l), w = W.dw(l);
        const int cv = __builtin_popcountll(v), cw = __builtin_popcountll(w);
        const int total = __builtin_popcountll(u) * cv * cw;
        for (int c = lane; c < total; c += 64) {
            const int e = (nth_bit(u, c / (cv * cw)) * W.Lv + nth_bit(v, (c / cw) % cv)) * W.Lw +
                          nth_bit(w, c % cw);
            rem[e] = (int16_t)(rem[e] + 1);
        }
        __syncthreads();
    }
    // the subtree's prefix: patterns of terms 0..P-1 from the mixed-radix id
    int64_t rest = sub;
    for (int l = a.P - 1; l >= 0; --l) {
        const int64_t radix = 1ll << nfree[l];
        if (lane == 0) pat[l] = rest % radix;
        rest /= radix;
    }
    __syncthreads();
    bool alive = true;
    for (int l = 0; l < a.P && alive; ++l) alive = W.apply(l, pat[l], -1);
    int status = alive ? 0 : 0;
    int64_t nodes = 0;
    if (alive) {
        int l = a.P;
        int64_t x = 0;
        bool found = a.P == a.r;
        while (!found) {
            // another wavefront found a solution in a smaller subtree
            if (a.replay < 0 && (nodes & 255) == 0 &&
                __atomic_load_n(a.first, __ATOMIC_RELAXED) < (unsigned long long)sub) {
                status = 3;
                break;
            }
            if (x == (1ll << nfree[l])) {
                // this level is exhausted: back to the previous free level
                if (l == a.P) break;
                --l;
                W.apply(l, pat[l], +1);
                x = pat[l] + 1;
                continue;
            }
            if (nodes >= a.max_nodes) {
                status = 2;
                break;
            }
            ++nodes;
            if (lane == 0) pat[l] = x;
            __syncthreads();
            if (W.apply(l, x, -1)) {
                ++l;
                x = 0;
                found = l == a.r;
            } else {
                W.apply(l, x, +1);
                ++x;
            }
        }
        if (found) status = 1;
    }
    if (lane == 0) *st = status;
    if (status == 1 && lane == 0 && a.replay < 0) atomicMin(a.first, (unsigned long long)sub);
    if (status == 1 && a.replay >= 0)
        for (int l = lane; l < a.r; l += 64) {
            uint64_t su, sv, sw;
            W.sign_masks(l, pat[l], su, sv, sw);
            a.signs[l * 3 + 0] = su;
            a.signs[l * 3 + 1] = sv;
            a.signs[l * 3 + 2] = sw;
        }
}

}  // namespace

extern "C" {

tsf_status tsf_lift(const tsf_scheme *z2, int64_t max_nodes, int32_t max_subtrees,
                    tsf_scheme *out, tsf_lift_result *res)
{
    if (!z2 || !out || !res || !z2->U || !z2->V || !z2->W || !out->U || !out->V || !out->W)
        return tsf_fail(TSF_E_ARG, "null argument");
    if (z2->d.mode != TSF_Z2) return tsf_fail(TSF_E_ARG, "the input must be a Z2 scheme");
    if (max_nodes < 1 || max_subtrees < 1) return tsf_fail(TSF_E_ARG, "bad search limits");
    const int m = z2->d.m, n = z2->d.n, p = z2->d.p, r = z2->d.rank;
    if (m < 1 || n < 1 || p < 1 || m * n > 64 || n * p > 64 || p * m > 64)
        return tsf_fail(TSF_E_FORMAT, "format (%d,%d,%d)", m, n, p);
    if ((int64_t)m * n * n * p * p * m > kLiftMaxEq)
        return tsf_fail(TSF_E_CAPACITY, "more than %d Brent equations", kLiftMaxEq);
    if (r < 1 || r > kLiftMaxTerms || r > z2->d.capacity || out->d.capacity < r)
        return tsf_fail(TSF_E_CAPACITY, "rank %d", r);
    const int len[3] = {m * n, n * p, p * m};
    const int8_t *mat[3] = {z2->U, z2->V, z2->W};
    std::vector<uint64_t> d((size_t)r * 3, 0);
    std::vector<int> nfree(r);
    for (int l = 0; l < r; ++l) {
        for (int X = 0; X < 3; ++X)
            for (int e = 0; e < len[X]; ++e) {
                const int8_t c = mat[X][(size_t)l * len[X] + e];
                if (c != 0 && c != 1) return tsf_fail(TSF_E_NOT_TERNARY, "Z2 coefficient %d", c);
                if (c) d[l * 3 + X] |= 1ull << e;
            }
        if (!d[l * 3] || !d[l * 3 + 1] || !d[l * 3 + 2])
            return tsf_fail(TSF_E_ARG, "term %d has a zero factor", l);
        nfree[l] = __builtin_popcountll(d[l * 3]) - 1 + __builtin_popcountll(d[l * 3 + 1]) - 1 +
                   __builtin_popcountll(d[l * 3 + 2]);
        if (nfree[l] > 40) return tsf_fail(TSF_E_CAPACITY, "term %d has %d free signs", l, nfree[l]);
    }
    // prefix terms: as many leading terms as keep the subtrees within the limit
    int P = 0;
    int64_t n_sub = 1;
    while (P < r && n_sub * (1ll << nfree[P]) <= max_subtrees) n_sub *= 1ll << nfree[P++];
    uint64_t *d_d = nullptr, *d_signs = nullptr;
    int32_t *d_status = nullptr;
    unsigned long long *d_first = nullptr;
    tsf_status st = TSF_OK;
    if (hipMalloc(&d_d, d.size() * 8) != hipSuccess || hipMalloc(&d_signs, d.size() * 8) != hipSuccess ||
        hipMalloc(&d_status, (size_t)n_sub * 4) != hipSuccess ||
        hipMalloc(&d_first, 8) != hipSuccess) {
        st = tsf_fail(TSF_E_DEVICE, "lift buffers");
    } else {
        const unsigned long long none = ~0ull;
        hipMemcpy(d_d, d.data(), d.size() * 8, hipMemcpyHostToDevice);
        hipMemcpy(d_first, &none, 8, hipMemcpyHostToDevice);
        LiftArgs a{d_d, m, n, p, r, P, n_sub, max_nodes, d_status, d_first, d_signs, -1};
        hipLaunchKernelGGL(lift_kernel, dim3((unsigned)n_sub), dim3(64), 0, 0, a);
        std::vector<int32_t> status((size_t)n_sub);
        unsigned long long first = none;
        if (hipGetLastError() != hipSuccess || hipDeviceSynchronize() != hipSuccess ||
            hipMemcpy(status.data(), d_status, (size_t)n_sub * 4, hipMemcpyDeviceToHost) != hipSuccess ||
            hipMemcpy(&first, d_first, 8, hipMemcpyDeviceToHost) != hipSuccess) {
            st = tsf_fail(TSF_E_DEVICE, "lift search failed");
        } else {
            int64_t budget_first = -1;
            for (int64_t q = 0; q < n_sub; ++q)
                if (status[q] == 2) {
                    budget_first = q;
                    break;
                }
            std::memset(res, 0, sizeof *res);
            res->subtrees = n_sub;
            res->prefix_terms = P;
            for (int64_t q = 0; q < n_sub; ++q) res->exhausted += status[q] == 0 || status[q] == 1;
            if (first != none) {
                res->status = (budget_first < 0 || (int64_t)first < budget_first) ? 1 : 2;
                res->subtree = (int64_t)first;
                a.replay = (int64_t)first;
                a.max_nodes = INT64_MAX;
                hipLaunchKernelGGL(lift_kernel, dim3(1), dim3(64), 0, 0, a);
                std::vector<uint64_t> s(d.size());
                if (hipGetLastError() != hipSuccess || hipDeviceSynchronize() != hipSuccess ||
                    hipMemcpy(s.data(), d_signs, s.size() * 8, hipMemcpyDeviceToHost) != hipSuccess) {
                    st = tsf_fail(TSF_E_DEVICE, "lift replay failed");
                } else {
                    const int32_t out_cap = out->d.capacity;   // the caller's buffers
                    out->d = z2->d;
                    out->d.capacity = out_cap;
                    out->d.mode = TSF_TERNARY;
                    int8_t *om[3] = {out->U, out->V, out->W};
                    for (int X = 0; X < 3; ++X)
                        std::memset(om[X], 0, (size_t)out->d.capacity * len[X]);
                    for (int l = 0; l < r; ++l)
                        for (int X = 0; X < 3; ++X)
                            for (int e = 0; e < len[X]; ++e)
                                if ((d[l * 3 + X] >> e) & 1)
                                    om[X][(size_t)l * len[X] + e] =
                                        ((s[l * 3 + X] >> e) & 1) ? -1 : 1;
                }
            } else {
                res->status = budget_first < 0 ? 0 : -1;
                res->subtree = -1;
            }
        }
    }
    if (d_d) hipFree(d_d);
    if (d_signs) hipFree(d_signs);
    if (d_status) hipFree(d_status);
    if (d_first) hipFree(d_first);
    return st;
}

}  // extern "C"
