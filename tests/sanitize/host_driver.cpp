// Sanitizer driver for the host half of libtsf (host.cpp): every host
// scheme operation of include/tsf.h on schemes of several formats and both
// coefficient sets, plus their error paths.  Built with AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_sanitize.py; exits 0 when every
// call behaves as declared (sanitizer findings abort the program).
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../../include/tsf.h"

namespace {

int failures = 0;

#define CHECK(cond)                                                                 \
    do {                                                                            \
        if (!(cond)) {                                                              \
            std::fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #cond); \
            ++failures;                                                             \
        }                                                                           \
    } while (0)

// a scheme whose buffers hold exactly `cap` rows of each factor
struct Owned {
    std::vector<int8_t> U, V, W;
    tsf_scheme s{};
    Owned(int m, int n, int p, int cap, int mode)
        : U((size_t)cap * m * n), V((size_t)cap * n * p), W((size_t)cap * p * m)
    {
        s.d = tsf_dims{m, n, p, 0, cap, mode};
        s.U = U.data();
        s.V = V.data();
        s.W = W.data();
    }
};

int64_t violations(const tsf_scheme &s)
{
    int64_t nv = -1;
    CHECK(tsf_verify(&s, &nv) == TSF_OK);
    return nv;
}

void one_format(int m, int n, int p, int mode)
{
    const int r0 = m * n * p;
    Owned a(m, n, p, r0, mode);
    CHECK(tsf_init_scheme(m, n, p, mode, &a.s) == TSF_OK);
    CHECK(a.s.d.rank == r0);
    CHECK(violations(a.s) == 0);
    CHECK(tsf_normalise(&a.s) == TSF_OK);
    int32_t red = -1;
    CHECK(tsf_reduce(&a.s, &red) == TSF_OK && red == 0);
    // pack / unpack round trip
    std::vector<uint64_t> packed((size_t)r0 * 6);
    CHECK(tsf_pack(&a.s, packed.data()) == TSF_OK);
    Owned b(m, n, p, r0, mode);
    CHECK(tsf_unpack(packed.data(), &a.s.d, &b.s) == TSF_OK);
    CHECK(b.U == a.U && b.V == a.V && b.W == a.W);
    // invariants
    std::vector<uint8_t> ranks((size_t)r0 * 3);
    tsf_invariants inv;
    CHECK(tsf_scheme_invariants(&a.s, ranks.data(), &inv) == TSF_OK);
    CHECK(inv.rank_sum[0] == r0 && inv.rank_sum[1] == r0 && inv.rank_sum[2] == r0);
    // project each index of each axis, then extend back along that axis
    const int dims[3] = {m, n, p};
    for (int axis = 0; axis < 3; ++axis) {
        if (dims[axis] < 2) continue;
        for (int idx = 0; idx < dims[axis]; ++idx) {
            const int pm = m - (axis == 0), pn = n - (axis == 1), pp = p - (axis == 2);
            Owned pr(pm, pn, pp, r0, mode);
            CHECK(tsf_meta_project(&a.s, axis, idx, &pr.s) == TSF_OK);
            CHECK(pr.s.d.rank == pm * pn * pp && violations(pr.s) == 0);
            const int extra = axis == 0 ? pn * pp : axis == 1 ? pm * pp : pm * pn;
            Owned ex(m, n, p, pr.s.d.rank + extra, mode);
            CHECK(tsf_meta_extend(&pr.s, axis, &ex.s) == TSF_OK);
            CHECK(ex.s.d.rank == r0 && violations(ex.s) == 0);
        }
        CHECK(tsf_meta_project(&a.s, axis, dims[axis], &b.s) == TSF_E_ARG);
    }
    // swap twice: back to the same format
    Owned sw(m, p, n, r0, mode), sw2(m, n, p, r0, mode);
    CHECK(tsf_meta_swap(&a.s, &sw.s) == TSF_OK && violations(sw.s) == 0);
    CHECK(tsf_meta_swap(&sw.s, &sw2.s) == TSF_OK && violations(sw2.s) == 0);
    // merge with itself along p (when the result fits)
    if (m * 2 * p <= 64 && n * 2 * p <= 64) {
        Owned mg(m, n, 2 * p, 2 * r0, mode);
        CHECK(tsf_meta_merge(&a.s, &a.s, 2, &mg.s) == TSF_OK && violations(mg.s) == 0);
    }
    // product with the (1,1,2) standard scheme (when it fits)
    if (m * 2 * p <= 64 && n * 2 * p <= 64) {
        Owned t(1, 1, 2, 2, mode), pd(m, n, 2 * p, 2 * r0, mode);
        CHECK(tsf_init_scheme(1, 1, 2, mode, &t.s) == TSF_OK);
        CHECK(tsf_meta_product(&a.s, &t.s, &pd.s) == TSF_OK && violations(pd.s) == 0);
    }
    // a broken coefficient is counted, an entry outside the set refused
    if (mode == TSF_TERNARY) {
        a.W[0] = (int8_t)(a.W[0] == 0 ? 1 : 0);
        CHECK(violations(a.s) > 0);
        a.W[0] = 2;
        int64_t nv = 0;
        CHECK(tsf_verify(&a.s, &nv) == TSF_E_NOT_TERNARY);
    }
}

void error_paths()
{
    int64_t nv = 0;
    int32_t red = 0;
    CHECK(tsf_verify(nullptr, &nv) == TSF_E_ARG);
    CHECK(tsf_reduce(nullptr, &red) == TSF_E_ARG);
    Owned small(3, 3, 3, 20, TSF_TERNARY);
    CHECK(tsf_init_scheme(3, 3, 3, TSF_TERNARY, &small.s) == TSF_E_CAPACITY);
    CHECK(tsf_init_scheme(0, 3, 3, TSF_TERNARY, &small.s) == TSF_E_FORMAT);
    CHECK(tsf_init_scheme(9, 8, 1, TSF_TERNARY, &small.s) == TSF_E_FORMAT);
    CHECK(tsf_pack(nullptr, nullptr) == TSF_E_ARG);
    uint64_t bad[6] = {0x3, 0x4, 0x1, 0, 0x1, 0};  // a sign outside the digits
    tsf_dims d{1, 2, 1, 1, 1, TSF_TERNARY};
    Owned one(1, 2, 1, 1, TSF_TERNARY);
    CHECK(tsf_unpack(bad, &d, &one.s) == TSF_E_NOT_TERNARY);
    CHECK(tsf_last_error() != nullptr);
}

}  // namespace

int main()
{
    const int fmts[][3] = {{1, 1, 1}, {2, 2, 2}, {2, 2, 3}, {2, 3, 4}, {3, 3, 3},
                           {3, 4, 5}, {4, 4, 4}, {4, 5, 12}, {6, 7, 9}};
    for (const auto &f : fmts)
        for (int mode : {TSF_TERNARY, TSF_Z2}) one_format(f[0], f[1], f[2], mode);
    error_paths();
    if (failures) {
        std::fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    std::printf("host driver ok\n");
    return 0;
}
