// Test shim: exposes the library's one-bit ternary arithmetic (tsf_bits.h)
// so the CPU tests can check it exhaustively against integer arithmetic.
#include "../paper_2511_20317_amd/csrc/tsf_bits.h"

extern "C" int shim_add(uint64_t da, uint64_t sa, uint64_t db, uint64_t sb, uint64_t *d,
                        uint64_t *s)
{
    return tern_add(da, sa, db, sb, *d, *s);
}
extern "C" int shim_sub(uint64_t da, uint64_t sa, uint64_t db, uint64_t sb, uint64_t *d,
                        uint64_t *s)
{
    return tern_sub(da, sa, db, sb, *d, *s);
}
extern "C" int shim_neg_eq(uint64_t da, uint64_t sa, uint64_t db, uint64_t sb)
{
    return tern_neg_eq(da, sa, db, sb);
}
extern "C" void shim_philox(uint64_t seed, int64_t t, uint32_t a, uint32_t dom, uint32_t *out)
{
    Philox4 p = walk_block(seed, t, a, dom);
    for (int k = 0; k < 4; ++k) out[k] = p.x[k];
}
