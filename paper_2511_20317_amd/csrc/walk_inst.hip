// walk_inst.hip -- one translation unit of walk-kernel instantiations.  It is
// compiled once per (word width, coefficient set) with TSFK_WIDE (0: 32-bit
// masks, 1: 64-bit masks) and TSFK_Z2 (0: ternary, 1: Z2) defined, so the
// builds of the four groups run in parallel.
#include "walk_kernel.h"

#ifndef TSFK_WIDE
#error "TSFK_WIDE must be defined"
#endif
#ifndef TSFK_Z2
#error "TSFK_Z2 must be defined"
#endif

namespace tsfk {

using Word = std::conditional_t<TSFK_WIDE != 0, uint64_t, uint32_t>;
constexpr bool kZ2 = TSFK_Z2 != 0;

// a walk kernel, or its checked variant (tsf_walk_checked), which exists for
// the default launch shapes only: 8 lanes per walk for the attempt-parallel
// strategies, 64 for the term-parallel one
template <int G, int S, bool AP, bool IX, bool PK = false>
KernelFn kern(bool chk)
{
    if constexpr ((G == 8 && AP) || (G == 64 && !AP)) {
        if (chk) return walk_kernel_checked<G, S, Word, kZ2, AP, IX, PK>;
    }
    if (chk) return nullptr;
    return walk_kernel<G, S, Word, kZ2, AP, IX, PK>;
}

// term-parallel kernels: S = term slots per lane (with 64 lanes per walk
// also 5, 6 and 7, so that large schemes are not rounded up to 8 slots)
template <int G>
KernelFn pick_s(int s, bool chk)
{
    switch (s) {
    case 1: return kern<G, 1, false, false>(chk);
    case 2: return kern<G, 2, false, false>(chk);
    case 4: return kern<G, 4, false, false>(chk);
    case 8: return kern<G, 8, false, false>(chk);
    default: break;
    }
    if constexpr (G == 64) {
        switch (s) {
        case 5: return kern<G, 5, false, false>(chk);
        case 6: return kern<G, 6, false, false>(chk);
        case 7: return kern<G, 7, false, false>(chk);
        default: break;
        }
    }
    return nullptr;
}

// attempt-parallel kernels: indexed (at most 64 terms; pk: factors of at
// most 16 entries packed in one 32-bit LDS word), or plain with partner sets
// of s = 1 or 2 words (at most 64 or 128 terms)
template <int G>
KernelFn pick_ap(bool ix, int s, bool pk, bool chk)
{
    if (ix) {
        if (s != 1) return nullptr;
        if constexpr (TSFK_WIDE == 0)
            if (pk) return kern<G, 1, true, true, true>(chk);
        return pk ? nullptr : kern<G, 1, true, true>(chk);
    }
    if (pk) return nullptr;
    switch (s) {
    case 1: return kern<G, 1, true, false>(chk);
    case 2: return kern<G, 2, true, false>(chk);
    default: return nullptr;
    }
}

#define TSF_CAT2(a, b, c) pick_kernel_w##a##_z##b##c
#define TSF_CAT(a, b) TSF_CAT2(a, b, )
// strategy: 1 attempt-parallel, 2 term-parallel, 3 indexed attempt-parallel,
// 4 indexed attempt-parallel with packed factors; chk: the checked variant
KernelFn TSF_CAT(TSFK_WIDE, TSFK_Z2)(int g, int s, int strategy, bool chk)
{
    if (strategy == 1 || strategy == 3 || strategy == 4) {
        const bool ix = strategy >= 3, pk = strategy == 4;
        switch (g) {
        case 4: return pick_ap<4>(ix, s, pk, chk);
        case 8: return pick_ap<8>(ix, s, pk, chk);
        case 16: return pick_ap<16>(ix, s, pk, chk);
        case 32: return pick_ap<32>(ix, s, pk, chk);
        default: return nullptr;
        }
    }
    switch (g) {
    case 8: return pick_s<8>(s, chk);
    case 16: return pick_s<16>(s, chk);
    case 32: return pick_s<32>(s, chk);
    case 64: return pick_s<64>(s, chk);
    default: return nullptr;
    }
}

}  // namespace tsfk
