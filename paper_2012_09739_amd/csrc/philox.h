// Philox4x32-10 counter-based generator, device side.
//
// The method needs i.i.d. uniforms U_n shared by the exact and the approximate inverse
// CDF (Section 3, coupling of exact and approximate variables); the generator itself is
// not fixed by the paper.  This is Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11):
// ten rounds of two 32x32->64 products with fixed odd multipliers, high halves xor-ed
// into the other two counter words and the round key, key bumped by Weyl constants.
//
// Counter layout used by every kernel of this library: key = (seed lo32, seed hi32) and
//   levels >= 2: counter = (n >> 2, path, (stream << 16) | level, pset), fine step n of a
//                path consumes output word (n & 3);
//   levels 0, 1: the S = 2^level < 4 steps of G = 4 / S consecutive paths share one call,
//                counter = (0, path / G, (stream << 16) | level, pset), step n of path p
//                consuming word (p mod G) S + n,
// so that no word is drawn and left unused.  The words depend only on (seed, stream, level,
// pset, path, n), never on the launch shape, so any tuning leaves the samples unchanged.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mlmc {

struct Words4 {
    uint32_t w[4];
};

// Three-input xor.  Rounds whose inputs are still wave-uniform (the counter words other
// than the path index are the same for every lane) are left to the compiler, which keeps
// them on the scalar unit; later rounds use the single-instruction 3-input bitwise op of
// gfx950 (truth table 0x96 = a ^ b ^ c).
template <bool kVector>
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
    if constexpr (kVector) return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
    else return a ^ b ^ c;
}

// kScalarRounds: leading rounds that may still run on uniform values (3 when only the path
// word varies across lanes, 0 when the caller's counters vary per lane anyway).
template <int kScalarRounds = 3>
__device__ __forceinline__ Words4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                                uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = r < kScalarRounds ? xor3<false>((uint32_t)(p1 >> 32), c1, k0)
                                              : xor3<true>((uint32_t)(p1 >> 32), c1, k0);
        const uint32_t n2 = r < kScalarRounds ? xor3<false>((uint32_t)(p0 >> 32), c3, k1)
                                              : xor3<true>((uint32_t)(p0 >> 32), c3, k1);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    Words4 out;
    out.w[0] = c0;
    out.w[1] = c1;
    out.w[2] = c2;
    out.w[3] = c3;
    return out;
}

}  // namespace mlmc
