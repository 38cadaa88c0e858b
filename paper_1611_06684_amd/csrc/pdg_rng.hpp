// Counter-based random numbers for the sweep kernels: Philox4x32 with 10
// rounds (Salmon, Moraes, Dror, Shaw, "Parallel Random Numbers: As Easy as
// 1, 2, 3", SC'11).  The key is the sampler seed and is the same for every
// lane of a launch, so its schedule stays in scalar registers.
//
// Counter of one call: (id_lo, id_hi, phase << 30 | sub, sweep).  One call
// gives five 24-bit integers: the top 24 bits of each output word and a fifth
// made of the low bytes of words 0, 1 and 2 (high to low).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pdg {

constexpr uint32_t kPhaseInit = 0u;
constexpr uint32_t kPhaseDual = 1u;
constexpr uint32_t kPhasePrimal = 2u;

struct Words {
    uint32_t w0, w1, w2, w3;
};

__device__ __forceinline__ Words philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2,
                                               uint32_t c3, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        // three-input xor in one v_bitop3_b32 (truth table 0x96)
        const uint32_t n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c1, k0, 0x96);
        const uint32_t n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c3, k1, 0x96);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return {c0, c1, c2, c3};
}

// Round keys of a launch: round r uses (k0 + r W0, k1 + r W1).  Computed once
// on the host and passed in kernel arguments, so no lane recomputes them.
struct RoundKeys {
    uint32_t k0[10], k1[10];
};

__host__ inline RoundKeys make_round_keys(uint64_t seed)
{
    RoundKeys rk;
    uint32_t a = (uint32_t)seed, b = (uint32_t)(seed >> 32);
    for (int r = 0; r < 10; ++r) {
        rk.k0[r] = a;
        rk.k1[r] = b;
        a += 0x9E3779B9u;
        b += 0xBB67AE85u;
    }
    return rk;
}

// Same generator with the round keys supplied.
__device__ __forceinline__ Words philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2,
                                               uint32_t c3, const RoundKeys &rk)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        const uint32_t n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c1, rk.k0[r], 0x96);
        const uint32_t n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c3, rk.k1[r], 0x96);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
    }
    return {c0, c1, c2, c3};
}

// The fifth 24-bit integer of a call.
__device__ __forceinline__ uint32_t fifth_u24(const Words &w)
{
    return ((w.w0 & 0xFFu) << 16) | ((w.w1 & 0xFFu) << 8) | (w.w2 & 0xFFu);
}

// The fifth 24-bit integer in the top bits of a word, as the dual compares it:
// bytes (high to low) w0.b0, w1.b0, w2.b0, 0, assembled by two byte
// permutes (selector 0..3: bytes of the second operand, 4..7: of the first,
// 12: zero).
__device__ __forceinline__ uint32_t fifth_w(const Words &w)
{
    const uint32_t t = __builtin_amdgcn_perm(w.w1, w.w2, 0x0C04000Cu);  // 0, w1.b0, w2.b0, 0
    return __builtin_amdgcn_perm(w.w0, t, 0x0402010Cu);                 // w0.b0, t.b2, t.b1, 0
}

// Word j (0..3) of a call, j runtime.
__device__ __forceinline__ uint32_t word_at(const Words &w, int j)
{
    uint32_t lo = (j & 1) ? w.w1 : w.w0;
    uint32_t hi = (j & 1) ? w.w3 : w.w2;
    return (j & 2) ? hi : lo;
}

}  // namespace pdg
