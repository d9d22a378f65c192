// rng.hpp -- counter-based random numbers for error sampling, pruning
// selection and shot sampling.
//
// Philox4x32 with 10 rounds (Salmon, Moraes, Dror, Shaw, SC'11): each round
// multiplies counter words 0 and 2 by two fixed 32-bit constants, mixes the
// high halves with words 1 and 3 and the key, and the key advances by two
// Weyl increments between rounds.  Usable from host and device code.
#pragma once

#include <cstdint>

#if defined(__HIPCC__)
#define TUSQ_HD __host__ __device__ inline
#define TUSQ_UNROLL _Pragma("unroll")
#else
#define TUSQ_HD inline
#define TUSQ_UNROLL
#endif

namespace tusq {

struct U4 {
    uint32_t x, y, z, w;
};

TUSQ_HD U4 philox10(U4 c, uint32_t k0, uint32_t k1) {
    constexpr uint32_t MA = 0xD2511F53u, MB = 0xCD9E8D57u;
    constexpr uint32_t WA = 0x9E3779B9u, WB = 0xBB67AE85u;
    TUSQ_UNROLL
    for (int round = 0; round < 10; ++round) {
        const uint64_t pa = static_cast<uint64_t>(MA) * c.x;
        const uint64_t pb = static_cast<uint64_t>(MB) * c.z;
        U4 d;
        d.x = static_cast<uint32_t>(pb >> 32) ^ c.y ^ k0;
        d.y = static_cast<uint32_t>(pb);
        d.z = static_cast<uint32_t>(pa >> 32) ^ c.w ^ k1;
        d.w = static_cast<uint32_t>(pa);
        c = d;
        k0 += WA;
        k1 += WB;
    }
    return c;
}

// The two 64-bit values of one Philox block.  Counter layout used by the
// whole engine: (sub-index, primary index, aux, stream); the key is the job
// seed.  Streams: 0 error sampling, 1 pruning selection, 2 shot sampling,
// 3 measurement outcomes.
struct Pair64 {
    uint64_t lo, hi;
};

TUSQ_HD Pair64 philox_pair(uint64_t seed, uint32_t sub, uint32_t primary, uint32_t aux,
                           uint32_t stream) {
    const U4 r = philox10(U4{sub, primary, aux, stream}, static_cast<uint32_t>(seed),
                          static_cast<uint32_t>(seed >> 32));
    return Pair64{(static_cast<uint64_t>(r.y) << 32) | r.x, (static_cast<uint64_t>(r.w) << 32) | r.z};
}

enum : uint32_t { STREAM_ERRORS = 0, STREAM_PRUNE = 1, STREAM_SHOTS = 2, STREAM_OUTCOMES = 3 };

}  // namespace tusq
