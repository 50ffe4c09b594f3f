// Counter-based random stream for the GPU path: Philox4x32-10 (Salmon, Moraes, Dror, Shaw,
// "Parallel random numbers: as easy as 1, 2, 3", SC'11). Every draw is a pure function of
// (seed, x, individual, generation, purpose), so any kernel can recompute any draw and no
// generator state is stored or carried between launches.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hpm {

enum : uint32_t { TAG_INIT = 0, TAG_SEL = 1, TAG_XOV = 2, TAG_MUT = 3 };
constexpr uint32_t GATE_X = 0xFFFFFFFFu;  // counter word x reserved for the crossover gate

struct u32x4 {
    uint32_t a, b, c, d;
};

__device__ __forceinline__ u32x4 philox(uint64_t seed, uint32_t x, uint32_t ind, uint32_t gen,
                                        uint32_t tag)
{
    uint32_t c0 = x, c1 = ind, c2 = gen, c3 = tag;
    uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
        const uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
        const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return {c0, c1, c2, c3};
}

// index in [0, k) from a 32-bit draw: (r * k) >> 32
__host__ __device__ __forceinline__ uint32_t pick(uint32_t r, uint32_t k)
{
    return (uint32_t)(((uint64_t)r * (uint64_t)k) >> 32);
}

// Bernoulli(p) as an integer comparison r < threshold, threshold = floor(p 2^32) (2^32 if p >= 1)
inline uint64_t bernoulli_threshold(double p)
{
    if (p >= 1.0) return (uint64_t)1 << 32;
    if (p <= 0.0) return 0;
    double t = p * 4294967296.0;  // exact scaling by a power of two
    uint64_t f = (uint64_t)t;     // truncation = floor for t >= 0
    return f;
}

}  // namespace hpm
