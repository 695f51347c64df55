// Counter-based random numbers for the MD and resampling kernels:
// Philox-4x32-10 of Salmon, Moraes, Dror & Shaw (SC'11, "Parallel random
// numbers: as easy as 1, 2, 3") -- 4 x 32-bit counter, 2 x 32-bit key, ten
// rounds; each round multiplies words 0 and 2 by fixed odd constants and
// mixes the high halves with words 1 / 3 and the key, and the key advances by
// two Weyl increments between rounds.
//
// Draw layout (counter = slot, step, block, stream):
//   stream 0  Andersen collision test: atom a reads word floor(a/16) mod 4
//             of block (a mod 16) + 16 floor(a/64)
//   stream 1  collision velocity of atom a: block a, three normals
//   stream 2  resampling uniform of slot j: step word = temperature index
//   stream 3  initial Maxwell-Boltzmann velocity of atom a: block a
//   stream 4  multinomial resampling: uniform of draw k in the slot word,
//             step word = temperature index
//   stream 5  Langevin noise of atom a: block a, three normals per step
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pamd {

struct u32x4 {
    uint32_t v[4];
};

__host__ __device__ __forceinline__ u32x4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                                  uint32_t k0, uint32_t k1)
{
    constexpr uint32_t kMulA = 0xD2511F53u, kMulB = 0xCD9E8D57u;
    constexpr uint32_t kBumpA = 0x9E3779B9u, kBumpB = 0xBB67AE85u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t pa = (uint64_t)kMulA * c0;
        const uint64_t pb = (uint64_t)kMulB * c2;
        const uint32_t y0 = (uint32_t)(pb >> 32) ^ c1 ^ k0;
        const uint32_t y2 = (uint32_t)(pa >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)pb;
        c3 = (uint32_t)pa;
        c0 = y0;
        c2 = y2;
        k0 += kBumpA;
        k1 += kBumpB;
    }
    return u32x4{{c0, c1, c2, c3}};
}

enum : uint32_t {
    kStreamCollide = 0,
    kStreamVelocity = 1,
    kStreamResample = 2,
    kStreamInit = 3,
    kStreamMultinomial = 4,
    kStreamLangevin = 5
};

// 53-bit uniform in [0, 1) from two words
__host__ __device__ __forceinline__ double uniform53(uint32_t a, uint32_t b)
{
    return ((double)(a >> 5) * 67108864.0 + (double)(b >> 6)) * (1.0 / 9007199254740992.0);
}

}  // namespace pamd
