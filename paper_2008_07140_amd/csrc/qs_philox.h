// Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw,
// "Parallel random numbers: as easy as 1, 2, 3", SC'11), usable on host and
// device.  Ten rounds of two 32x32->64 multiplications with a Weyl key bump.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace qs {

struct Philox4 {
    uint32_t w[4];
};

__host__ __device__ inline Philox4 philox4x32_10(Philox4 ctr, uint32_t k0, uint32_t k1)
{
    constexpr uint32_t kMul0 = 0xD2511F53u, kMul1 = 0xCD9E8D57u;
    constexpr uint32_t kWeyl0 = 0x9E3779B9u, kWeyl1 = 0xBB67AE85u;
    for (int round = 0; round < 10; ++round) {
        const uint64_t p0 = uint64_t(kMul0) * ctr.w[0];
        const uint64_t p1 = uint64_t(kMul1) * ctr.w[2];
        Philox4 nx;
        nx.w[0] = uint32_t(p1 >> 32) ^ ctr.w[1] ^ k0;
        nx.w[1] = uint32_t(p1);
        nx.w[2] = uint32_t(p0 >> 32) ^ ctr.w[3] ^ k1;
        nx.w[3] = uint32_t(p0);
        ctr = nx;
        k0 += kWeyl0;
        k1 += kWeyl1;
    }
    return ctr;
}

// Uniform in [0, 1) for (seed, trajectory, site): counter = (site lo, site hi,
// traj lo, traj hi), key = (seed lo, seed hi), 53 high bits of words 1:0.
__host__ __device__ inline double noise_uniform(uint64_t seed, uint64_t traj, uint64_t site)
{
    Philox4 c;
    c.w[0] = uint32_t(site);
    c.w[1] = uint32_t(site >> 32);
    c.w[2] = uint32_t(traj);
    c.w[3] = uint32_t(traj >> 32);
    const Philox4 r = philox4x32_10(c, uint32_t(seed), uint32_t(seed >> 32));
    const uint64_t x = (uint64_t(r.w[1]) << 32) | r.w[0];
    return double(x >> 11) * 0x1.0p-53;
}

}  // namespace qs
