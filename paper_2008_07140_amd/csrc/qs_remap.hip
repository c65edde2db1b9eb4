// Pack / unpack of the qubit-remap exchange of a sharded state.
//
// The paper divides the amplitudes of a state equally over its nodes (Sec.
// 2.1, the first level of its parallel scheme), so the top g qubits of an
// n-qubit state name the node that holds an amplitude; a gate on such a
// global qubit needs partner amplitudes from another node, which is where
// the paper loses most of its speed (Sec. 3.1, Fig. 4).  The remedy planned
// here is to swap the g global qubits with g local ones, lq[0..g-1], by one
// all-to-all: each shard of L = n - g local qubits is packed into 2^g chunks
// of 2^(L-g) amplitudes, chunk d holding the amplitudes whose local bits lq
// read d (bit i of d at qubit lq[i]), in ascending order of the other local
// bits; chunk d goes to the node whose global index is d, which unpacks the
// chunk from node r with lq reading r.  Afterwards local qubit lq[i] carries
// the former global qubit L + i and global qubit L + i the former lq[i].
//
// Both directions are one bit-permutation sweep that reads and writes every
// amplitude of the shard once (HBM-bound).  A lane moves 16 bytes: one
// complex128 amplitude, or two adjacent complex64 amplitudes when bit 0 is
// not among lq (they are then adjacent in the shard as well).  Consecutive
// lanes take consecutive elements of the side that is written (the buffer
// for pack, the shard for unpack), so stores fill whole lines and the reads
// gather runs of 2^min(lq) amplitudes; when bit 0 is among lq the lanes
// walk the shard in both directions: the buffer side then has two runs of
// 32 lanes instead of every other unit of the shard.
#include <hip/hip_runtime.h>

#include "qs_internal.h"

namespace qs {

namespace {

typedef double vd2 __attribute__((ext_vector_type(2)));
typedef float vf4 __attribute__((ext_vector_type(4)));
typedef float vf2 __attribute__((ext_vector_type(2)));

constexpr int kRemapBlock = 256;
constexpr int kRemapUnroll = 4;
constexpr uint64_t kRemapMaxBlocks = 1 << 20;

struct RemapArgs {
    int cbits;               // L - g: bits of the index inside a chunk
    int g;
    int zpos[QS_REMAP_MAX_G];  // lq ascending: zero bits inserted into the chunk index
    int dpos[QS_REMAP_MAX_G];  // lq in the caller's order: bit i of the chunk number
};

// shard index of element b of the packed buffer
__device__ __forceinline__ uint64_t remap_index(uint64_t b, const RemapArgs &ra)
{
    const uint64_t d = b >> ra.cbits;
    uint64_t x = b & ((uint64_t(1) << ra.cbits) - 1);
    for (int k = 0; k < ra.g; ++k) {
        const uint64_t lo = x & ((uint64_t(1) << ra.zpos[k]) - 1);
        x = ((x ^ lo) << 1) | lo;
    }
    for (int i = 0; i < ra.g; ++i) x |= ((d >> i) & 1) << ra.dpos[i];
    return x;
}

// buffer element of shard index s (the inverse of remap_index)
__device__ __forceinline__ uint64_t remap_inverse(uint64_t s, const RemapArgs &ra)
{
    uint64_t d = 0;
    for (int i = 0; i < ra.g; ++i) d |= ((s >> ra.dpos[i]) & 1) << i;
    uint64_t x = s;
    for (int k = ra.g - 1; k >= 0; --k) {
        const int p = ra.zpos[k];
        x = ((x >> (p + 1)) << p) | (x & ((uint64_t(1) << p) - 1));
    }
    return (d << ra.cbits) | x;
}

// U = 16-byte unit (two doubles / four floats) or one complex64 amplitude (bit 0 in lq);
// SHIFT = log2 of the amplitudes per unit.  PACK: buf[b] = shard[remap(b)];
// otherwise shard[remap(b)] = buf[b].  BYSHARD: lane index = shard unit,
// else buffer unit.
template <typename U, int SHIFT, bool PACK, bool BYSHARD>
__global__ __launch_bounds__(kRemapBlock) void k_remap(U *shard, U *buf, uint64_t nunits, RemapArgs ra)
{
    const uint64_t per = uint64_t(kRemapBlock) * kRemapUnroll;
    const uint64_t stride = uint64_t(gridDim.x) * per;
    for (uint64_t base = uint64_t(blockIdx.x) * per + threadIdx.x; base < nunits; base += stride) {
        U v[kRemapUnroll];
        uint64_t si[kRemapUnroll], bi[kRemapUnroll];
#pragma unroll
        for (int u = 0; u < kRemapUnroll; ++u) {
            const uint64_t t = base + uint64_t(u) * kRemapBlock;
            const uint64_t tc = t < nunits ? t : 0;
            si[u] = BYSHARD ? tc : remap_index(tc << SHIFT, ra) >> SHIFT;
            bi[u] = BYSHARD ? remap_inverse(tc << SHIFT, ra) >> SHIFT : tc;
            if (t < nunits) v[u] = __builtin_nontemporal_load(PACK ? shard + si[u] : buf + bi[u]);
        }
#pragma unroll
        for (int u = 0; u < kRemapUnroll; ++u) {
            const uint64_t t = base + uint64_t(u) * kRemapBlock;
            if (t < nunits) __builtin_nontemporal_store(v[u], PACK ? buf + bi[u] : shard + si[u]);
        }
    }
}

template <typename U, int SHIFT, bool PACK, bool BYSHARD>
void launch_remap_k(void *shard, void *buf, uint64_t nunits, uint64_t grid, const RemapArgs &ra, hipStream_t st)
{
    hipLaunchKernelGGL((k_remap<U, SHIFT, PACK, BYSHARD>), dim3(unsigned(grid)), dim3(kRemapBlock), 0, st,
                       (U *)shard, (U *)buf, nunits, ra);
}

template <typename U, int SHIFT>
hipError_t launch_remap_t(void *shard, void *buf, int L, const RemapArgs &ra, bool pack, bool bit0,
                          hipStream_t st)
{
    const uint64_t nunits = (uint64_t(1) << L) >> SHIFT;
    uint64_t grid = (nunits + kRemapBlock * kRemapUnroll - 1) / (kRemapBlock * kRemapUnroll);
    if (grid == 0) grid = 1;
    if (grid > kRemapMaxBlocks) grid = kRemapMaxBlocks;
    if (!pack)
        launch_remap_k<U, SHIFT, false, true>(shard, buf, nunits, grid, ra, st);
    else if (bit0)
        launch_remap_k<U, SHIFT, true, true>(shard, buf, nunits, grid, ra, st);
    else
        launch_remap_k<U, SHIFT, true, false>(shard, buf, nunits, grid, ra, st);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_remap(qs_dtype dt, void *shard, void *buf, int L, int g, const int *lq, bool pack,
                        hipStream_t st)
{
    RemapArgs ra{};
    ra.cbits = L - g;
    ra.g = g;
    bool bit0 = false;
    for (int i = 0; i < g; ++i) {
        ra.dpos[i] = lq[i];
        ra.zpos[i] = lq[i];
        bit0 |= lq[i] == 0;
    }
    // ascending order for the zero insertion
    for (int i = 1; i < g; ++i)
        for (int j = i; j > 0 && ra.zpos[j - 1] > ra.zpos[j]; --j) {
            const int t = ra.zpos[j];
            ra.zpos[j] = ra.zpos[j - 1];
            ra.zpos[j - 1] = t;
        }
    if (dt == QS_C128) return launch_remap_t<vd2, 0>(shard, buf, L, ra, pack, bit0, st);
    // pairs need bit 0 outside lq (then g < L and a chunk index has a bit 0)
    if (bit0 || L == 0) return launch_remap_t<vf2, 0>(shard, buf, L, ra, pack, bit0, st);
    return launch_remap_t<vf4, 1>(shard, buf, L, ra, pack, bit0, st);
}

}  // namespace qs
