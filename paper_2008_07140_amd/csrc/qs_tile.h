// Device-side description of a tile sweep (see qs_fused.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "qs_internal.h"

namespace qs {

// Tile t covers the amplitudes base(t) | (offsets over the tile qubits), where
// base(t) deposits the bits of t on the qubits outside the tile (ascending).
struct TileArgs {
    int m;               // tile qubits (10..13)
    int nops;
    int nouter;          // n - m
    int order;           // tile order of the sweep, 0 .. 3 (tile_base)
    uint64_t omask;      // qubits outside the tile
    uint8_t q[16];       // global position of local bit b (b < m)
};

struct TileOpDev {
    int kind;            // 0 = dense block, 1 = phase
    int k;               // dense: 4 or 5 qubits; phase: number of tile bits (0..3)
    int no;              // number of outer selector bits (0..5)
    uint32_t data_off;   // offset of fragments / table in the data buffer, 16-byte units
    int lpos[6];         // tile-local bit positions, [0] = most significant
    int opos[5];         // global positions of the outer bits, [0] = most significant
    uint32_t skip;       // dense: bit p set = identity for outer pattern p
    uint32_t frag_stride;  // dense: 16-byte units per outer pattern
    uint32_t colmask;    // dense: the 4 tile bits that index the 16 columns of a matrix-core tile
    uint32_t offs_off;   // dense: per-lane LDS byte offsets (tile_lane_offsets), 16-byte units
    uint32_t cimg[6];    // dense: LDS byte offsets of the column-tile index bits (lowest first)
};

// LDS layout of a tile: amplitude j (j < 2^13) lives in 8-byte slot
// j ^ g(j >> 5), where g XORs a fixed 5-bit image for each set bit among
// tile bits 5..12 (a bijection: bits 5.. are kept).  LDS banks see slot mod
// 32 for a 32-lane 8-byte read and slot mod 16 for a 16-lane 8-byte write,
// so tile bit p lands on bank vector image(p) (e_p for p < 5).  The images of
// bits 5..12 were searched so that almost every 4- or 5-qubit op has four
// column bits whose images are independent mod 16 and a lane qubit that
// completes them to rank 5: its reads and writes are then conflict-free.
constexpr uint32_t kTileSwizzleImage[8] = {11, 31, 31, 21, 14, 28, 3, 28};

__host__ __device__ inline uint32_t tile_swizzle(uint32_t j)
{
    uint32_t x = 0;
#pragma unroll
    for (int b = 0; b < 8; ++b)
        if ((j >> (5 + b)) & 1u) x ^= kTileSwizzleImage[b];
    return j ^ x;
}

// Per-lane LDS byte offsets of a dense k-qubit tile op (k = 4, 5; D = 2^k,
// MT = 2D / 16 row tiles, KS = 2D / 32 k-steps) relative to the column tile:
// lane l reads amplitudes 16 s + 4 (l / 16) + jj (s < KS, jj < 4) and writes
// amplitudes 8 mt + 2 (l / 16) + jj (mt < MT, jj < 2) of the group whose
// column bits (colmask) hold l % 16.  Stored lane by lane: KS * 4 read
// offsets, then MT * 2 write offsets, as uint32.
constexpr int tile_lane_offsets(int k) { return (2 << k) / 32 * 4 + (2 << k) / 16 * 2; }

// Batched sweeps: one entry per workgroup.
struct TileTask {
    uint32_t arg;   // index into the TileArgsDev array
    uint32_t tile;  // tile index within that state
};

struct TileArgsDev {
    float2 *amp;
    uint32_t op_off;  // first op of this state's sweep in the op array
    uint32_t slot;    // trajectory slot whose activity flag gates the sweep (device-sampled passes)
    TileArgs ta;
};

// k5: the op list holds 5-qubit blocks (selects the kernel configuration).
hipError_t launch_tile(void *amp, int n, const TileArgs &ta, const TileOpDev *dev_ops,
                       const void *dev_data, bool k5, hipStream_t st);
// active: NULL, or one flag per trajectory slot; workgroups of a slot whose
// flag is 0 return at once (the state is left as it is).
hipError_t launch_tile_multi(int m, uint32_t ntasks, const TileTask *tasks, const TileArgsDev *args,
                             const TileOpDev *dev_ops, const void *dev_data, bool k5, const int *active,
                             hipStream_t st);

}  // namespace qs
