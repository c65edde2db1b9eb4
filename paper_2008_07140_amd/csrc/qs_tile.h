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
    int pad;
    uint64_t slot[16];   // global offset of local index 512 r (the r-th 16-byte slot of a thread)
    uint64_t omask;      // qubits outside the tile
    uint16_t qlo[10];    // global positions of local bits 0..9
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
};

// Batched sweeps: one entry per workgroup.
struct TileTask {
    uint32_t arg;   // index into the TileArgsDev array
    uint32_t tile;  // tile index within that state
};

struct TileArgsDev {
    float2 *amp;
    uint32_t op_off;  // first op of this state's sweep in the op array
    uint32_t pad;
    TileArgs ta;
};

hipError_t launch_tile(void *amp, int n, const TileArgs &ta, const TileOpDev *dev_ops,
                       const void *dev_data, hipStream_t st);
hipError_t launch_tile_multi(int m, uint32_t ntasks, const TileTask *tasks, const TileArgsDev *args,
                             const TileOpDev *dev_ops, const void *dev_data, hipStream_t st);

}  // namespace qs
