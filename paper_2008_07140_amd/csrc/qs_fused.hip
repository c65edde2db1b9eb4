// Tile sweep kernel for complex64 states on gfx950.
//
// One workgroup holds a tile of 2^m amplitudes in LDS: the amplitudes whose
// index differs only in the tile qubits Q (ascending, Q[b] = b for b < L, so
// a tile is 2^(m-L) contiguous runs of 2^L amplitudes).  The other n - m bits
// select the tile.  After the tile is loaded, a list of ops is applied to it
// in LDS, then the tile is written back: one HBM read and one write of the
// state for the whole list.
//
// Ops:
//  - DENSE: a fused 2^k x 2^k complex block (k = 4 or 5) on k tile qubits,
//    applied to the 2^(m-k) groups of the tile as a real GEMM on the matrix
//    cores: with re/im interleaved, Y = A X where A is the 2^(k+1)-square real
//    form [[Re U, -Im U], [Im U, Re U]] (entry by entry) and X holds one group
//    per column.  Both operands are split as hi + lo bfloat16 values and three
//    v_mfma_f32_16x16x32_bf16 products (hi*hi + hi*lo + lo*hi) are accumulated
//    in FP32, which keeps about 16 significant bits per product.
//  - PHASE: a diagonal factor chosen by up to 3 tile bits and up to 3 bits
//    outside the tile (constant per tile), e.g. a CZ between a tile qubit and
//    an outer qubit.
// Ops may carry a condition: a set of outer qubits that must all be 1 (a gate
// controlled from outside the tile), evaluated once per tile.
#include <hip/hip_runtime.h>

#include "qs_internal.h"
#include "qs_tile.h"

namespace qs {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float vf4 __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;

__device__ __forceinline__ uint32_t insert_zero_bits(uint32_t t, const int *pos, int np)
{
    for (int b = 0; b < np; ++b) {
        const uint32_t lo = t & ((1u << pos[b]) - 1u);
        t = ((t ^ lo) << 1) | lo;
    }
    return t;
}

constexpr int kMaxM = 13;

// local tile index j -> global index bits (without the tile base)
__device__ __forceinline__ uint64_t scatter_local(uint32_t j, const TileArgs &ta)
{
    uint64_t g = j & ((1u << ta.L) - 1u);
#pragma unroll
    for (int b = 1; b < kMaxM; ++b)
        if (b >= ta.L && b < ta.m && ((j >> b) & 1u)) g |= uint64_t(1) << ta.Q[b];
    return g;
}

template <int K>
__device__ void dense_op(float2 *tile, const TileOpDev &op, const uint4 *data, int m, int outer)
{
    constexpr int D = 1 << K;
    constexpr int MT = 2 * D / 16;  // row tiles of the real form
    constexpr int KS = 2 * D / 32;  // K steps of the real form
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const bf16x8 *fr =
        reinterpret_cast<const bf16x8 *>(data + op.data_off + uint32_t(outer) * op.frag_stride);
    bf16x8 ahi[MT][KS], alo[MT][KS];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            ahi[mt][s] = fr[(mt * KS + s) * 64 + lane];
            alo[mt][s] = fr[MT * KS * 64 + (mt * KS + s) * 64 + lane];
        }
    // block qubit positions in the tile, op.lpos[0] = most significant
    int srt[K];
#pragma unroll
    for (int b = 0; b < K; ++b) srt[b] = op.lpos[b];
#pragma unroll
    for (int i = 1; i < K; ++i)
#pragma unroll
        for (int j = K - 1; j >= i; --j)
            if (srt[j - 1] > srt[j]) {
                const int t = srt[j];
                srt[j] = srt[j - 1];
                srt[j - 1] = t;
            }
    auto offset = [&](int x) {
        uint32_t o = 0;
#pragma unroll
        for (int b = 0; b < K; ++b)
            if ((x >> (K - 1 - b)) & 1) o |= 1u << op.lpos[b];
        return o;
    };
    uint32_t roff[KS][4], woff[MT][2];
#pragma unroll
    for (int s = 0; s < KS; ++s)
#pragma unroll
        for (int j = 0; j < 4; ++j) roff[s][j] = offset(16 * s + 4 * (lane >> 4) + j);
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int j = 0; j < 2; ++j) woff[mt][j] = offset(8 * mt + 2 * (lane >> 4) + j);
    const int ntiles = 1 << (m - K - 4);  // 16 groups per column tile
    for (int nt = wave; nt < ntiles; nt += kThreads / 64) {
        const uint32_t g = uint32_t(nt) * 16 + (lane & 15);
        const uint32_t gb = insert_zero_bits(g, srt, K);
        bf16x8 bhi[KS], blo[KS];
#pragma unroll
        for (int s = 0; s < KS; ++s)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const float2 v = tile[gb | roff[s][j]];
                const __bf16 hr = __bf16(v.x), hi = __bf16(v.y);
                bhi[s][2 * j] = hr;
                bhi[s][2 * j + 1] = hi;
                blo[s][2 * j] = __bf16(v.x - float(hr));
                blo[s][2 * j + 1] = __bf16(v.y - float(hi));
            }
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int s = 0; s < KS; ++s) {
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi[mt][s], bhi[s], acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi[mt][s], blo[s], acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo[mt][s], bhi[s], acc, 0, 0, 0);
            }
            tile[gb | woff[mt][0]] = make_float2(acc[0], acc[1]);
            tile[gb | woff[mt][1]] = make_float2(acc[2], acc[3]);
        }
    }
}

__device__ void phase_op(float2 *tile, float2 *ptab, const TileOpDev &op, const uint4 *data,
                         int outer, int m)
{
    const float2 *tab = reinterpret_cast<const float2 *>(data + op.data_off);
    const int D = 1 << op.k;
    if (int(threadIdx.x) < D) ptab[threadIdx.x] = tab[(outer << op.k) | threadIdx.x];
    __syncthreads();
    int active = 0;
    for (int x = 0; x < D; ++x)
        if (!(ptab[x].x == 1.f && ptab[x].y == 0.f)) active |= 1 << x;
    if (!active) return;
    int lp[3], sh[3];
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        lp[b] = b < op.k ? op.lpos[b] : 0;
        sh[b] = b < op.k ? op.k - 1 - b : 0;
    }
    const uint32_t n_amp = 1u << m;
    for (uint32_t j = threadIdx.x; j < n_amp; j += kThreads) {
        int x = 0;
#pragma unroll
        for (int b = 0; b < 3; ++b)
            if (b < op.k) x |= int((j >> lp[b]) & 1) << sh[b];
        if ((active >> x) & 1) {
            const float2 f = ptab[x];
            const float2 v = tile[j];
            tile[j] = make_float2(f.x * v.x - f.y * v.y, f.x * v.y + f.y * v.x);
        }
    }
}

__global__ __launch_bounds__(kThreads) void k_tile(float2 *amp, uint64_t ntiles, TileArgs ta,
                                                   const TileOpDev *ops, const uint4 *data)
{
    extern __shared__ float2 lds[];
    float2 *tile = lds;
    float2 *ptab = lds + (size_t(1) << ta.m);
    const uint32_t n_amp = 1u << ta.m;
    const int per = int(n_amp / (2 * kThreads));  // float4 (2 amplitudes) per thread
    // global offset of this thread's first amplitude pair within a tile; the
    // pair r adds the (uniform) offset of local index 512 r
    const uint64_t toff = scatter_local(2u * threadIdx.x, ta);
    for (uint64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        // tile base: insert a zero at every tile qubit
        uint64_t base = t;
#pragma unroll
        for (int b = 0; b < kMaxM; ++b)
            if (b < ta.m) {
                const uint64_t lo = base & ((uint64_t(1) << ta.Q[b]) - 1);
                base = ((base ^ lo) << 1) | lo;
            }
        // ---- load (non-temporal: every amplitude is read once per sweep)
        constexpr int kMaxPer = 16;
        vf4 buf[kMaxPer];
#pragma unroll
        for (int r = 0; r < kMaxPer; ++r)
            if (r < per) {
                const uint64_t gi = base | toff | scatter_local(uint32_t(r) * 2u * kThreads, ta);
                buf[r] = __builtin_nontemporal_load(reinterpret_cast<const vf4 *>(amp + gi));
            }
#pragma unroll
        for (int r = 0; r < kMaxPer; ++r)
            if (r < per) {
                const uint32_t j = 2u * (threadIdx.x + uint32_t(r) * kThreads);
                *reinterpret_cast<vf4 *>(tile + j) = buf[r];
            }
        __syncthreads();
        // ---- ops
        for (int oi = 0; oi < ta.nops; ++oi) {
            const TileOpDev op = ops[oi];
            int outer = 0;
#pragma unroll
            for (int b = 0; b < 3; ++b)
                if (b < op.no) outer = (outer << 1) | int((base >> op.opos[b]) & 1);
            if (op.kind == 0) {
                if ((op.skip >> outer) & 1u) continue;  // identity on this tile
                if (op.k == 4)
                    dense_op<4>(tile, op, data, ta.m, outer);
                else
                    dense_op<5>(tile, op, data, ta.m, outer);
            } else {
                phase_op(tile, ptab, op, data, outer, ta.m);
            }
            __syncthreads();
        }
        // ---- store
#pragma unroll
        for (int r = 0; r < kMaxPer; ++r)
            if (r < per) {
                const uint32_t j = 2u * (threadIdx.x + uint32_t(r) * kThreads);
                buf[r] = *reinterpret_cast<const vf4 *>(tile + j);
            }
#pragma unroll
        for (int r = 0; r < kMaxPer; ++r)
            if (r < per) {
                const uint64_t gi = base | toff | scatter_local(uint32_t(r) * 2u * kThreads, ta);
                __builtin_nontemporal_store(buf[r], reinterpret_cast<vf4 *>(amp + gi));
            }
        __syncthreads();
    }
}

}  // namespace

size_t tile_lds_bytes(int m) { return (size_t(8) << m) + 64 * sizeof(float2); }

hipError_t launch_tile(void *amp, int n, const TileArgs &ta, const TileOpDev *dev_ops,
                       const void *dev_data, hipStream_t st)
{
    if (ta.m < 9 || ta.m > 13 || ta.L < 1 || ta.L > ta.m || ta.m > n) return hipErrorInvalidValue;
    const size_t lds = tile_lds_bytes(ta.m);
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void *)k_tile, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           int(tile_lds_bytes(13)));
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    const uint64_t ntiles = uint64_t(1) << (n - ta.m);
    const uint64_t grid = ntiles < (uint64_t(1) << 20) ? ntiles : (uint64_t(1) << 20);
    hipLaunchKernelGGL(k_tile, dim3(unsigned(grid)), dim3(kThreads), lds, st, (float2 *)amp, ntiles, ta,
                       dev_ops, (const uint4 *)dev_data);
    return hipGetLastError();
}

}  // namespace qs
