// Tile sweep kernel for complex64 states on gfx950.
//
// One workgroup holds a tile of 2^m amplitudes in LDS: the amplitudes whose
// index differs only in the tile qubits Q (ascending, Q[b] = b for the lowest
// few b, so a tile is a set of contiguous runs of at least 128 bytes).  The other n - m bits
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
//  - PHASE: a diagonal factor chosen by up to 3 tile bits.
// Every op may also depend on up to 5 bits outside the tile (constant over a
// tile): they select one of 2^no precomputed operators, which is how gates
// controlled from, or diagonal on, qubits outside the tile (a CZ or CU3 that
// crosses the tile boundary) stay inside fused blocks.
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

typedef float v2f __attribute__((ext_vector_type(2)));
typedef __bf16 v2bf __attribute__((ext_vector_type(2)));

// Split two floats into bfloat16 hi parts and the bfloat16 of the remainders
// (packed conversions; the remainder of each is exact in FP32).
__device__ __forceinline__ void split2(float a, float b, v2bf &hi, v2bf &lo)
{
    hi = __builtin_convertvector(v2f{a, b}, v2bf);
    lo = __builtin_convertvector(v2f{a - float(hi[0]), b - float(hi[1])}, v2bf);
}

// LDS layout of a tile: amplitude j lives at j ^ ((j >> 5) & 31).  Blocks on
// the low tile qubits make the 16 groups of a matrix-core operand differ
// only in high index bits; the XOR spreads those accesses over the banks.
__device__ __forceinline__ uint32_t sw(uint32_t j) { return j ^ ((j >> 5) & 31u); }

// Four-qubit blocks in real form: A is the 32 x 32 real matrix
// [[Re U, -Im U], [Im U, Re U]] (entry by entry, re/im interleaved); fragment
// (mt, 0) of lane l holds A[16 mt + l % 16][8 (l / 16) + j].  Each wave takes
// two column tiles at a time so that four accumulators interleave.
__device__ void dense_op4(float2 *tile, const TileOpDev &op, const uint4 *data, int m, int outer)
{
    constexpr int K = 4;
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
    const bf16x8 *fr =
        reinterpret_cast<const bf16x8 *>(data + op.data_off + uint32_t(outer) * op.frag_stride);
    bf16x8 ahi[2], alo[2];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
        ahi[mt] = fr[mt * 64 + lane];
        alo[mt] = fr[2 * 64 + mt * 64 + lane];
    }
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
    const uint32_t gl = insert_zero_bits(uint32_t(lane & 15), srt, K);
    uint32_t rd[4], wr[2][2];
#pragma unroll
    for (int j = 0; j < 4; ++j) rd[j] = sw(gl | offset(4 * (lane >> 4) + j)) * 8u;
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int j = 0; j < 2; ++j) wr[mt][j] = sw(gl | offset(8 * mt + 2 * (lane >> 4) + j)) * 8u;
    char *tb = reinterpret_cast<char *>(tile);
    const int ntiles = 1 << (m - K - 4);
    constexpr int kWaves = kThreads / 64;
    for (int nt0 = 2 * wave; nt0 < ntiles; nt0 += 2 * kWaves) {
        uint32_t gt[2];
        bf16x8 bhi[2], blo[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            gt[h] = sw(insert_zero_bits(uint32_t(nt0 + h) * 16u, srt, K)) * 8u;  // uniform
            float2 v[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) v[j] = *reinterpret_cast<const float2 *>(tb + (rd[j] ^ gt[h]));
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                v2bf hh, ll;
                split2(v[j].x, v[j].y, hh, ll);
                bhi[h][2 * j] = hh[0];
                bhi[h][2 * j + 1] = hh[1];
                blo[h][2 * j] = ll[0];
                blo[h][2 * j + 1] = ll[1];
            }
        }
        f32x4 acc[2][2];
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int mt = 0; mt < 2; ++mt) acc[h][mt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
            for (int h = 0; h < 2; ++h)
                acc[h][mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi[mt], bhi[h], acc[h][mt], 0, 0, 0);
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
            for (int h = 0; h < 2; ++h)
                acc[h][mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi[mt], blo[h], acc[h][mt], 0, 0, 0);
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
            for (int h = 0; h < 2; ++h)
                acc[h][mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo[mt], bhi[h], acc[h][mt], 0, 0, 0);
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int mt = 0; mt < 2; ++mt) {
                *reinterpret_cast<float2 *>(tb + (wr[mt][0] ^ gt[h])) = make_float2(acc[h][mt][0], acc[h][mt][1]);
                *reinterpret_cast<float2 *>(tb + (wr[mt][1] ^ gt[h])) = make_float2(acc[h][mt][2], acc[h][mt][3]);
            }
    }
}

// Five-qubit blocks in split form: with Ur = Re U and Ui = Im U (32 x 32
// each) and the re / im parts of a group as separate columns,
//   Yr = Ur Xr - Ui Xi,   Yi = Ui Xr + Ur Xi,
// which needs half the operand registers of the real form at the same
// number of matrix-core products.  Fragment order: Ur row tiles 0, 1, Ui row
// tiles 0, 1 (hi), then the same four (lo).
__device__ void dense_op5(float2 *tile, const TileOpDev &op, const uint4 *data, int m, int outer)
{
    constexpr int K = 5;
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
    const bf16x8 *fr =
        reinterpret_cast<const bf16x8 *>(data + op.data_off + uint32_t(outer) * op.frag_stride);
    // fragments: Ur, Ui, -Ui row tiles (hi), then the same (lo)
    bf16x8 urh[2], uih[2], nuih[2], url[2], uil[2], nuil[2];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
        urh[mt] = fr[(0 + mt) * 64 + lane];
        uih[mt] = fr[(2 + mt) * 64 + lane];
        nuih[mt] = fr[(4 + mt) * 64 + lane];
        url[mt] = fr[(6 + mt) * 64 + lane];
        uil[mt] = fr[(8 + mt) * 64 + lane];
        nuil[mt] = fr[(10 + mt) * 64 + lane];
    }
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
    // The group base and the LDS swizzle are linear over disjoint bits, so an
    // address is (per-lane part) ^ (per-column-tile part): precompute the
    // per-lane byte offsets once.
    const uint32_t gl = insert_zero_bits(uint32_t(lane & 15), srt, K);
    uint32_t rd[8], wr[2][4];
#pragma unroll
    for (int j = 0; j < 8; ++j) rd[j] = sw(gl | offset(8 * (lane >> 4) + j)) * 8u;
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int j = 0; j < 4; ++j) wr[mt][j] = sw(gl | offset(16 * mt + 4 * (lane >> 4) + j)) * 8u;
    char *tb = reinterpret_cast<char *>(tile);
    const int ntiles = 1 << (m - K - 4);
    constexpr int kWaves = kThreads / 64;
    for (int nt = wave; nt < ntiles; nt += kWaves) {
        const uint32_t gt = sw(insert_zero_bits(uint32_t(nt) * 16u, srt, K)) * 8u;  // uniform
        float2 v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = *reinterpret_cast<const float2 *>(tb + (rd[j] ^ gt));
        bf16x8 xrh, xrl, xih, xil;
#pragma unroll
        for (int j = 0; j < 8; j += 2) {
            v2bf h, l;
            split2(v[j].x, v[j + 1].x, h, l);
            xrh[j] = h[0];
            xrh[j + 1] = h[1];
            xrl[j] = l[0];
            xrl[j + 1] = l[1];
            split2(v[j].y, v[j + 1].y, h, l);
            xih[j] = h[0];
            xih[j + 1] = h[1];
            xil[j] = l[0];
            xil[j + 1] = l[1];
        }
        f32x4 ar[2], ai[2];
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) {
            ar[mt] = f32x4{0.f, 0.f, 0.f, 0.f};
            ai[mt] = f32x4{0.f, 0.f, 0.f, 0.f};
        }
        // Yr = Ur Xr - Ui Xi, Yi = Ui Xr + Ur Xi; hi*hi + hi*lo + lo*hi each
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) {
            ar[mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(urh[mt], xrh, ar[mt], 0, 0, 0);
            ai[mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(uih[mt], xrh, ai[mt], 0, 0, 0);
        }
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) {
            ar[mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nuih[mt], xih, ar[mt], 0, 0, 0);
            ai[mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(urh[mt], xih, ai[mt], 0, 0, 0);
        }
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) {
            ar[mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(urh[mt], xrl, ar[mt], 0, 0, 0);
            ai[mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(uih[mt], xrl, ai[mt], 0, 0, 0);
        }
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) {
            ar[mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nuih[mt], xil, ar[mt], 0, 0, 0);
            ai[mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(urh[mt], xil, ai[mt], 0, 0, 0);
        }
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) {
            ar[mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(url[mt], xrh, ar[mt], 0, 0, 0);
            ai[mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(uil[mt], xrh, ai[mt], 0, 0, 0);
        }
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) {
            ar[mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nuil[mt], xih, ar[mt], 0, 0, 0);
            ai[mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(url[mt], xih, ai[mt], 0, 0, 0);
        }
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                *reinterpret_cast<float2 *>(tb + (wr[mt][j] ^ gt)) = make_float2(ar[mt][j], ai[mt][j]);
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
            const float2 v = tile[sw(j)];
            tile[sw(j)] = make_float2(f.x * v.x - f.y * v.y, f.x * v.y + f.y * v.x);
        }
    }
}

// One tile: load, apply ops, store.  `toff` is this thread's offset within
// a tile (local index 2 * tid spread over the tile qubits).
template <int M>
__device__ __forceinline__ void tile_pass(float2 *amp, uint64_t t, const TileArgs &ta, uint64_t toff,
                                          const TileOpDev *ops, const uint4 *data, float2 *tile,
                                          float2 *ptab)
{
    constexpr int PER = (1 << M) / (2 * kThreads);  // 16-byte slots (2 amplitudes) per thread
    // tile base: the tile index spread over the bits outside the tile
    uint64_t base = 0;
    for (int b = 0; b < ta.nouter; ++b)
        if ((t >> b) & 1) base |= uint64_t(1) << ta.outer[b];
    // ---- load (non-temporal: every amplitude is read once per sweep)
    vf4 buf[PER];
#pragma unroll
    for (int r = 0; r < PER; ++r)
        buf[r] = __builtin_nontemporal_load(reinterpret_cast<const vf4 *>(amp + (base | toff | ta.slot[r])));
#pragma unroll
    for (int r = 0; r < PER; ++r) {
        const uint32_t j = 2u * (threadIdx.x + uint32_t(r) * kThreads);
        tile[sw(j)] = make_float2(buf[r].x, buf[r].y);
        tile[sw(j + 1)] = make_float2(buf[r].z, buf[r].w);
    }
    __syncthreads();
    // ---- ops
    for (int oi = 0; oi < ta.nops; ++oi) {
        const TileOpDev op = ops[oi];
        int outer = 0;
#pragma unroll
        for (int b = 0; b < 5; ++b)
            if (b < op.no) outer = (outer << 1) | int((base >> op.opos[b]) & 1);
        if (op.kind == 0) {
            if ((op.skip >> outer) & 1u) continue;  // identity on this tile
            if (op.k == 4)
                dense_op4(tile, op, data, M, outer);
            else
                dense_op5(tile, op, data, M, outer);
        } else {
            phase_op(tile, ptab, op, data, outer, M);
        }
        __syncthreads();
    }
    // ---- store
#pragma unroll
    for (int r = 0; r < PER; ++r) {
        const uint32_t j = 2u * (threadIdx.x + uint32_t(r) * kThreads);
        const float2 a0 = tile[sw(j)], a1 = tile[sw(j + 1)];
        buf[r] = vf4{a0.x, a0.y, a1.x, a1.y};
    }
#pragma unroll
    for (int r = 0; r < PER; ++r)
        __builtin_nontemporal_store(buf[r], reinterpret_cast<vf4 *>(amp + (base | toff | ta.slot[r])));
    __syncthreads();
}

__device__ __forceinline__ uint64_t thread_offset(const TileArgs &ta)
{
    // local index 2 * tid (bits 1..8); slot r adds the uniform ta.slot[r]
    uint64_t toff = 0;
#pragma unroll
    for (int b = 1; b < 9; ++b)
        if (((2u * threadIdx.x) >> b) & 1u) toff |= uint64_t(1) << ta.qlo[b];
    return toff;
}

template <int M>
__global__ __launch_bounds__(kThreads) void k_tile(float2 *amp, uint64_t ntiles, TileArgs ta,
                                                   const TileOpDev *ops, const uint4 *data)
{
    extern __shared__ float2 lds[];
    float2 *ptab = lds + (size_t(1) << M);
    const uint64_t toff = thread_offset(ta);
    for (uint64_t t = blockIdx.x; t < ntiles; t += gridDim.x)
        tile_pass<M>(amp, t, ta, toff, ops, data, lds, ptab);
}

// Batched form: workgroup b runs tile tasks[b].tile of the state described by
// args[tasks[b].arg] (its own amplitudes, tile qubits and op list), so one
// launch covers one sweep of many independent states.
template <int M>
__global__ __launch_bounds__(kThreads) void k_tile_multi(const TileTask *tasks, const TileArgsDev *args,
                                                         const TileOpDev *ops, const uint4 *data)
{
    extern __shared__ float2 lds[];
    float2 *ptab = lds + (size_t(1) << M);
    const TileTask task = tasks[blockIdx.x];
    const TileArgsDev &ad = args[task.arg];
    const uint64_t toff = thread_offset(ad.ta);
    tile_pass<M>(ad.amp, task.tile, ad.ta, toff, ops + ad.op_off, data, lds, ptab);
}

}  // namespace

size_t tile_lds_bytes(int m) { return (size_t(8) << m) + 64 * sizeof(float2); }

template <typename F>
hipError_t set_lds_attr(F kernel)
{
    return hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                               int(tile_lds_bytes(13)));
}

hipError_t ensure_attrs()
{
    static bool done = false;
    if (done) return hipSuccess;
    hipError_t e = set_lds_attr(k_tile<13>);
    if (e == hipSuccess) e = set_lds_attr(k_tile<12>);
    if (e == hipSuccess) e = set_lds_attr(k_tile_multi<13>);
    if (e == hipSuccess) e = set_lds_attr(k_tile_multi<12>);
    if (e == hipSuccess) done = true;
    return e;
}

hipError_t launch_tile(void *amp, int n, const TileArgs &ta, const TileOpDev *dev_ops,
                       const void *dev_data, hipStream_t st)
{
    if (ta.m < 10 || ta.m > 13 || ta.m > n || ta.nouter != n - ta.m) return hipErrorInvalidValue;
    const size_t lds = tile_lds_bytes(ta.m);
    if (hipError_t e = ensure_attrs()) return e;
    const uint64_t ntiles = uint64_t(1) << (n - ta.m);
    const uint64_t grid = ntiles < (uint64_t(1) << 20) ? ntiles : (uint64_t(1) << 20);
    float2 *a = (float2 *)amp;
    const uint4 *d = (const uint4 *)dev_data;
    switch (ta.m) {
    case 10:
        hipLaunchKernelGGL(k_tile<10>, dim3(unsigned(grid)), dim3(kThreads), lds, st, a, ntiles, ta, dev_ops, d);
        break;
    case 11:
        hipLaunchKernelGGL(k_tile<11>, dim3(unsigned(grid)), dim3(kThreads), lds, st, a, ntiles, ta, dev_ops, d);
        break;
    case 12:
        hipLaunchKernelGGL(k_tile<12>, dim3(unsigned(grid)), dim3(kThreads), lds, st, a, ntiles, ta, dev_ops, d);
        break;
    default:
        hipLaunchKernelGGL(k_tile<13>, dim3(unsigned(grid)), dim3(kThreads), lds, st, a, ntiles, ta, dev_ops, d);
        break;
    }
    return hipGetLastError();
}

hipError_t launch_tile_multi(int m, uint32_t ntasks, const TileTask *tasks, const TileArgsDev *args,
                             const TileOpDev *dev_ops, const void *dev_data, hipStream_t st)
{
    if (m < 10 || m > 13 || ntasks == 0) return hipErrorInvalidValue;
    const size_t lds = tile_lds_bytes(m);
    if (hipError_t e = ensure_attrs()) return e;
    const uint4 *d = (const uint4 *)dev_data;
    switch (m) {
    case 10:
        hipLaunchKernelGGL(k_tile_multi<10>, dim3(ntasks), dim3(kThreads), lds, st, tasks, args, dev_ops, d);
        break;
    case 11:
        hipLaunchKernelGGL(k_tile_multi<11>, dim3(ntasks), dim3(kThreads), lds, st, tasks, args, dev_ops, d);
        break;
    case 12:
        hipLaunchKernelGGL(k_tile_multi<12>, dim3(ntasks), dim3(kThreads), lds, st, tasks, args, dev_ops, d);
        break;
    default:
        hipLaunchKernelGGL(k_tile_multi<13>, dim3(ntasks), dim3(kThreads), lds, st, tasks, args, dev_ops, d);
        break;
    }
    return hipGetLastError();
}

}  // namespace qs
