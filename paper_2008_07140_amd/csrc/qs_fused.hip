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


typedef float v2f __attribute__((ext_vector_type(2)));
typedef __bf16 v2bf __attribute__((ext_vector_type(2)));

// A bf16 pair with the given bits, held in a scalar register.  The pairs
// (-1, 0) and (0, -1) feed the remainder dot products below; left visible, the
// compiler encodes (-1, 0) as the inline constant -1.0, which the hardware
// does not read as that pair (measured: wrong remainders), so the bits are
// hidden behind an empty asm statement.
__device__ __forceinline__ v2bf scalar_pair(uint32_t bits)
{
    asm("" : "+s"(bits));
    return __builtin_bit_cast(v2bf, bits);
}

// Split two floats into bfloat16 hi parts and the bfloat16 of the remainders
// (packed conversions).  Each remainder a - hi[0] is a bf16 dot product of the
// packed hi parts with m0 = (-1, 0) (m1 = (0, -1) for b) accumulated onto a:
// one instruction, with no conversion of hi back to FP32, and exact (the
// remainder fits in FP32).
__device__ __forceinline__ void split2(float a, float b, v2bf m0, v2bf m1, v2bf &hi, v2bf &lo)
{
    hi = __builtin_convertvector(v2f{a, b}, v2bf);
    lo = __builtin_convertvector(
        v2f{__builtin_amdgcn_fdot2_f32_bf16(hi, m0, a, false), __builtin_amdgcn_fdot2_f32_bf16(hi, m1, b, false)},
        v2bf);
}

__device__ __forceinline__ uint32_t sw(uint32_t j) { return tile_swizzle(j); }

// Operand fragments of a dense k-qubit block (k = 4, 5) for one outer pattern
// and this lane's LDS offsets, in registers.  The block is applied in real
// form: with D = 2^k, A is the 2D x 2D real matrix [[Re U, -Im U], [Im U, Re U]]
// (entry by entry, re / im interleaved) and a group of the tile is one column
// of X, so the re and im parts of an output amplitude come out in adjacent
// accumulator registers.  Fragment (mt, s) of lane l holds
// A[16 mt + l % 16][32 s + 8 (l / 16) + j], j < 8 (hi parts of all fragments,
// then the remainders).
template <int K>
struct Frags {
    static constexpr int D = 1 << K, MT = 2 * D / 16, KS = 2 * D / 32, NQ = tile_lane_offsets(K) / 4;
    bf16x8 ahi[MT][KS], alo[MT][KS];
    uint32_t ofs[4 * NQ];  // KS * 4 read offsets, then MT * 2 write offsets
};

template <int K>
__device__ __forceinline__ void load_frags(Frags<K> &f, const bf16x8 *fr, const uint4 *offs)
{
    constexpr int MT = Frags<K>::MT, KS = Frags<K>::KS, NQ = Frags<K>::NQ;
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            f.ahi[mt][s] = fr[(mt * KS + s) * 64 + lane];
            f.alo[mt][s] = fr[MT * KS * 64 + (mt * KS + s) * 64 + lane];
        }
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const uint4 o = offs[lane * NQ + q];
        f.ofs[4 * q] = o.x;
        f.ofs[4 * q + 1] = o.y;
        f.ofs[4 * q + 2] = o.z;
        f.ofs[4 * q + 3] = o.w;
    }
}

// Apply one dense block to the tile with fragments f; NW waves share the
// column tiles.  Column c of a matrix-core tile sits on the 4 tile bits of
// op.colmask, the column tile index on the other bits outside the op.  A wave
// walks its column tiles in Gray-code order, so the uniform part of the LDS
// address changes by one precomputed XOR per step, and reads the next tile's
// amplitudes while the current one is multiplied.  `prefetch` is called once
// on every path, after the wave's last LDS read of the op (its input buffers
// are then free): the caller loads the next op's fragments there, so their
// latency overlaps the last multiplications, the write-back and the barrier.
template <int K, int NW, class Prefetch>
__device__ __forceinline__ void dense_op(float2 *tile, const TileOpDev &op, const Frags<K> &f, int m,
                                         Prefetch &&prefetch)
{
    constexpr int MT = Frags<K>::MT, KS = Frags<K>::KS;
    constexpr int H = K == 4 ? 2 : 1;  // column tiles per step: at least 4 accumulator chains
    constexpr int LB = (H == 2 ? 1 : 0) + (NW == 8 ? 3 : NW == 4 ? 2 : NW == 2 ? 1 : 0);
    constexpr int MAXSTEPS = 4;  // at most 32 column tiles (m <= 13) over H * NW >= 8 per step
    const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
    const int ntiles = 1 << (m - K - 4);
    if (H * wave >= ntiles) {  // fewer column tiles than waves
        prefetch();
        return;
    }
    const uint32_t *rd = f.ofs, *wr = f.ofs + KS * 4;
    // LDS byte offsets of the column-tile index bits (tile bits outside the
    // op and its column bits), from the host
    uint32_t img[LB + 2];
#pragma unroll
    for (int t = 0; t < LB + 2; ++t) img[t] = t < 6 ? op.cimg[t] : 0u;
    uint32_t gt = 0;  // first column tile of this wave: index H * wave
#pragma unroll
    for (int b = 0; b < LB; ++b)
        if (((H * wave) >> b) & 1) gt ^= img[b];
    gt = __builtin_amdgcn_readfirstlane(gt);
    const int steps = ntiles > H * NW ? ntiles / (H * NW) : 1;
    char *tb = reinterpret_cast<char *>(tile);
    const v2bf m0 = scalar_pair(0x0000bf80u), m1 = scalar_pair(0xbf800000u);
    float2 v[2][H][KS][4];
    auto read_x = [&](float2 (&dst)[H][KS][4], uint32_t g0) {
#pragma unroll
        for (int h = 0; h < H; ++h) {
            const uint32_t gh = h ? g0 ^ img[0] : g0;
#pragma unroll
            for (int s = 0; s < KS; ++s)
#pragma unroll
                for (int jj = 0; jj < 4; ++jj)
                    dst[h][s][jj] = *reinterpret_cast<const float2 *>(tb + (rd[s * 4 + jj] ^ gh));
        }
    };
    read_x(v[0], gt);
#pragma unroll
    for (int g = 0; g < MAXSTEPS; ++g) {
        if (g >= steps) break;
        const uint32_t gn = gt ^ (((g + 1) & 1) ? img[LB] : img[LB + 1]);
        if (g + 1 < steps) read_x(v[(g + 1) & 1], gn);
        float2 (&x)[H][KS][4] = v[g & 1];
        bf16x8 bhi[H][KS], blo[H][KS];
#pragma unroll
        for (int h = 0; h < H; ++h)
#pragma unroll
            for (int s = 0; s < KS; ++s)
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) {
                    v2bf hh, ll;
                    split2(x[h][s][jj].x, x[h][s][jj].y, m0, m1, hh, ll);
                    bhi[h][s][2 * jj] = hh[0];
                    bhi[h][s][2 * jj + 1] = hh[1];
                    blo[h][s][2 * jj] = ll[0];
                    blo[h][s][2 * jj + 1] = ll[1];
                }
        if (g + 1 == steps) prefetch();
        f32x4 acc[H][MT];
#pragma unroll
        for (int h = 0; h < H; ++h)
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) acc[h][mt] = f32x4{0.f, 0.f, 0.f, 0.f};
        // hi * hi, hi * lo, lo * hi, each over the k-steps
#pragma unroll
        for (int s = 0; s < KS; ++s)
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int h = 0; h < H; ++h)
                    acc[h][mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(f.ahi[mt][s], bhi[h][s], acc[h][mt], 0, 0, 0);
#pragma unroll
        for (int s = 0; s < KS; ++s)
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int h = 0; h < H; ++h)
                    acc[h][mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(f.ahi[mt][s], blo[h][s], acc[h][mt], 0, 0, 0);
#pragma unroll
        for (int s = 0; s < KS; ++s)
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int h = 0; h < H; ++h)
                    acc[h][mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(f.alo[mt][s], bhi[h][s], acc[h][mt], 0, 0, 0);
#pragma unroll
        for (int h = 0; h < H; ++h) {
            const uint32_t gh = h ? gt ^ img[0] : gt;
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                *reinterpret_cast<float2 *>(tb + (wr[mt * 2] ^ gh)) = make_float2(acc[h][mt][0], acc[h][mt][1]);
                *reinterpret_cast<float2 *>(tb + (wr[mt * 2 + 1] ^ gh)) = make_float2(acc[h][mt][2], acc[h][mt][3]);
            }
        }
        gt = gn;
    }
}

template <int NT>
__device__ void phase_op(float2 *tile, float2 *ptab, const TileOpDev &op, const uint4 *data,
                         int outer, int m)
{
    const float2 *tab = reinterpret_cast<const float2 *>(data + op.data_off + uint32_t(outer) * op.frag_stride);
    const int D = 1 << op.k;
    if (int(threadIdx.x) < D) ptab[threadIdx.x] = tab[threadIdx.x];
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
    // rows j = tid + NT i, i in Gray-code order: the swizzle is linear, so
    // sw(j) = sw(tid) ^ sw(NT i) and one bit of i changes per step
    const uint32_t st = sw(threadIdx.x);
    const int rows = (1 << m) / NT;
    uint32_t i = 0, su = 0;
    for (int g = 0; g < rows; ++g) {
        if (g) {
            const int b = __builtin_ctz(uint32_t(g));
            i ^= 1u << b;
            su ^= sw(uint32_t(NT) << b);
        }
        const uint32_t j = i * NT + threadIdx.x;
        int x = 0;
#pragma unroll
        for (int b = 0; b < 3; ++b)
            if (b < op.k) x |= int((j >> lp[b]) & 1) << sh[b];
        if ((active >> x) & 1) {
            const uint32_t a = st ^ su;
            const float2 f = ptab[x];
            const float2 v = tile[a];
            tile[a] = make_float2(f.x * v.x - f.y * v.y, f.x * v.y + f.y * v.x);
        }
    }
}

// Scatter the low bits of x onto the set bits of mask (ascending).
__device__ __forceinline__ uint64_t deposit_bits(uint64_t x, uint64_t mask)
{
    uint64_t r = 0;
    for (uint64_t mm = mask; mm; mm &= mm - 1, x >>= 1)
        if (x & 1) r |= mm & (~mm + 1);
    return r;
}

// Global base index of tile t under the sweep's tile order.  Tiles that
// run at the same time share the low bits of t, and the order decides which
// outer qubits those bits select, hence how the concurrent 128-byte runs of
// a sweep spread over HBM; which order is fastest depends on the sweep's
// tile qubits and is measured by the host.  Workgroups are dispatched to the
// eight XCDs in turn, so bits 0..2 of t name the XCD running the tile.
//   0: bits 0..2 select the three highest outer qubits (each XCD streams its
//      own eighth of the state), the rest walk the others from the lowest;
//   1: as 0, and bits 3..5 select the next three highest;
//   2: t walks the outer qubits from the lowest;
//   3: t walks the outer qubits from the highest.
// Every order is a bijection of [0, 2^nouter).
__device__ __forceinline__ uint64_t tile_base(uint64_t t, const TileArgs &ta)
{
    const int no = ta.nouter;
    switch (ta.order) {
    case 0:
        if (no >= 3) t = (t >> 3) | ((t & 7) << (no - 3));
        break;
    case 1:
        if (no >= 6)
            t = (t >> 6) | (((t >> 3) & 7) << (no - 6)) | ((t & 7) << (no - 3));
        else if (no >= 3)
            t = (t >> 3) | ((t & 7) << (no - 3));
        break;
    case 3: {
        uint64_t r = 0;
        for (int b = 0; b < no; ++b) r |= ((t >> b) & 1) << (no - 1 - b);
        t = r;
        break;
    }
    default:
        break;
    }
    return deposit_bits(t, ta.omask);
}

// Outer pattern of an op on the tile at `base` (opos[0] most significant).
__device__ __forceinline__ int op_pattern(const TileOpDev &op, uint64_t base)
{
    int outer = 0;
#pragma unroll
    for (int b = 0; b < 5; ++b)
        if (b < op.no) outer = (outer << 1) | int((base >> op.opos[b]) & 1);
    return outer;
}

// Global offset of local index r << TB (the r-th 16-byte slot of a thread,
// TB = log2(2 NT)): bit i of r lands on tile qubit q[TB + i].  The positions
// pass through an empty asm statement so the offsets are recomputed where
// they are used (a few scalar instructions) instead of held in scalar
// registers across the op loop.
template <int TB, int PER>
__device__ __forceinline__ uint64_t slot_offset(const TileArgs &ta, int r)
{
    static_assert(TB == 9 || TB == 10, "thread bits");
    uint32_t w = uint32_t(ta.q[TB]) | uint32_t(ta.q[TB + 1]) << 8 | uint32_t(ta.q[TB + 2]) << 16 |
                 (TB == 9 ? uint32_t(ta.q[TB + 3]) << 24 : 0u);
    w = __builtin_amdgcn_readfirstlane(w);
    asm("" : "+s"(w));
    uint64_t off = 0;
#pragma unroll
    for (int i = 0; (1 << i) < PER; ++i)
        if ((r >> i) & 1) off |= uint64_t(1) << ((w >> (8 * i)) & 63u);
    return off;
}

// One tile: load, apply ops, store, with NT threads; K5: the op list may
// hold 5-qubit blocks.  `toff` is this thread's offset within a tile (local
// index 2 * tid spread over the tile qubits); thread slot r adds the uniform
// slot_offset (local index 2 NT r).
template <int M, int NT, bool K5>
__device__ __forceinline__ void tile_pass(float2 *amp, uint64_t t, const TileArgs &ta, uint64_t toff,
                                          const TileOpDev *ops, const uint4 *data, float2 *tile,
                                          float2 *ptab)
{
    constexpr int PER = (1 << M) / (2 * NT);  // 16-byte slots (2 amplitudes) per thread
    constexpr int TB = NT == 512 ? 10 : 9;
    // tile base: the tile index spread over the bits outside the tile
    const uint64_t base = tile_base(t, ta);
    // ---- load (non-temporal: every amplitude is read once per sweep)
    vf4 buf[PER];
#pragma unroll
    for (int r = 0; r < PER; ++r)
        buf[r] = __builtin_nontemporal_load(
            reinterpret_cast<const vf4 *>(amp + (base | toff | slot_offset<TB, PER>(ta, r))));
    // amplitudes 2 t and 2 t + 1 of a thread share one 16-byte LDS unit
    // (sw(j + 1) = sw(j) ^ 1 for even j): one 16-byte access each, halves
    // swapped when sw(j) is odd
    const uint32_t st = sw(2u * threadIdx.x);
#pragma unroll
    for (int r = 0; r < PER; ++r) {
        const uint32_t s0 = st ^ sw(2u * uint32_t(r) * NT);
        vf4 *u = reinterpret_cast<vf4 *>(tile) + (s0 >> 1);
        *u = (s0 & 1u) ? vf4{buf[r].z, buf[r].w, buf[r].x, buf[r].y} : buf[r];
    }
    __syncthreads();
    // ---- ops (an op whose matrix is the identity on this tile's outer
    // pattern is skipped, barrier included: the pattern is uniform)
    if constexpr (K5) {
        for (int oi = 0; oi < ta.nops; ++oi) {
            const TileOpDev op = ops[oi];
            const int outer = op_pattern(op, base);
            if (op.kind == 0) {
                if ((op.skip >> outer) & 1u) continue;
                const bf16x8 *fr =
                    reinterpret_cast<const bf16x8 *>(data + op.data_off + uint32_t(outer) * op.frag_stride);
                if (op.k == 4) {
                    Frags<4> f;
                    load_frags<4>(f, fr, data + op.offs_off);
                    dense_op<4, NT / 64>(tile, op, f, M, [] {});
                } else {
                    Frags<5> f;
                    load_frags<5>(f, fr, data + op.offs_off);
                    dense_op<5, NT / 64>(tile, op, f, M, [] {});
                }
            } else {
                phase_op<NT>(tile, ptab, op, data, outer, M);
            }
            __syncthreads();
        }
    } else {
        // 4-qubit blocks only: the descriptor and fragments of op i + 1 load
        // while op i finishes, into two register sets used in turn
        // Descriptors are read where they are used, through a pointer the
        // compiler cannot see through, so at most one and a few fields of the
        // next stay in scalar registers.
        auto desc = [&](int i) {
            uint32_t ui = __builtin_amdgcn_readfirstlane(uint32_t(i));
            asm("" : "+s"(ui));
            return ops + ui;
        };
        Frags<4> fa, fb;
        // (written on every path, so the previous contents of a set are dead)
        auto fetch = [&](Frags<4> &f, const TileOpDev &o, int pat) {
            if (o.kind == 0 && !((o.skip >> pat) & 1u))
                load_frags<4>(f, reinterpret_cast<const bf16x8 *>(data + o.data_off + uint32_t(pat) * o.frag_stride),
                              data + o.offs_off);
            else
                f = Frags<4>{};
        };
        if (ta.nops > 0) {
            const TileOpDev *p0 = desc(0);
            fetch(fa, *p0, op_pattern(*p0, base));
        }
        auto run = [&](int oi, const Frags<4> &cur, Frags<4> &nxt) {
            const TileOpDev &op = *desc(oi);
            const int outer = op_pattern(op, base);
            // the next op's fields that locate its fragments are read now, so
            // their scalar loads complete while this op runs
            const bool has_next = oi + 1 < ta.nops;
            const TileOpDev &nop = *desc(has_next ? oi + 1 : oi);
            const int npat = op_pattern(nop, base);
            const bool nload = has_next && nop.kind == 0 && !((nop.skip >> npat) & 1u);
            const uint32_t nfr = nop.data_off + uint32_t(npat) * nop.frag_stride, noffs = nop.offs_off;
            auto prefetch = [&] {
                if (nload)
                    load_frags<4>(nxt, reinterpret_cast<const bf16x8 *>(data + nfr), data + noffs);
                else
                    nxt = Frags<4>{};
            };
            if (op.kind != 0) {
                prefetch();
                phase_op<NT>(tile, ptab, op, data, outer, M);
                __syncthreads();
            } else if ((op.skip >> outer) & 1u) {
                prefetch();
            } else {
                dense_op<4, NT / 64>(tile, op, cur, M, prefetch);
                __syncthreads();
            }
        };
        for (int oi = 0; oi < ta.nops; oi += 2) {
            run(oi, fa, fb);
            if (oi + 1 >= ta.nops) break;
            run(oi + 1, fb, fa);
        }
    }
    // ---- store
#pragma unroll
    for (int r = 0; r < PER; ++r) {
        const uint32_t s0 = st ^ sw(2u * uint32_t(r) * NT);
        const vf4 u = reinterpret_cast<const vf4 *>(tile)[s0 >> 1];
        buf[r] = (s0 & 1u) ? vf4{u.z, u.w, u.x, u.y} : u;
    }
#pragma unroll
    for (int r = 0; r < PER; ++r)
        __builtin_nontemporal_store(buf[r],
                                    reinterpret_cast<vf4 *>(amp + (base | toff | slot_offset<TB, PER>(ta, r))));
    __syncthreads();
}

template <int NT>
__device__ __forceinline__ uint64_t thread_offset(const TileArgs &ta)
{
    // local index 2 * tid: bits 1 .. log2(2 NT) - 1
    constexpr int TB = NT == 512 ? 10 : 9;
    uint64_t toff = 0;
#pragma unroll
    for (int b = 1; b < TB; ++b)
        if (((2u * threadIdx.x) >> b) & 1u) toff |= uint64_t(1) << ta.q[b];
    return toff;
}

// Workgroup shapes.  Op lists with 5-qubit blocks: 256 threads, two waves
// per SIMD (their operand fragments need up to 256 registers).  Lists of
// 4-qubit blocks and phase ops: at most 128 registers, four waves per SIMD,
// so each wave's waits are better covered; 512 threads on tiles of 12 or 13
// qubits (16 or 32 column tiles per 4-qubit block, enough for 8 waves), 256
// threads on smaller tiles (four workgroups per compute unit).
constexpr int tile_threads(int m, bool k5) { return k5 || m < 12 ? 256 : 512; }
#define QS_TILE_ATTRS(NT, K5) __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(K5 ? 2 : 4, K5 ? 2 : 4)))

template <int M, int NT, bool K5>
__global__ QS_TILE_ATTRS(NT, K5) void k_tile(float2 *__restrict__ amp, uint64_t ntiles, TileArgs ta,
                                         const TileOpDev *__restrict__ ops, const uint4 *__restrict__ data)
{
    __shared__ __attribute__((aligned(16))) float2 lds[(1 << M) + 64];  // the tile, then a phase table
    const uint64_t toff = thread_offset<NT>(ta);
    for (uint64_t t = blockIdx.x; t < ntiles; t += gridDim.x)
        tile_pass<M, NT, K5>(amp, t, ta, toff, ops, data, lds, lds + (1 << M));
}

// Batched form: workgroup b runs tile tasks[b].tile of the state described by
// args[tasks[b].arg] (its own amplitudes, tile qubits and op list), so one
// launch covers one sweep of many independent states.
template <int M, int NT, bool K5>
__global__ QS_TILE_ATTRS(NT, K5) void k_tile_multi(const TileTask *__restrict__ tasks,
                                               const TileArgsDev *__restrict__ args,
                                               const TileOpDev *__restrict__ ops,
                                               const uint4 *__restrict__ data,
                                               const int *__restrict__ active)
{
    __shared__ __attribute__((aligned(16))) float2 lds[(1 << M) + 64];
    const TileTask task = tasks[blockIdx.x];
    const TileArgsDev ad = args[task.arg];
    if (active && !active[ad.slot]) return;  // uniform over the workgroup, before any barrier
    const uint64_t toff = thread_offset<NT>(ad.ta);
    tile_pass<M, NT, K5>(ad.amp, task.tile, ad.ta, toff, ops + ad.op_off, data, lds, lds + (1 << M));
}

template <int M, bool K5>
void launch_m(float2 *a, uint64_t grid, uint64_t ntiles, const TileArgs &ta, const TileOpDev *ops,
              const uint4 *d, hipStream_t st)
{
    constexpr int NT = tile_threads(M, K5);
    hipLaunchKernelGGL((k_tile<M, NT, K5>), dim3(unsigned(grid)), dim3(NT), 0, st, a, ntiles, ta, ops, d);
}

template <int M, bool K5>
void launch_multi_m(uint32_t ntasks, const TileTask *tasks, const TileArgsDev *args, const TileOpDev *ops,
                    const uint4 *d, const int *active, hipStream_t st)
{
    constexpr int NT = tile_threads(M, K5);
    hipLaunchKernelGGL((k_tile_multi<M, NT, K5>), dim3(ntasks), dim3(NT), 0, st, tasks, args, ops, d, active);
}

}  // namespace

hipError_t launch_tile(void *amp, int n, const TileArgs &ta, const TileOpDev *dev_ops,
                       const void *dev_data, bool k5, hipStream_t st)
{
    if (ta.m < 10 || ta.m > 13 || ta.m > n || ta.nouter != n - ta.m) return hipErrorInvalidValue;
    const uint64_t ntiles = uint64_t(1) << (n - ta.m);
    const uint64_t grid = ntiles < (uint64_t(1) << 20) ? ntiles : (uint64_t(1) << 20);
    float2 *a = (float2 *)amp;
    const uint4 *d = (const uint4 *)dev_data;
    switch (ta.m * 2 + int(k5)) {
    case 20: launch_m<10, false>(a, grid, ntiles, ta, dev_ops, d, st); break;
    case 21: launch_m<10, true>(a, grid, ntiles, ta, dev_ops, d, st); break;
    case 22: launch_m<11, false>(a, grid, ntiles, ta, dev_ops, d, st); break;
    case 23: launch_m<11, true>(a, grid, ntiles, ta, dev_ops, d, st); break;
    case 24: launch_m<12, false>(a, grid, ntiles, ta, dev_ops, d, st); break;
    case 25: launch_m<12, true>(a, grid, ntiles, ta, dev_ops, d, st); break;
    case 26: launch_m<13, false>(a, grid, ntiles, ta, dev_ops, d, st); break;
    default: launch_m<13, true>(a, grid, ntiles, ta, dev_ops, d, st); break;
    }
    return hipGetLastError();
}

hipError_t launch_tile_multi(int m, uint32_t ntasks, const TileTask *tasks, const TileArgsDev *args,
                             const TileOpDev *dev_ops, const void *dev_data, bool k5, const int *active,
                             hipStream_t st)
{
    if (m < 10 || m > 13 || ntasks == 0) return hipErrorInvalidValue;
    const uint4 *d = (const uint4 *)dev_data;
    switch (m * 2 + int(k5)) {
    case 20: launch_multi_m<10, false>(ntasks, tasks, args, dev_ops, d, active, st); break;
    case 21: launch_multi_m<10, true>(ntasks, tasks, args, dev_ops, d, active, st); break;
    case 22: launch_multi_m<11, false>(ntasks, tasks, args, dev_ops, d, active, st); break;
    case 23: launch_multi_m<11, true>(ntasks, tasks, args, dev_ops, d, active, st); break;
    case 24: launch_multi_m<12, false>(ntasks, tasks, args, dev_ops, d, active, st); break;
    case 25: launch_multi_m<12, true>(ntasks, tasks, args, dev_ops, d, active, st); break;
    case 26: launch_multi_m<13, false>(ntasks, tasks, args, dev_ops, d, active, st); break;
    default: launch_multi_m<13, true>(ntasks, tasks, args, dev_ops, d, active, st); break;
    }
    return hipGetLastError();
}

}  // namespace qs
