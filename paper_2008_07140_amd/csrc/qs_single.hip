// Single-amplitude mode (Sec. 2.3): the vertex eliminations of the
// graphical model as batched complex FP64 tensor contractions.
//
// Every tensor index is one Boolean variable (a vertex), so every dimension
// is 2 and a tensor of r indices holds 2^r complex doubles.  A merge of two
// tensors that sums the shared vertices no other tensor holds is a batched
// product Z[t, b, m, n] = sum_k X[t, b, m, k] Y[t, b, n, k] (t = batch
// element: a bitstring and a slice).  The host lays every operand out for
// the merge that consumes it (summed bits lowest), so the product reads
// both operands with unit stride along k; only the result is written
// through a bit permutation.  The MI355X's FP64 matrix and vector peaks are
// equal (78.6 TFLOP/s), so the products run on the vector units: large ones
// as 64 x 64 LDS tiles, small ones one wave or one thread per result.
#include <hip/hip_runtime.h>

#include "qs_single.h"

namespace qs {

namespace {

constexpr int kT = 256;

// Non-temporal 16-byte load and store, for the streaming merges of one or
// a few summed vertices whose every access instruction covers whole lines
// (k_sa_pairs reads and writes, k_sa_rows writes for 1-3 summed vertices).
// Measured on the 60-qubit workload: a fifth less time in all than cached
// accesses; non-temporal reads of k_sa_rows' 32-byte-strided rows made the
// run 2.5 times slower, and non-temporal writes in the tiled merges (whose
// results are read again by the next merge) twice as slow.
typedef double v2d __attribute__((ext_vector_type(2)));

__device__ __forceinline__ double2 ld_nt(const double2 *p)
{
    const v2d v = __builtin_nontemporal_load(reinterpret_cast<const v2d *>(p));
    return make_double2(v.x, v.y);
}

__device__ __forceinline__ void st_nt(double2 *p, double2 v)
{
    v2d w;
    w.x = v.x;
    w.y = v.y;
    __builtin_nontemporal_store(w, reinterpret_cast<v2d *>(p));
}

__device__ __forceinline__ uint64_t deposit(uint64_t v, int nbits, const uint8_t *pos)
{
    uint64_t r = 0;
    for (int j = 0; j < nbits; ++j) r |= ((v >> j) & 1ull) << pos[j];
    return r;
}

// The bits of storage index a at positions pos[0..nbits) (inverse of deposit).
__device__ __forceinline__ uint64_t extract(uint64_t a, int nbits, const uint8_t *pos)
{
    uint64_t r = 0;
    for (int j = 0; j < nbits; ++j) r |= ((a >> pos[j]) & 1ull) << j;
    return r;
}

// Start of operand row (b, o) and the stride between its summed entries:
// k lowest ((b << no | o) << nk, stride 1) or own lowest ((b << nk) << no | o,
// stride 2^no).
__device__ __forceinline__ uint64_t row_start(uint64_t b, uint64_t o, int no, int nk, int own_low)
{
    return own_low ? (((b << nk) << no) | o) : (((b << no) | o) << nk);
}

__device__ __forceinline__ void cmac(double2 &acc, double2 a, double2 b)
{
    acc.x = fma(a.x, b.x, acc.x);
    acc.x = fma(-a.y, b.y, acc.x);
    acc.y = fma(a.x, b.y, acc.y);
    acc.y = fma(a.y, b.x, acc.y);
}

// One thread per result element (few summed vertices), walked in the
// result's storage order: the writes of a wave are contiguous, and each
// thread reads its own rows of X and Y (2^nk neighbouring entries each).
__global__ __launch_bounds__(kT) void k_sa_thread(SaContract c)
{
    const int nr = c.nb + c.nm + c.nn;
    const uint64_t per = 1ull << nr, total = uint64_t(c.nbt) * per, K = 1ull << c.nk;
    for (uint64_t i = uint64_t(blockIdx.x) * kT + threadIdx.x; i < total; i += uint64_t(gridDim.x) * kT) {
        const uint64_t t = i >> nr, a = i & (per - 1);
        const uint64_t b = extract(a, c.nb, c.pb), m = extract(a, c.nm, c.pm), n = extract(a, c.nn, c.pn);
        const double2 *xp = c.x + t * c.sx + row_start(b, m, c.nm, c.nk, c.xo);
        const double2 *yp = c.y + t * c.sy + row_start(b, n, c.nn, c.nk, c.yo);
        const uint64_t kx = c.xo ? (1ull << c.nm) : 1ull, ky = c.yo ? (1ull << c.nn) : 1ull;
        double2 acc = make_double2(0.0, 0.0);
        for (uint64_t k = 0; k < K; ++k) cmac(acc, xp[k * kx], yp[k * ky]);
        c.z[t * c.sz + a] = acc;
    }
}

// Offset of operand row start for storage index a of the result: the
// row of X (Y) is a linear function of the bits of a (each bit of b, m or n
// lands on one bit of the row index), so offsets of disjoint bit fields add.
__device__ __forceinline__ uint64_t x_row(const SaContract &c, uint64_t a)
{
    return row_start(extract(a, c.nb, c.pb), extract(a, c.nm, c.pm), c.nm, c.nk, c.xo);
}

__device__ __forceinline__ uint64_t y_row(const SaContract &c, uint64_t a)
{
    return row_start(extract(a, c.nb, c.pb), extract(a, c.nn, c.pn), c.nn, c.nk, c.yo);
}

// The per-result form for results of at least 2^8 entries: a wave takes
// blocks of 256 consecutive results (storage order), R = 4 per lane, lane l
// and step r on result 64 r + l of the block.  The row offsets of the block
// (its high bits and batch element, uniform over the wave) come from the
// scalar units once per block; those of the lane bits and of the step bits
// are computed once per kernel, so a result costs a few additions instead
// of a walk over its bits.  NK > 0 fixes the number of summed vertices
// (1-3); the loads of several results of a lane are then issued before any
// product.
template <int NK>
__global__ __launch_bounds__(kT) void k_sa_rows(SaContract c)
{
    constexpr int R = 4;
    const int nr = c.nb + c.nm + c.nn, nk = NK > 0 ? NK : c.nk;
    const uint64_t per = 1ull << nr, K = 1ull << nk;
    const uint64_t blocks = (uint64_t(c.nbt) * per) >> 8;
    const uint64_t kx = c.xo ? (1ull << c.nm) : 1ull, ky = c.yo ? (1ull << c.nn) : 1ull;
    const double2 *__restrict__ X = c.x;
    const double2 *__restrict__ Y = c.y;
    double2 *__restrict__ Z = c.z;
    const uint32_t lane = threadIdx.x & 63;
    const uint64_t lx = x_row(c, lane), ly = y_row(c, lane);
    uint64_t rx[R], ry[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        rx[r] = x_row(c, uint64_t(r) << 6);
        ry[r] = y_row(c, uint64_t(r) << 6);
    }
    const uint64_t w0 = __builtin_amdgcn_readfirstlane(blockIdx.x * (kT / 64) + (threadIdx.x >> 6));
    const uint64_t nw = uint64_t(gridDim.x) * (kT / 64);
    for (uint64_t w = w0; w < blocks; w += nw) {
        const uint64_t i0 = w << 8, t = i0 >> nr, a0 = i0 & (per - 1);
        const double2 *xb = X + t * c.sx + x_row(c, a0) + lx;
        const double2 *yb = Y + t * c.sy + y_row(c, a0) + ly;
        double2 *zb = Z + t * c.sz + a0 + lane;
        if constexpr (NK > 0) {
            // G results at a time, 2 G 2^NK loads (16) in flight
            constexpr int KK = 1 << NK, G = NK == 1 ? 4 : NK == 2 ? 2 : 1;
#pragma unroll
            for (int r0 = 0; r0 < R; r0 += G) {
                double2 xv[G][KK], yv[G][KK];
#pragma unroll
                for (int g = 0; g < G; ++g)
#pragma unroll
                    for (int k = 0; k < KK; ++k) {
                        xv[g][k] = xb[rx[r0 + g] + k * kx];
                        yv[g][k] = yb[ry[r0 + g] + k * ky];
                    }
#pragma unroll
                for (int g = 0; g < G; ++g) {
                    double2 acc = make_double2(0.0, 0.0);
#pragma unroll
                    for (int k = 0; k < KK; ++k) cmac(acc, xv[g][k], yv[g][k]);
                    st_nt(zb + ((r0 + g) << 6), acc);
                }
            }
        } else {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                double2 acc = make_double2(0.0, 0.0);
                for (uint64_t k = 0; k < K; ++k) cmac(acc, xb[rx[r] + k * kx], yb[ry[r] + k * ky]);
                zb[r << 6] = acc;
            }
        }
    }
}

// One summed vertex stored lowest in Y (its two entries of a row adjacent)
// with the result's six lowest storage bits Y's own lowest vertices in
// order: the rows of 64 consecutive results are then 128 consecutive
// entries of Y, and X's row is the same for all 64.  Lane l reads entries
// l and 64 + l of that run (whole 1 KiB lines per instruction, where a lane
// per result would read its two entries at a 32-byte stride), multiplies by
// X's entry k = l & 1, and adds its neighbour's product: lane 2j then holds
// result j and lane 2j + 1 result 32 + j.  Block structure as k_sa_rows;
// Y's reads and Z's writes are non-temporal.
__global__ __launch_bounds__(kT) void k_sa_pairs(SaContract c)
{
    constexpr int R = 4;
    const int nr = c.nb + c.nm + c.nn;
    const uint64_t per = 1ull << nr;
    const uint64_t blocks = (uint64_t(c.nbt) * per) >> 8;
    const uint64_t kx = c.xo ? (1ull << c.nm) : 1ull;
    const double2 *__restrict__ X = c.x;
    const double2 *__restrict__ Y = c.y;
    double2 *__restrict__ Z = c.z;
    const uint32_t lane = threadIdx.x & 63, k = lane & 1;
    const uint32_t zl = (lane >> 1) + (k << 5);  // result of this lane within 64
    uint64_t rx[R], ry[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        rx[r] = x_row(c, uint64_t(r) << 6);
        ry[r] = y_row(c, uint64_t(r) << 6);
    }
    const uint64_t w0 = __builtin_amdgcn_readfirstlane(blockIdx.x * (kT / 64) + (threadIdx.x >> 6));
    const uint64_t nw = uint64_t(gridDim.x) * (kT / 64);
    for (uint64_t w = w0; w < blocks; w += nw) {
        const uint64_t i0 = w << 8, t = i0 >> nr, a0 = i0 & (per - 1);
        const double2 *xb = X + t * c.sx + x_row(c, a0) + k * kx;
        const double2 *yb = Y + t * c.sy + y_row(c, a0) + lane;
        double2 *zb = Z + t * c.sz + a0 + zl;
        double2 e1[R], e2[R], xv[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            e1[r] = ld_nt(yb + ry[r]);
            e2[r] = ld_nt(yb + ry[r] + 64);
            xv[r] = xb[rx[r]];
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            double2 p1 = make_double2(0.0, 0.0), p2 = make_double2(0.0, 0.0);
            cmac(p1, xv[r], e1[r]);
            cmac(p2, xv[r], e2[r]);
            p1.x += __shfl_xor(p1.x, 1);
            p1.y += __shfl_xor(p1.y, 1);
            p2.x += __shfl_xor(p2.x, 1);
            p2.y += __shfl_xor(p2.y, 1);
            st_nt(zb + (r << 6), k ? p2 : p1);
        }
    }
}

// Whether k_sa_pairs applies: one summed vertex, Y's two entries of a row
// adjacent, and the six lowest storage bits of the result Y's vertices 0..5.
// The same merge with the roles of X and Y exchanged (the product of two
// complex numbers commutes).
SaContract swapped(const SaContract &c)
{
    SaContract d = c;
    d.x = c.y;
    d.y = c.x;
    d.sx = c.sy;
    d.sy = c.sx;
    d.nm = c.nn;
    d.nn = c.nm;
    d.xo = c.yo;
    d.yo = c.xo;
    for (int j = 0; j < kSaMaxBits; ++j) {
        d.pm[j] = c.pn[j];
        d.pn[j] = c.pm[j];
    }
    return d;
}

bool pairs_layout(const SaContract &c)
{
    if (c.nk != 1 || c.yo || c.nn < 6 || c.nb + c.nm + c.nn < 8) return false;
    for (int j = 0; j < 6; ++j)
        if (c.pn[j] != j) return false;
    return true;
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// One wave per result element: lanes split the summed vertices.
__global__ __launch_bounds__(kT) void k_sa_wave(SaContract c)
{
    const int nr = c.nb + c.nm + c.nn;
    const uint64_t per = 1ull << nr, total = uint64_t(c.nbt) * per, K = 1ull << c.nk;
    const int lane = threadIdx.x & 63;
    const uint64_t nw = uint64_t(gridDim.x) * (kT / 64);
    for (uint64_t i = uint64_t(blockIdx.x) * (kT / 64) + (threadIdx.x >> 6); i < total; i += nw) {
        const uint64_t t = i >> nr, a = i & (per - 1);
        const uint64_t b = extract(a, c.nb, c.pb), m = extract(a, c.nm, c.pm), n = extract(a, c.nn, c.pn);
        const double2 *xp = c.x + t * c.sx + row_start(b, m, c.nm, c.nk, c.xo);
        const double2 *yp = c.y + t * c.sy + row_start(b, n, c.nn, c.nk, c.yo);
        const uint64_t kx = c.xo ? (1ull << c.nm) : 1ull, ky = c.yo ? (1ull << c.nn) : 1ull;
        double2 acc = make_double2(0.0, 0.0);
        for (uint64_t k = lane; k < K; k += 64) cmac(acc, xp[k * kx], yp[k * ky]);
        acc.x = wave_sum(acc.x);
        acc.y = wave_sum(acc.y);
        if (lane == 0) c.z[t * c.sz + a] = acc;
    }
}

// 64 x 64 result tiles (nm, nn >= 6, nk >= 3): the summed vertices are
// walked eight at a time through LDS, each thread accumulates 4 x 4 results
// (rows 4 ty .. 4 ty + 3, columns tx + 16 j, so that the lanes of a wave
// read neighbouring LDS entries and write neighbouring results).
__global__ __launch_bounds__(kT) void k_sa_tile(SaContract c)
{
    __shared__ double2 xs[8][65];  // one spare entry per row: the eight rows written together
    __shared__ double2 ys[8][65];  // (consecutive threads, stride 1040 B) fall on different banks
    const uint64_t mt = 1ull << (c.nm - 6), nt = 1ull << (c.nn - 6);
    const uint64_t tiles_per = mt * nt;
    const uint64_t total = uint64_t(c.nbt) * (1ull << c.nb) * tiles_per;
    const uint64_t K = 1ull << c.nk;
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    // Workgroups are dealt to the eight XCDs in turn (block i to XCD i mod 8),
    // each with its own L2.  When the result's lowest storage bits are shared
    // vertices (bfast), the eight neighbouring b of one line of results are
    // given to blocks eight apart, which run on one XCD at about the same
    // time, so their partial writes of each line meet in one L2.
    const bool swap = c.bfast && c.nb >= 3 && (total & 63) == 0;
    for (uint64_t blk = blockIdx.x; blk < total; blk += gridDim.x) {
        const uint64_t tile = swap ? ((blk & ~uint64_t(63)) | ((blk & 7) << 3) | ((blk >> 3) & 7)) : blk;
        uint64_t t, b, r;
        if (c.bfast) {
            // the result's lowest storage bits are shared vertices: workgroups
            // running together take neighbouring b, whose writes share lines
            b = tile & ((1ull << c.nb) - 1);
            const uint64_t rest = tile >> c.nb;
            t = rest / tiles_per;
            r = rest % tiles_per;
        } else {
            const uint64_t tb = tile / tiles_per;
            r = tile % tiles_per;
            t = tb >> c.nb;
            b = tb & ((1ull << c.nb) - 1);
        }
        const uint64_t m0 = (r / nt) << 6, n0 = (r % nt) << 6;
        const double2 *xp = c.x + t * c.sx + row_start(b, m0, c.nm, c.nk, c.xo);
        const double2 *yp = c.y + t * c.sy + row_start(b, n0, c.nn, c.nk, c.yo);
        double2 acc[4][4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[i][j] = make_double2(0.0, 0.0);
        // 512 entries per operand and k-step: with k lowest, eight
        // neighbouring lanes read one row's eight summed entries; with the
        // own index lowest, 64 neighbouring lanes read one summed entry of 64
        // rows.  A thread's four loads are issued together (addresses by
        // select, no load under a branch), and the next k-step's are in
        // flight while this one is multiplied.
        const int e0 = int(threadIdx.x), e1 = int(threadIdx.x) + kT;
        auto xat = [&](uint64_t k0, int e) -> uint64_t {
            return c.xo ? (((k0 + uint64_t(e >> 6)) << c.nm) + uint64_t(e & 63))
                        : ((uint64_t(e >> 3) << c.nk) + k0 + uint64_t(e & 7));
        };
        auto yat = [&](uint64_t k0, int e) -> uint64_t {
            return c.yo ? (((k0 + uint64_t(e >> 6)) << c.nn) + uint64_t(e & 63))
                        : ((uint64_t(e >> 3) << c.nk) + k0 + uint64_t(e & 7));
        };
        double2 x0 = xp[xat(0, e0)], x1 = xp[xat(0, e1)], y0 = yp[yat(0, e0)], y1 = yp[yat(0, e1)];
        // LDS slot of entry e: [k][row]
        const int xk0 = c.xo ? e0 >> 6 : e0 & 7, xr0 = c.xo ? e0 & 63 : e0 >> 3;
        const int xk1 = c.xo ? e1 >> 6 : e1 & 7, xr1 = c.xo ? e1 & 63 : e1 >> 3;
        const int yk0 = c.yo ? e0 >> 6 : e0 & 7, yr0 = c.yo ? e0 & 63 : e0 >> 3;
        const int yk1 = c.yo ? e1 >> 6 : e1 & 7, yr1 = c.yo ? e1 & 63 : e1 >> 3;
        for (uint64_t k0 = 0; k0 < K; k0 += 8) {
            xs[xk0][xr0] = x0;
            xs[xk1][xr1] = x1;
            ys[yk0][yr0] = y0;
            ys[yk1][yr1] = y1;
            if (k0 + 8 < K) {
                x0 = xp[xat(k0 + 8, e0)];
                x1 = xp[xat(k0 + 8, e1)];
                y0 = yp[yat(k0 + 8, e0)];
                y1 = yp[yat(k0 + 8, e1)];
            }
            __syncthreads();
#pragma unroll
            for (int kk = 0; kk < 8; ++kk) {
                double2 a[4], bb[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    a[i] = xs[kk][ty * 4 + i];
                    bb[i] = ys[kk][tx + 16 * i];  // neighbouring lanes, neighbouring entries
                }
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j) cmac(acc[i][j], a[i], bb[j]);
            }
            __syncthreads();
        }
        const uint64_t zb = t * c.sz + deposit(b, c.nb, c.pb);
        uint64_t zm[4], zn[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            zm[i] = deposit(m0 + ty * 4 + i, c.nm, c.pm);
            zn[i] = deposit(n0 + tx + 16 * i, c.nn, c.pn);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) c.z[zb + zm[i] + zn[j]] = acc[i][j];
    }
}

__global__ __launch_bounds__(kT) void k_sa_prep(SaPrep p, const uint64_t *__restrict__ bits)
{
    const uint64_t per = 1ull << p.r, total = uint64_t(p.nbt) * per;
    for (uint64_t i = uint64_t(blockIdx.x) * kT + threadIdx.x; i < total; i += uint64_t(gridDim.x) * kT) {
        const uint64_t t = i >> p.r, f = i & (per - 1);
        const uint64_t w = t / p.slices, s = t % p.slices;
        uint64_t a = deposit(f, p.r, p.src);
        for (int j = 0; j < p.nf; ++j) {
            uint64_t v = 0;
            if (p.fkind[j] == 1) v = (bits[w] >> p.fwhich[j]) & 1ull;
            else if (p.fkind[j] == 2) v = (s >> p.fwhich[j]) & 1ull;
            a |= v << p.fpos[j];
        }
        p.out[t * p.so + f] = p.base[a];
    }
}

__global__ __launch_bounds__(kT) void k_sa_finish(const double2 *const *__restrict__ scal,
                                                  const uint64_t *__restrict__ strides, int nscal,
                                                  uint32_t words, uint32_t slices,
                                                  const uint64_t *__restrict__ bits, uint64_t idle, double2 *out)
{
    const uint32_t w = blockIdx.x * kT + threadIdx.x;
    if (w >= words) return;
    if (bits[w] & idle) {
        out[w] = make_double2(0.0, 0.0);
        return;
    }
    double2 acc = make_double2(0.0, 0.0);
    for (uint32_t s = 0; s < slices; ++s) {
        const uint64_t t = uint64_t(w) * slices + s;
        double2 pr = make_double2(1.0, 0.0);
        for (int c = 0; c < nscal; ++c) {
            const double2 v = scal[c][t * strides[c]];
            pr = make_double2(pr.x * v.x - pr.y * v.y, pr.x * v.y + pr.y * v.x);
        }
        acc.x += pr.x;
        acc.y += pr.y;
    }
    out[w] = acc;
}

uint32_t grid_of(uint64_t work, uint64_t per_block)
{
    const uint64_t g = (work + per_block - 1) / per_block;
    return uint32_t(g < 1 ? 1 : (g > (1u << 20) ? (1u << 20) : g));
}

// Workgroups of the block-walking kernels (k_sa_rows, k_sa_pairs): one
// 256-result block per wave and pass, at most 2048 workgroups (eight per
// compute unit of 256), so that each wave's set-up (its lane and step
// offsets, one walk over the result's bits each) is spread over many blocks.
uint32_t block_grid(uint64_t outs)
{
    const uint64_t g = (outs + 4 * kT - 1) / (4 * kT);
    return uint32_t(g < 1 ? 1 : (g > 2048 ? 2048 : g));
}

}  // namespace

hipError_t launch_sa_prep(const SaPrep &p, const uint64_t *bits, hipStream_t st)
{
    const uint64_t total = uint64_t(p.nbt) << p.r;
    hipLaunchKernelGGL(k_sa_prep, dim3(grid_of(total, kT)), dim3(kT), 0, st, p, bits);
    return hipGetLastError();
}

hipError_t launch_sa_contract(const SaContract &c, int kernel, hipStream_t st)
{
    const uint64_t outs = uint64_t(c.nbt) << (c.nb + c.nm + c.nn);
    if (kernel == SA_TILE) {
        if (c.nm < 6 || c.nn < 6 || c.nk < 3) return hipErrorInvalidValue;
        hipLaunchKernelGGL(k_sa_tile, dim3(grid_of(outs, 4096)), dim3(kT), 0, st, c);
    } else if (kernel == SA_WAVE) {
        hipLaunchKernelGGL(k_sa_wave, dim3(grid_of(outs, kT / 64)), dim3(kT), 0, st, c);
    } else if (pairs_layout(c)) {
        hipLaunchKernelGGL(k_sa_pairs, dim3(block_grid(outs)), dim3(kT), 0, st, c);
    } else if (pairs_layout(swapped(c))) {
        hipLaunchKernelGGL(k_sa_pairs, dim3(block_grid(outs)), dim3(kT), 0, st, swapped(c));
    } else if (c.nb + c.nm + c.nn >= 8) {
        const uint32_t g = block_grid(outs);
        switch (c.nk) {
        case 1: hipLaunchKernelGGL(k_sa_rows<1>, dim3(g), dim3(kT), 0, st, c); break;
        case 2: hipLaunchKernelGGL(k_sa_rows<2>, dim3(g), dim3(kT), 0, st, c); break;
        case 3: hipLaunchKernelGGL(k_sa_rows<3>, dim3(g), dim3(kT), 0, st, c); break;
        default: hipLaunchKernelGGL(k_sa_rows<0>, dim3(g), dim3(kT), 0, st, c); break;
        }
    } else {
        hipLaunchKernelGGL(k_sa_thread, dim3(grid_of(outs, kT)), dim3(kT), 0, st, c);
    }
    return hipGetLastError();
}

hipError_t launch_sa_finish(const double2 *const *scal, const uint64_t *strides, int nscal, uint32_t words,
                            uint32_t slices, const uint64_t *bits, uint64_t idle, double2 *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_sa_finish, dim3((words + kT - 1) / kT), dim3(kT), 0, st, scal, strides, nscal, words,
                       slices, bits, idle, out);
    return hipGetLastError();
}

}  // namespace qs
