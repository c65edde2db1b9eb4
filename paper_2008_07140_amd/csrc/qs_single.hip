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
        for (uint64_t k0 = 0; k0 < K; k0 += 8) {
            // 512 entries per operand: with k lowest, eight neighbouring lanes
            // read one row's eight summed entries; with the own index lowest,
            // 64 neighbouring lanes read one summed entry of 64 rows
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int e = threadIdx.x + h * kT;
                if (c.xo) {
                    const int row = e & 63, kk = e >> 6;
                    xs[kk][row] = xp[((k0 + kk) << c.nm) + row];
                } else {
                    const int row = e >> 3, kk = e & 7;
                    xs[kk][row] = xp[(uint64_t(row) << c.nk) + k0 + kk];
                }
                if (c.yo) {
                    const int row = e & 63, kk = e >> 6;
                    ys[kk][row] = yp[((k0 + kk) << c.nn) + row];
                } else {
                    const int row = e >> 3, kk = e & 7;
                    ys[kk][row] = yp[(uint64_t(row) << c.nk) + k0 + kk];
                }
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
