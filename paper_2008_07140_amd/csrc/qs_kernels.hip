// HIP kernels for gfx950 (MI355X): per-gate sweeps, diagonal gates, FP64
// reductions.  Amplitudes are interleaved complex (double2 / float2), qubit k
// = bit k of the index (Sec. 2.2, Eq. 1).
//
// Every gate kernel enumerates the 2^(n - npos) groups of amplitudes that a
// gate mixes (the "i_k = 0" enumeration of Eq. 2 plus the control condition of
// Eq. 3): consecutive lanes take consecutive work items, so for every target
// position the lanes of a wavefront read contiguous runs of amplitudes and
// the two (or 2^nt) streams of a group are each coalesced.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "qs_internal.h"

namespace qs {

namespace {

constexpr int kBlock = 256;
constexpr uint64_t kMaxBlocks = 1u << 22;  // grid-stride above this (grid * 256 < 2^32)

__device__ __forceinline__ uint64_t insert_zeros(uint64_t t, const IdxSpec &ix)
{
    for (int k = 0; k < ix.npos; ++k) {
        const uint64_t lo = t & ((uint64_t(1) << ix.pos[k]) - 1);
        t = ((t ^ lo) << 1) | lo;
    }
    return t | ix.set;
}

// Chunk of a streaming kernel's grid-stride step c0.  Workgroups are dealt
// to the eight XCDs in turn (block b to XCD b mod 8, and the grid is a
// multiple of 8 or equals the chunk count), so with 8 | nchunks XCD x takes
// the x-th eighth of the chunks in order: each XCD streams one contiguous
// eighth of the state instead of every eighth chunk of all of it (measured
// on single-target complex128 sweeps of 30 qubits: 6.0 against 5.75 TB/s).
// A bijection of [0, nchunks) either way.
__device__ __forceinline__ uint64_t xcd_chunk(uint64_t c0, uint64_t nchunks)
{
    return (nchunks & 7) ? c0 : ((c0 & 7) * (nchunks >> 3) + (c0 >> 3));
}

template <typename C, typename R>
__device__ __forceinline__ C cmul(R ar, R ai, C b)
{
    C r;
    r.x = ar * b.x - ai * b.y;
    r.y = ar * b.y + ai * b.x;
    return r;
}

template <typename C, typename R>
__device__ __forceinline__ void cfma(C &acc, R ar, R ai, C b)
{
    acc.x += ar * b.x - ai * b.y;
    acc.y += ar * b.y + ai * b.x;
}

uint64_t grid_for(uint64_t items, uint64_t per_block)
{
    uint64_t g = (items + per_block - 1) / per_block;
    if (g == 0) g = 1;
    return g < kMaxBlocks ? g : kMaxBlocks;
}

// ------------------------------------------------------------------ init --

template <typename R>
__global__ __launch_bounds__(kBlock) void k_init(typename Cpx<R>::T *a, uint64_t n_amp)
{
    using C = typename Cpx<R>::T;
    const uint64_t stride = uint64_t(gridDim.x) * kBlock;
    for (uint64_t i = uint64_t(blockIdx.x) * kBlock + threadIdx.x; i < n_amp; i += stride) {
        C v;
        v.x = (i == 0) ? R(1) : R(0);
        v.y = R(0);
        a[i] = v;
    }
}

template <typename R>
__global__ __launch_bounds__(kBlock) void k_scale(typename Cpx<R>::T *a, uint64_t n_amp, R s)
{
    const uint64_t stride = uint64_t(gridDim.x) * kBlock;
    for (uint64_t i = uint64_t(blockIdx.x) * kBlock + threadIdx.x; i < n_amp; i += stride) {
        auto v = a[i];
        v.x *= s;
        v.y *= s;
        a[i] = v;
    }
}

// Streaming loads and stores of amplitudes.  A gate sweep touches every
// amplitude once, so the accesses are marked non-temporal (no reuse).
template <typename R>
struct Vec2;
template <>
struct Vec2<double> {
    typedef double T __attribute__((ext_vector_type(2)));
};
template <>
struct Vec2<float> {
    typedef float T __attribute__((ext_vector_type(2)));
};

template <typename C>
__device__ __forceinline__ C ld_stream(const C *p)
{
    using R = decltype(C().x);
    using V = typename Vec2<R>::T;
    const V v = __builtin_nontemporal_load(reinterpret_cast<const V *>(p));
    C c;
    c.x = v.x;
    c.y = v.y;
    return c;
}

template <typename C>
__device__ __forceinline__ void st_stream(C *p, C c)
{
    using R = decltype(C().x);
    using V = typename Vec2<R>::T;
    V v;
    v.x = c.x;
    v.y = c.y;
    __builtin_nontemporal_store(v, reinterpret_cast<V *>(p));
}

// ------------------------------------------------------ one target, Eq. 2 --
// U pairs per thread: all loads are issued before any store so that 2U
// independent requests are in flight per lane.

template <typename C, bool NT>
__device__ __forceinline__ C ld_amp(const C *p)
{
    if constexpr (NT) return ld_stream(p);
    else return *p;
}

template <typename C, bool NT>
__device__ __forceinline__ void st_amp(C *p, C v)
{
    if constexpr (NT) st_stream(p, v);
    else *p = v;
}

// Non-temporal accesses pay off only when every 128-byte line a wavefront
// touches is fully used by one instruction: the lowest inserted bit must
// leave contiguous runs of at least 128 bytes.
template <typename R>
bool stream_ok(const IdxSpec &ix)
{
    const int need = sizeof(R) == 8 ? 3 : 4;  // 2^need amplitudes = 128 bytes
    for (int k = 0; k < ix.npos; ++k)
        if (ix.pos[k] < need) return false;
    return true;
}

template <typename R, int U, bool NT>
__global__ __launch_bounds__(kBlock) void k_dense1(typename Cpx<R>::T *a, uint64_t npairs,
                                                   IdxSpec ix, uint64_t tbit, MatArg<R, 2> m)
{
    using C = typename Cpx<R>::T;
    const uint64_t per = uint64_t(kBlock) * U;
    const uint64_t nchunks = (npairs + per - 1) / per;
    for (uint64_t c0 = blockIdx.x; c0 < nchunks; c0 += gridDim.x) {
        const uint64_t ch = xcd_chunk(c0, nchunks);
        const uint64_t base = ch * per + threadIdx.x;
        C x0[U], x1[U];
        uint64_t i0[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint64_t t = base + uint64_t(u) * kBlock;
            i0[u] = insert_zeros(t < npairs ? t : 0, ix);
            if (t < npairs) {
                x0[u] = ld_amp<C, NT>(a + i0[u]);
                x1[u] = ld_amp<C, NT>(a + (i0[u] | tbit));
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint64_t t = base + uint64_t(u) * kBlock;
            if (t < npairs) {
                C y0 = cmul<C, R>(m.v[0], m.v[1], x0[u]);
                cfma<C, R>(y0, m.v[2], m.v[3], x1[u]);
                C y1 = cmul<C, R>(m.v[4], m.v[5], x0[u]);
                cfma<C, R>(y1, m.v[6], m.v[7], x1[u]);
                st_amp<C, NT>(a + i0[u], y0);
                st_amp<C, NT>(a + (i0[u] | tbit), y1);
            }
        }
    }
}

// A controlled single-target gate with a control below the 128-byte run
// length (a CU3 controlled by qubit 0, 1 or 2 of a complex128 state): the
// pairs it changes leave gaps inside every line.  Here every pair whose
// high controls (hx, with the target: positions, set = values) match is
// read and written back whole-line, non-temporal, and transformed only
// where its low control bits (lmask) read lval.
template <typename R>
__global__ __launch_bounds__(kBlock) void k_dense1_runs(typename Cpx<R>::T *a, uint64_t npairs, IdxSpec hx,
                                                        uint64_t tbit, uint64_t lmask, uint64_t lval,
                                                        MatArg<R, 2> m)
{
    using C = typename Cpx<R>::T;
    constexpr int U = 2;
    const uint64_t per = uint64_t(kBlock) * U;
    const uint64_t nchunks = (npairs + per - 1) / per;
    for (uint64_t c0 = blockIdx.x; c0 < nchunks; c0 += gridDim.x) {
        const uint64_t ch = xcd_chunk(c0, nchunks);
        const uint64_t base = ch * per + threadIdx.x;
        C x0[U], x1[U];
        uint64_t i0[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint64_t t = base + uint64_t(u) * kBlock;
            i0[u] = insert_zeros(t < npairs ? t : 0, hx);
            if (t < npairs) {
                x0[u] = ld_stream(a + i0[u]);
                x1[u] = ld_stream(a + (i0[u] | tbit));
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (base + uint64_t(u) * kBlock >= npairs) continue;
            C y0 = x0[u], y1 = x1[u];
            if ((i0[u] & lmask) == lval) {
                y0 = cmul<C, R>(m.v[0], m.v[1], x0[u]);
                cfma<C, R>(y0, m.v[2], m.v[3], x1[u]);
                y1 = cmul<C, R>(m.v[4], m.v[5], x0[u]);
                cfma<C, R>(y1, m.v[6], m.v[7], x1[u]);
            }
            st_stream(a + i0[u], y0);
            st_stream(a + (i0[u] | tbit), y1);
        }
    }
}

// Target below 6 (its partner lies in the same wavefront) and no control
// below 6: lane l of a wavefront holds amplitude i with the low six bits of i
// equal to l, so every load and store is one contiguous run; the partner
// amplitude alpha_{i ^ 2^k} comes from lane l ^ 2^k by a cross-lane shuffle.
template <typename R, int U>
__global__ __launch_bounds__(kBlock) void k_dense1_lane(typename Cpx<R>::T *a, uint64_t nitems,
                                                        IdxSpec ix, int k, MatArg<R, 2> m)
{
    using C = typename Cpx<R>::T;
    const uint64_t per = uint64_t(kBlock) * U;
    const uint64_t nchunks = (nitems + per - 1) / per;
    const int lane_bit = (threadIdx.x >> k) & 1;
    // own coefficient and partner coefficient of the output row of this lane
    const R sr = lane_bit ? m.v[6] : m.v[0], si = lane_bit ? m.v[7] : m.v[1];
    const R pr = lane_bit ? m.v[4] : m.v[2], pi = lane_bit ? m.v[5] : m.v[3];
    const int xmask = 1 << k;
    for (uint64_t c0 = blockIdx.x; c0 < nchunks; c0 += gridDim.x) {
        const uint64_t ch = xcd_chunk(c0, nchunks);
        const uint64_t base = ch * per + threadIdx.x;
        C x[U];
        uint64_t idx[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint64_t t = base + uint64_t(u) * kBlock;
            idx[u] = insert_zeros(t < nitems ? t : 0, ix);
            if (t < nitems) x[u] = ld_stream(a + idx[u]);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint64_t t = base + uint64_t(u) * kBlock;
            C p;
            p.x = __shfl_xor(x[u].x, xmask);
            p.y = __shfl_xor(x[u].y, xmask);
            if (t < nitems) {
                C y = cmul<C, R>(sr, si, x[u]);
                cfma<C, R>(y, pr, pi, p);
                st_stream(a + idx[u], y);
            }
        }
    }
}

// ---------------------------------------------------- 2 and 3 targets --

template <typename R, int NT, int U, bool STREAM>
__global__ __launch_bounds__(kBlock) void k_dense_small(typename Cpx<R>::T *a, uint64_t ngroups,
                                                        IdxSpec ix, MatArg<R, (1 << NT)> m,
                                                        int tq0, int tq1, int tq2)
{
    using C = typename Cpx<R>::T;
    constexpr int D = 1 << NT;
    const int tq[3] = {tq0, tq1, tq2};
    uint64_t off[D];
#pragma unroll
    for (int x = 0; x < D; ++x) {
        uint64_t o = 0;
#pragma unroll
        for (int b = 0; b < NT; ++b)
            if ((x >> (NT - 1 - b)) & 1) o |= uint64_t(1) << tq[b];
        off[x] = o;
    }
    const uint64_t per = uint64_t(kBlock) * U;
    const uint64_t nchunks = (ngroups + per - 1) / per;
    for (uint64_t c0 = blockIdx.x; c0 < nchunks; c0 += gridDim.x) {
        const uint64_t ch = xcd_chunk(c0, nchunks);
        const uint64_t base = ch * per + threadIdx.x;
        C v[U][D];
        uint64_t i0[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint64_t t = base + uint64_t(u) * kBlock;
            i0[u] = insert_zeros(t < ngroups ? t : 0, ix);
            if (t < ngroups) {
#pragma unroll
                for (int x = 0; x < D; ++x) v[u][x] = ld_amp<C, STREAM>(a + (i0[u] | off[x]));
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint64_t t = base + uint64_t(u) * kBlock;
            if (t < ngroups) {
#pragma unroll
                for (int r = 0; r < D; ++r) {
                    C acc;
                    acc.x = R(0);
                    acc.y = R(0);
#pragma unroll
                    for (int c = 0; c < D; ++c)
                        cfma<C, R>(acc, m.v[2 * (r * D + c)], m.v[2 * (r * D + c) + 1], v[u][c]);
                    st_amp<C, STREAM>(a + (i0[u] | off[r]), acc);
                }
            }
        }
    }
}

// ------------------------------------------------------ 4 to 6 targets --
// A block loads its matrix into LDS once, then processes G = 256 / 2^NT
// groups per step: lane (x, g) loads amplitude x of group g into LDS, and
// after a barrier computes row x of group g.

template <typename R, int NT>
__global__ __launch_bounds__(kBlock) void k_denseN(typename Cpx<R>::T *a, uint64_t ngroups,
                                                   IdxSpec ix, const typename Cpx<R>::T *mat,
                                                   int tq0, int tq1, int tq2, int tq3, int tq4,
                                                   int tq5)
{
    using C = typename Cpx<R>::T;
    constexpr int D = 1 << NT;
    constexpr int G = kBlock / D;
    __shared__ C sm[D * D];
    __shared__ C tile[kBlock];
    const int tq[6] = {tq0, tq1, tq2, tq3, tq4, tq5};
    for (int k = threadIdx.x; k < D * D; k += kBlock) sm[k] = mat[k];
    const int g = threadIdx.x % G;
    const int x = threadIdx.x / G;
    uint64_t offx = 0;
    for (int b = 0; b < NT; ++b)
        if ((x >> (NT - 1 - b)) & 1) offx |= uint64_t(1) << tq[b];
    const uint64_t nsteps = (ngroups + G - 1) / G;
    for (uint64_t s = blockIdx.x; s < nsteps; s += gridDim.x) {
        const uint64_t grp = s * G + g;
        const bool ok = grp < ngroups;
        const uint64_t idx = insert_zeros(ok ? grp : 0, ix) | offx;
        __syncthreads();
        if (ok) tile[g * D + x] = a[idx];
        __syncthreads();
        if (ok) {
            C acc;
            acc.x = R(0);
            acc.y = R(0);
            for (int c = 0; c < D; ++c) {
                const C mm = sm[x * D + c];
                cfma<C, R>(acc, mm.x, mm.y, tile[g * D + c]);
            }
            a[idx] = acc;
        }
    }
}

// ------------------------------------------------------------- diagonal --
// The amplitudes whose control bits are 1 are multiplied by d[x], x = the
// pattern of the (at most 3) remaining target bits; factors equal to 1 are
// skipped, so only changed amplitudes are read and written.

template <typename R, int U, bool STREAM>
__global__ __launch_bounds__(kBlock) void k_phase(typename Cpx<R>::T *a, uint64_t ngroups,
                                                  IdxSpec ix, DiagArg<R> d)
{
    using C = typename Cpx<R>::T;
    const int D = 1 << d.nt;
    const uint64_t per = uint64_t(kBlock) * U;
    const uint64_t nchunks = (ngroups + per - 1) / per;
    for (uint64_t c0 = blockIdx.x; c0 < nchunks; c0 += gridDim.x) {
        const uint64_t ch = xcd_chunk(c0, nchunks);
        const uint64_t base = ch * per + threadIdx.x;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint64_t t = base + uint64_t(u) * kBlock;
            if (t >= ngroups) continue;
            const uint64_t i0 = insert_zeros(t, ix);
            for (int x = 0; x < D; ++x) {
                if (!((d.active >> x) & 1)) continue;
                uint64_t o = 0;
                for (int b = 0; b < d.nt; ++b)
                    if ((x >> (d.nt - 1 - b)) & 1) o |= uint64_t(1) << d.tq[b];
                const C v = ld_amp<C, STREAM>(a + (i0 | o));
                st_amp<C, STREAM>(a + (i0 | o), cmul<C, R>(d.v[2 * x], d.v[2 * x + 1], v));
            }
        }
    }
}

// The common diagonal gate: one factor f != 1 on the amplitudes whose bits
// in ix.pos read `o` (CZ, T, S, Z, CR after canonicalisation: all their
// qubits are controls and the table has one entry).  U groups per thread,
// all loads issued before any multiply or store, so each thread keeps U
// amplitudes in flight (a load-multiply-store per group would wait on every
// load, as the stores may alias the next loads).
template <typename R, int U, bool STREAM>
__global__ __launch_bounds__(kBlock) void k_phase1(typename Cpx<R>::T *a, uint64_t ngroups, IdxSpec ix,
                                                   uint64_t o, R fr, R fi)
{
    using C = typename Cpx<R>::T;
    const uint64_t per = uint64_t(kBlock) * U;
    const uint64_t nchunks = (ngroups + per - 1) / per;
    for (uint64_t c0 = blockIdx.x; c0 < nchunks; c0 += gridDim.x) {
        const uint64_t ch = xcd_chunk(c0, nchunks);
        const uint64_t base = ch * per + threadIdx.x;
        uint64_t idx[U];
        C v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint64_t t = base + uint64_t(u) * kBlock;
            idx[u] = insert_zeros(t < ngroups ? t : 0, ix) | o;
            if (t < ngroups) v[u] = ld_amp<C, STREAM>(a + idx[u]);
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (base + uint64_t(u) * kBlock < ngroups) st_amp<C, STREAM>(a + idx[u], cmul<C, R>(fr, fi, v[u]));
    }
}

// The same gate when a condition bit lies below the 128-byte run length
// (CZ or T with a qubit among the lowest three of a complex128 state): the
// amplitudes it changes leave gaps inside every line, and reading and
// writing only them moves whole sectors at partial-line rates.  Here every
// amplitude whose high condition bits (hx: positions, set = their values)
// match is read and written back whole-line, non-temporal, multiplied by f
// only where its low condition bits (lmask) read lval.
template <typename R, int U>
__global__ __launch_bounds__(kBlock) void k_phase1_runs(typename Cpx<R>::T *a, uint64_t nitems, IdxSpec hx,
                                                        uint64_t lmask, uint64_t lval, R fr, R fi)
{
    using C = typename Cpx<R>::T;
    const uint64_t per = uint64_t(kBlock) * U;
    const uint64_t nchunks = (nitems + per - 1) / per;
    for (uint64_t c0 = blockIdx.x; c0 < nchunks; c0 += gridDim.x) {
        const uint64_t ch = xcd_chunk(c0, nchunks);
        const uint64_t base = ch * per + threadIdx.x;
        uint64_t idx[U];
        C v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint64_t t = base + uint64_t(u) * kBlock;
            idx[u] = insert_zeros(t < nitems ? t : 0, hx);
            if (t < nitems) v[u] = ld_stream(a + idx[u]);
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (base + uint64_t(u) * kBlock < nitems)
                st_stream(a + idx[u], (idx[u] & lmask) == lval ? cmul<C, R>(fr, fi, v[u]) : v[u]);
    }
}

// ----------------------------------------------------------- reductions --

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Sum of one value per thread over the block; result valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double *lds)
{
    v = wave_sum(v);
    const int w = threadIdx.x / 64, l = threadIdx.x % 64;
    __syncthreads();
    if (l == 0) lds[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < kBlock / 64; ++k) s += lds[k];
    return s;
}

constexpr uint64_t kRedBlocks = 1024;

// Per-block sums of NB bins; bin of amplitude i = its measured bits.
template <typename R, int NB>
__global__ __launch_bounds__(kBlock) void k_probs_reg(const typename Cpx<R>::T *a, uint64_t n_amp,
                                                      int nq, IdxSpec q, double *partials)
{
    // q.pos[b] = qubit of output bit (nq-1-b)
    double acc[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[b] = 0.0;
    // four amplitudes per lane and step, loaded before any is summed, so
    // that enough loads are in flight to keep HBM busy on complex64 states
    // With the grid and the state a multiple of 8 workgroups / amplitudes,
    // XCD x (workgroups x, x + 8, ...) sums the x-th eighth of the state, as
    // xcd_chunk does for the streaming kernels.
    constexpr int U = 4;
    uint64_t first = uint64_t(blockIdx.x) * kBlock + threadIdx.x, end = n_amp,
             stride = uint64_t(gridDim.x) * kBlock;
    if ((gridDim.x & 7) == 0 && (n_amp & 7) == 0) {
        const uint64_t x = blockIdx.x & 7, per = n_amp >> 3;
        first = x * per + uint64_t(blockIdx.x >> 3) * kBlock + threadIdx.x;
        end = (x + 1) * per;
        stride = uint64_t(gridDim.x >> 3) * kBlock;
    }
    for (uint64_t i0 = first; i0 < end; i0 += U * stride) {
        typename Cpx<R>::T v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint64_t i = i0 + u * stride;
            if (i < end) v[u] = a[i];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint64_t i = i0 + u * stride;
            if (i >= end) break;
            const double p = double(v[u].x) * double(v[u].x) + double(v[u].y) * double(v[u].y);
            int x = 0;
            for (int b = 0; b < nq; ++b) x = (x << 1) | int((i >> q.pos[b]) & 1);
#pragma unroll
            for (int b = 0; b < NB; ++b) acc[b] += (x == b) ? p : 0.0;
        }
    }
    __shared__ double lds[kBlock / 64];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const double s = block_sum(acc[b], lds);
        if (threadIdx.x == 0) partials[uint64_t(blockIdx.x) * NB + b] = s;
    }
}

// Larger bin counts (up to 1024): per-block LDS histogram with FP64 atomics.
template <typename R>
__global__ __launch_bounds__(kBlock) void k_probs_lds(const typename Cpx<R>::T *a, uint64_t n_amp,
                                                      int nq, IdxSpec q, double *partials)
{
    __shared__ double bins[1024];
    const int nb = 1 << nq;
    for (int b = threadIdx.x; b < nb; b += kBlock) bins[b] = 0.0;
    __syncthreads();
    const uint64_t stride = uint64_t(gridDim.x) * kBlock;
    for (uint64_t i = uint64_t(blockIdx.x) * kBlock + threadIdx.x; i < n_amp; i += stride) {
        const auto v = a[i];
        const double p = double(v.x) * double(v.x) + double(v.y) * double(v.y);
        int x = 0;
        for (int b = 0; b < nq; ++b) x = (x << 1) | int((i >> q.pos[b]) & 1);
        atomicAdd(&bins[x], p);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < nb; b += kBlock) partials[uint64_t(blockIdx.x) * nb + b] = bins[b];
}

// out[b] = sum over blocks of partials[blk][b]
__global__ __launch_bounds__(kBlock) void k_sum_columns(const double *partials, int nblk, int nb,
                                                        double *out)
{
    for (int b = blockIdx.x * kBlock + threadIdx.x; b < nb; b += gridDim.x * kBlock) {
        double s = 0.0;
        for (int k = 0; k < nblk; ++k) s += partials[uint64_t(k) * nb + b];
        out[b] = s;
    }
}

// All n qubits listed: out[x] = |alpha_i|^2 with x the permuted index.
template <typename R>
__global__ __launch_bounds__(kBlock) void k_probs_perm(const typename Cpx<R>::T *a, uint64_t n_amp,
                                                       int nq, IdxSpec q, double *out)
{
    const uint64_t stride = uint64_t(gridDim.x) * kBlock;
    for (uint64_t i = uint64_t(blockIdx.x) * kBlock + threadIdx.x; i < n_amp; i += stride) {
        const auto v = a[i];
        uint64_t x = 0;
        for (int b = 0; b < nq; ++b) x = (x << 1) | ((i >> q.pos[b]) & 1);
        out[x] = double(v.x) * double(v.x) + double(v.y) * double(v.y);
    }
}

// Between 11 and n-1 listed qubits: one thread per outcome sums its
// 2^(n - nq) amplitudes (rest = the unlisted qubits, ascending in rest).
template <typename R>
__global__ __launch_bounds__(kBlock) void k_probs_bins(const typename Cpx<R>::T *a, int nq,
                                                       IdxSpec q, IdxSpec rest, uint64_t nrest,
                                                       double *out)
{
    const uint64_t nb = uint64_t(1) << nq;
    const uint64_t stride = uint64_t(gridDim.x) * kBlock;
    for (uint64_t x = uint64_t(blockIdx.x) * kBlock + threadIdx.x; x < nb; x += stride) {
        uint64_t base = 0;
        for (int b = 0; b < nq; ++b)
            if ((x >> (nq - 1 - b)) & 1) base |= uint64_t(1) << q.pos[b];
        double s = 0.0;
        for (uint64_t r = 0; r < nrest; ++r) {
            uint64_t idx = 0;
            for (int k = 0; k < rest.npos; ++k)
                if ((r >> k) & 1) idx |= uint64_t(1) << rest.pos[k];
            const auto v = a[base | idx];
            s += double(v.x) * double(v.x) + double(v.y) * double(v.y);
        }
        out[x] = s;
    }
}

// Reduced density matrix of NT <= 2 targets.
template <typename R, int NT>
__global__ __launch_bounds__(kBlock) void k_rdm(const typename Cpx<R>::T *a, uint64_t ngroups,
                                                IdxSpec ix, int tq0, int tq1, double *partials)
{
    constexpr int D = 1 << NT;
    const int tq[2] = {tq0, tq1};
    uint64_t off[D];
#pragma unroll
    for (int x = 0; x < D; ++x) {
        uint64_t o = 0;
#pragma unroll
        for (int b = 0; b < NT; ++b)
            if ((x >> (NT - 1 - b)) & 1) o |= uint64_t(1) << tq[b];
        off[x] = o;
    }
    double re[D][D], im[D][D];
#pragma unroll
    for (int r = 0; r < D; ++r)
#pragma unroll
        for (int c = 0; c < D; ++c) re[r][c] = im[r][c] = 0.0;
    const uint64_t stride = uint64_t(gridDim.x) * kBlock;
    for (uint64_t t = uint64_t(blockIdx.x) * kBlock + threadIdx.x; t < ngroups; t += stride) {
        const uint64_t i0 = insert_zeros(t, ix);
        double vr[D], vi[D];
#pragma unroll
        for (int x = 0; x < D; ++x) {
            const auto v = a[i0 | off[x]];
            vr[x] = double(v.x);
            vi[x] = double(v.y);
        }
#pragma unroll
        for (int r = 0; r < D; ++r)
#pragma unroll
            for (int c = 0; c < D; ++c) {
                // v_r * conj(v_c)
                re[r][c] += vr[r] * vr[c] + vi[r] * vi[c];
                im[r][c] += vi[r] * vr[c] - vr[r] * vi[c];
            }
    }
    __shared__ double lds[kBlock / 64];
#pragma unroll
    for (int r = 0; r < D; ++r)
#pragma unroll
        for (int c = 0; c < D; ++c) {
            const double sr = block_sum(re[r][c], lds);
            const double si = block_sum(im[r][c], lds);
            if (threadIdx.x == 0) {
                partials[uint64_t(blockIdx.x) * 2 * D * D + 2 * (r * D + c)] = sr;
                partials[uint64_t(blockIdx.x) * 2 * D * D + 2 * (r * D + c) + 1] = si;
            }
        }
}

// Per-block sums of |alpha_i|^2 (bin 0) and of |alpha_i|^2 i_q for every
// qubit q < n (bins 1 + q); <Z_q> = total - 2 * bin(1 + q).
template <typename R>
__global__ __launch_bounds__(kBlock) void k_zsum(const typename Cpx<R>::T *a, int n,
                                                 double *partials)
{
    double acc[1 + kMaxQ];
#pragma unroll
    for (int b = 0; b <= kMaxQ; ++b) acc[b] = 0.0;
    const uint64_t n_amp = uint64_t(1) << n;
    const uint64_t stride = uint64_t(gridDim.x) * kBlock;
    for (uint64_t i = uint64_t(blockIdx.x) * kBlock + threadIdx.x; i < n_amp; i += stride) {
        const auto v = a[i];
        const double p = double(v.x) * double(v.x) + double(v.y) * double(v.y);
        acc[0] += p;
#pragma unroll
        for (int q = 0; q < kMaxQ; ++q) acc[1 + q] += ((i >> q) & 1) ? p : 0.0;
    }
    __shared__ double lds[kBlock / 64];
    for (int b = 0; b <= n; ++b) {
        double v = 0.0;
#pragma unroll
        for (int k = 0; k <= kMaxQ; ++k)
            if (k == b) v = acc[k];
        const double s = block_sum(v, lds);
        if (threadIdx.x == 0) partials[uint64_t(blockIdx.x) * (n + 1) + b] = s;
    }
}

__global__ void k_z_finish(const double *sums, int n, double *out)
{
    const int q = threadIdx.x;
    if (q < n) out[q] = sums[0] - 2.0 * sums[1 + q];
}

template <typename R>
__global__ __launch_bounds__(kBlock) void k_gather(const typename Cpx<R>::T *a, const uint64_t *idx,
                                                   uint64_t m, double2 *out)
{
    const uint64_t stride = uint64_t(gridDim.x) * kBlock;
    for (uint64_t k = uint64_t(blockIdx.x) * kBlock + threadIdx.x; k < m; k += stride) {
        const auto v = a[idx[k]];
        out[k] = make_double2(double(v.x), double(v.y));
    }
}

// Partial-amplitude recombination (Sec. 2.2 (partial), last step): one term
// of acc[k] = sum_w psiA_w(ia[k]) psiB_w(ib[k]), added in FP64.
template <typename R>
__global__ __launch_bounds__(kBlock) void k_partial_cmac(const typename Cpx<R>::T *a, const typename Cpx<R>::T *b,
                                                         const uint64_t *ia, const uint64_t *ib, uint64_t m,
                                                         double2 *acc)
{
    const uint64_t stride = uint64_t(gridDim.x) * kBlock;
    for (uint64_t k = uint64_t(blockIdx.x) * kBlock + threadIdx.x; k < m; k += stride) {
        const auto x = a[ia[k]];
        const auto y = b[ib[k]];
        const double xr = x.x, xi = x.y, yr = y.x, yi = y.y;
        double2 r = acc[k];
        r.x += xr * yr - xi * yi;
        r.y += xr * yi + xi * yr;
        acc[k] = r;
    }
}

template <typename R>
hipError_t dense1_impl(void *amp, int n, const IdxSpec &ix, int target, const double *m,
                       hipStream_t st)
{
    using C = typename Cpx<R>::T;
    MatArg<R, 2> mm;
    for (int k = 0; k < 8; ++k) mm.v[k] = R(m[k]);
    bool low_ctl = false;
    for (int k = 0; k < ix.npos; ++k)
        if (ix.pos[k] < 6 && ix.pos[k] != target) low_ctl = true;
    constexpr int U = 2;
    if (target < 6 && !low_ctl && n >= 8) {
        // enumerate every amplitude whose control bits are set (the target
        // bit is not removed: both halves of each pair are work items)
        IdxSpec cx{};
        int c = 0;
        for (int k = 0; k < ix.npos; ++k)
            if (ix.pos[k] != target) cx.pos[c++] = ix.pos[k];
        cx.npos = c;
        cx.set = ix.set;
        const uint64_t nitems = uint64_t(1) << (n - c);
        const uint64_t grid = grid_for(nitems, uint64_t(kBlock) * U);
        hipLaunchKernelGGL((k_dense1_lane<R, U>), dim3(unsigned(grid)), dim3(kBlock), 0, st,
                           (C *)amp, nitems, cx, target, mm);
        return hipGetLastError();
    }
    // a control below the 128-byte run with the target above it: whole runs
    const int need = sizeof(R) == 8 ? 3 : 4;  // 2^need amplitudes = 128 bytes
    if (target >= need) {
        uint64_t lmask = 0;
        IdxSpec hx{};
        for (int k = 0; k < ix.npos; ++k) {
            if (ix.pos[k] < need)
                lmask |= uint64_t(1) << ix.pos[k];
            else
                hx.pos[hx.npos++] = ix.pos[k];
        }
        if (lmask) {
            std::sort(hx.pos, hx.pos + hx.npos);
            uint64_t hmask = 0;
            for (int k = 0; k < hx.npos; ++k) hmask |= uint64_t(1) << hx.pos[k];
            hx.set = ix.set & hmask;
            const uint64_t np = uint64_t(1) << (n - hx.npos);
            hipLaunchKernelGGL((k_dense1_runs<R>), dim3(unsigned(grid_for(np, uint64_t(kBlock) * 2))),
                               dim3(kBlock), 0, st, (C *)amp, np, hx, uint64_t(1) << target, lmask, ix.set & lmask,
                               mm);
            return hipGetLastError();
        }
    }
    // one pair per thread (with the XCD-aware chunk order, 6.12 TB/s
    // against 6.05 for two and 5.58 for four on 30-qubit complex128 sweeps)
    constexpr int UP = 1;
    const uint64_t npairs = uint64_t(1) << (n - ix.npos);
    const uint64_t grid = grid_for(npairs, uint64_t(kBlock) * UP);
    if (stream_ok<R>(ix))
        hipLaunchKernelGGL((k_dense1<R, UP, true>), dim3(unsigned(grid)), dim3(kBlock), 0, st,
                           (C *)amp, npairs, ix, uint64_t(1) << target, mm);
    else
        hipLaunchKernelGGL((k_dense1<R, UP, false>), dim3(unsigned(grid)), dim3(kBlock), 0, st,
                           (C *)amp, npairs, ix, uint64_t(1) << target, mm);
    return hipGetLastError();
}

template <typename R, int NT>
hipError_t dense_small_impl(void *amp, int n, const IdxSpec &ix, const int *tq, const double *m,
                            hipStream_t st)
{
    using C = typename Cpx<R>::T;
    constexpr int D = 1 << NT;
    MatArg<R, D> mm;
    for (int k = 0; k < 2 * D * D; ++k) mm.v[k] = R(m[k]);
    const uint64_t ng = uint64_t(1) << (n - ix.npos);
    constexpr int U = (NT == 2) ? 2 : 1;
    const uint64_t grid = grid_for(ng, uint64_t(kBlock) * U);
    if (stream_ok<R>(ix))
        hipLaunchKernelGGL((k_dense_small<R, NT, U, true>), dim3(unsigned(grid)), dim3(kBlock), 0,
                           st, (C *)amp, ng, ix, mm, tq[0], NT > 1 ? tq[1] : 0, NT > 2 ? tq[2] : 0);
    else
        hipLaunchKernelGGL((k_dense_small<R, NT, U, false>), dim3(unsigned(grid)), dim3(kBlock), 0,
                           st, (C *)amp, ng, ix, mm, tq[0], NT > 1 ? tq[1] : 0, NT > 2 ? tq[2] : 0);
    return hipGetLastError();
}

template <typename R>
hipError_t denseN_impl(void *amp, int n, const IdxSpec &ix, const int *tq, int nt,
                       const void *dev_m, hipStream_t st)
{
    using C = typename Cpx<R>::T;
    const uint64_t ng = uint64_t(1) << (n - ix.npos);
    int t[6] = {0, 0, 0, 0, 0, 0};
    for (int b = 0; b < nt; ++b) t[b] = tq[b];
    const uint64_t G = kBlock >> nt;
    const uint64_t grid = grid_for(ng, G * 8);
    const C *m = (const C *)dev_m;
    switch (nt) {
    case 4:
        hipLaunchKernelGGL((k_denseN<R, 4>), dim3(unsigned(grid)), dim3(kBlock), 0, st, (C *)amp,
                           ng, ix, m, t[0], t[1], t[2], t[3], t[4], t[5]);
        break;
    case 5:
        hipLaunchKernelGGL((k_denseN<R, 5>), dim3(unsigned(grid)), dim3(kBlock), 0, st, (C *)amp,
                           ng, ix, m, t[0], t[1], t[2], t[3], t[4], t[5]);
        break;
    case 6:
        hipLaunchKernelGGL((k_denseN<R, 6>), dim3(unsigned(grid)), dim3(kBlock), 0, st, (C *)amp,
                           ng, ix, m, t[0], t[1], t[2], t[3], t[4], t[5]);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename R>
hipError_t phase_impl(void *amp, int n, const IdxSpec &ix, const int *tq, int nt, const double *d,
                      hipStream_t st)
{
    using C = typename Cpx<R>::T;
    DiagArg<R> da;
    da.nt = nt;
    da.active = 0;
    for (int b = 0; b < 6; ++b) da.tq[b] = b < nt ? tq[b] : 0;
    for (int x = 0; x < 64; ++x) {
        const double re = x < (1 << nt) ? d[2 * x] : 1.0;
        const double im = x < (1 << nt) ? d[2 * x + 1] : 0.0;
        da.v[2 * x] = R(re);
        da.v[2 * x + 1] = R(im);
        if (x < (1 << nt) && !(re == 1.0 && im == 0.0)) da.active |= uint64_t(1) << x;
    }
    const uint64_t ng = uint64_t(1) << (n - ix.npos);
    if (__builtin_popcountll(da.active) == 1) {
        const int x = __builtin_ctzll(da.active);
        uint64_t o = 0;
        for (int b = 0; b < nt; ++b)
            if ((x >> (nt - 1 - b)) & 1) o |= uint64_t(1) << tq[b];
        constexpr int U1 = 8;
        const uint64_t g1 = grid_for(ng, uint64_t(kBlock) * U1);
        const int need = sizeof(R) == 8 ? 3 : 4;  // 2^need amplitudes = 128 bytes
        uint64_t lmask = 0;
        IdxSpec hx{};
        for (int k = 0; k < ix.npos; ++k) {
            if (ix.pos[k] < need)
                lmask |= uint64_t(1) << ix.pos[k];
            else
                hx.pos[hx.npos++] = ix.pos[k];
        }
        if (lmask) {
            std::sort(hx.pos, hx.pos + hx.npos);
            const uint64_t want = ix.set | o;  // every condition bit's value
            uint64_t hmask = 0;
            for (int k = 0; k < hx.npos; ++k) hmask |= uint64_t(1) << hx.pos[k];
            hx.set = want & hmask;
            const uint64_t nitems = uint64_t(1) << (n - hx.npos);
            constexpr int UR = 4;
            hipLaunchKernelGGL((k_phase1_runs<R, UR>), dim3(unsigned(grid_for(nitems, uint64_t(kBlock) * UR))),
                               dim3(kBlock), 0, st, (C *)amp, nitems, hx, lmask, want & lmask, da.v[2 * x],
                               da.v[2 * x + 1]);
            return hipGetLastError();
        }
        if (stream_ok<R>(ix))
            hipLaunchKernelGGL((k_phase1<R, U1, true>), dim3(unsigned(g1)), dim3(kBlock), 0, st, (C *)amp, ng, ix,
                               o, da.v[2 * x], da.v[2 * x + 1]);
        else
            hipLaunchKernelGGL((k_phase1<R, U1, false>), dim3(unsigned(g1)), dim3(kBlock), 0, st, (C *)amp, ng, ix,
                               o, da.v[2 * x], da.v[2 * x + 1]);
        return hipGetLastError();
    }
    constexpr int U = 4;
    const uint64_t grid = grid_for(ng, uint64_t(kBlock) * U);
    if (stream_ok<R>(ix))
        hipLaunchKernelGGL((k_phase<R, U, true>), dim3(unsigned(grid)), dim3(kBlock), 0, st, (C *)amp,
                           ng, ix, da);
    else
        hipLaunchKernelGGL((k_phase<R, U, false>), dim3(unsigned(grid)), dim3(kBlock), 0, st,
                           (C *)amp, ng, ix, da);
    return hipGetLastError();
}

IdxSpec spec_from(const int *q, int nq)
{
    IdxSpec s{};
    s.npos = nq;
    for (int b = 0; b < nq; ++b) s.pos[b] = q[b];
    s.set = 0;
    return s;
}

IdxSpec sorted_spec(const int *q, int nq)
{
    IdxSpec s = spec_from(q, nq);
    for (int i = 1; i < nq; ++i)
        for (int j = i; j > 0 && s.pos[j - 1] > s.pos[j]; --j) {
            int t = s.pos[j];
            s.pos[j] = s.pos[j - 1];
            s.pos[j - 1] = t;
        }
    return s;
}

template <typename R>
hipError_t probs_impl(const void *amp, int n, const int *q, int nq, double *scratch,
                      double *dev_out, hipStream_t st)
{
    using C = typename Cpx<R>::T;
    const C *a = (const C *)amp;
    const uint64_t n_amp = uint64_t(1) << n;
    IdxSpec qs = spec_from(q, nq);
    if (nq == n) {
        const uint64_t grid = grid_for(n_amp, kBlock);
        hipLaunchKernelGGL((k_probs_perm<R>), dim3(unsigned(grid)), dim3(kBlock), 0, st, a, n_amp,
                           nq, qs, dev_out);
        return hipGetLastError();
    }
    if (nq > 10) {
        int rest[kMaxQ];
        int nr = 0;
        for (int k = 0; k < n; ++k) {
            bool listed = false;
            for (int b = 0; b < nq; ++b) listed |= q[b] == k;
            if (!listed) rest[nr++] = k;
        }
        IdxSpec rs = spec_from(rest, nr);
        const uint64_t grid = grid_for(uint64_t(1) << nq, kBlock);
        hipLaunchKernelGGL((k_probs_bins<R>), dim3(unsigned(grid)), dim3(kBlock), 0, st, a, nq, qs,
                           rs, uint64_t(1) << nr, dev_out);
        return hipGetLastError();
    }
    const int nb = 1 << nq;
    const uint64_t grid = grid_for(n_amp, kBlock) < kRedBlocks ? grid_for(n_amp, kBlock)
                                                               : kRedBlocks;
    switch (nb) {
    case 2:
        hipLaunchKernelGGL((k_probs_reg<R, 2>), dim3(unsigned(grid)), dim3(kBlock), 0, st, a, n_amp,
                           nq, qs, scratch);
        break;
    case 4:
        hipLaunchKernelGGL((k_probs_reg<R, 4>), dim3(unsigned(grid)), dim3(kBlock), 0, st, a, n_amp,
                           nq, qs, scratch);
        break;
    case 8:
        hipLaunchKernelGGL((k_probs_reg<R, 8>), dim3(unsigned(grid)), dim3(kBlock), 0, st, a, n_amp,
                           nq, qs, scratch);
        break;
    default:
        hipLaunchKernelGGL((k_probs_lds<R>), dim3(unsigned(grid)), dim3(kBlock), 0, st, a, n_amp,
                           nq, qs, scratch);
        break;
    }
    hipLaunchKernelGGL(k_sum_columns, dim3(unsigned((nb + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                       st, scratch, int(grid), nb, dev_out);
    return hipGetLastError();
}

template <typename R>
hipError_t rdm_impl(const void *amp, int n, const int *tq, int nt, double *scratch,
                    double *dev_out, hipStream_t st)
{
    using C = typename Cpx<R>::T;
    IdxSpec ix = sorted_spec(tq, nt);
    const uint64_t ng = uint64_t(1) << (n - nt);
    const uint64_t g0 = grid_for(ng, kBlock);
    const uint64_t grid = g0 < kRedBlocks ? g0 : kRedBlocks;
    const int nval = 2 << (2 * nt);
    if (nt == 1)
        hipLaunchKernelGGL((k_rdm<R, 1>), dim3(unsigned(grid)), dim3(kBlock), 0, st, (const C *)amp,
                           ng, ix, tq[0], 0, scratch);
    else
        hipLaunchKernelGGL((k_rdm<R, 2>), dim3(unsigned(grid)), dim3(kBlock), 0, st, (const C *)amp,
                           ng, ix, tq[0], tq[1], scratch);
    hipLaunchKernelGGL(k_sum_columns, dim3(1), dim3(kBlock), 0, st, scratch, int(grid), nval,
                       dev_out);
    return hipGetLastError();
}

}  // namespace

// ------------------------------------------------------------ launchers --

hipError_t launch_init(qs_dtype dt, void *amp, uint64_t n_amp, hipStream_t st)
{
    const uint64_t grid = grid_for(n_amp, kBlock);
    if (dt == QS_C128)
        hipLaunchKernelGGL((k_init<double>), dim3(unsigned(grid)), dim3(kBlock), 0, st,
                           (double2 *)amp, n_amp);
    else
        hipLaunchKernelGGL((k_init<float>), dim3(unsigned(grid)), dim3(kBlock), 0, st,
                           (float2 *)amp, n_amp);
    return hipGetLastError();
}

hipError_t launch_scale(qs_dtype dt, void *amp, uint64_t n_amp, double scale, hipStream_t st)
{
    const uint64_t grid = grid_for(n_amp, kBlock);
    if (dt == QS_C128)
        hipLaunchKernelGGL((k_scale<double>), dim3(unsigned(grid)), dim3(kBlock), 0, st,
                           (double2 *)amp, n_amp, scale);
    else
        hipLaunchKernelGGL((k_scale<float>), dim3(unsigned(grid)), dim3(kBlock), 0, st,
                           (float2 *)amp, n_amp, float(scale));
    return hipGetLastError();
}

hipError_t launch_dense1(qs_dtype dt, void *amp, int n, const IdxSpec &ix, int target,
                         const double *m, hipStream_t st)
{
    return dt == QS_C128 ? dense1_impl<double>(amp, n, ix, target, m, st)
                         : dense1_impl<float>(amp, n, ix, target, m, st);
}

hipError_t launch_dense2(qs_dtype dt, void *amp, int n, const IdxSpec &ix, const int *tq,
                         const double *m, hipStream_t st)
{
    return dt == QS_C128 ? dense_small_impl<double, 2>(amp, n, ix, tq, m, st)
                         : dense_small_impl<float, 2>(amp, n, ix, tq, m, st);
}

hipError_t launch_dense3(qs_dtype dt, void *amp, int n, const IdxSpec &ix, const int *tq,
                         const double *m, hipStream_t st)
{
    return dt == QS_C128 ? dense_small_impl<double, 3>(amp, n, ix, tq, m, st)
                         : dense_small_impl<float, 3>(amp, n, ix, tq, m, st);
}

hipError_t launch_denseN(qs_dtype dt, void *amp, int n, const IdxSpec &ix, const int *tq, int nt,
                         const void *dev_m, hipStream_t st)
{
    return dt == QS_C128 ? denseN_impl<double>(amp, n, ix, tq, nt, dev_m, st)
                         : denseN_impl<float>(amp, n, ix, tq, nt, dev_m, st);
}

hipError_t launch_phase(qs_dtype dt, void *amp, int n, const IdxSpec &ix, const int *tq, int nt,
                        const double *d, hipStream_t st)
{
    return dt == QS_C128 ? phase_impl<double>(amp, n, ix, tq, nt, d, st)
                         : phase_impl<float>(amp, n, ix, tq, nt, d, st);
}

size_t reduce_scratch_doubles(int n, int nbins)
{
    (void)n;
    size_t per = size_t(nbins) > size_t(1 + kMaxQ) ? size_t(nbins) : size_t(1 + kMaxQ);
    if (per < 32) per = 32;
    return kRedBlocks * per + 64;
}

hipError_t launch_norm2(qs_dtype dt, const void *amp, int n, double *scratch, double *dev_out,
                        hipStream_t st)
{
    // probabilities of zero listed qubits = the squared norm: one bin
    const uint64_t n_amp = uint64_t(1) << n;
    const uint64_t g0 = grid_for(n_amp, kBlock);
    const uint64_t grid = g0 < kRedBlocks ? g0 : kRedBlocks;
    IdxSpec none{};
    if (dt == QS_C128)
        hipLaunchKernelGGL((k_probs_reg<double, 1>), dim3(unsigned(grid)), dim3(kBlock), 0, st,
                           (const double2 *)amp, n_amp, 0, none, scratch);
    else
        hipLaunchKernelGGL((k_probs_reg<float, 1>), dim3(unsigned(grid)), dim3(kBlock), 0, st,
                           (const float2 *)amp, n_amp, 0, none, scratch);
    hipLaunchKernelGGL(k_sum_columns, dim3(1), dim3(kBlock), 0, st, scratch, int(grid), 1, dev_out);
    return hipGetLastError();
}

hipError_t launch_probs(qs_dtype dt, const void *amp, int n, const int *q, int nq, double *scratch,
                        double *dev_out, hipStream_t st)
{
    return dt == QS_C128 ? probs_impl<double>(amp, n, q, nq, scratch, dev_out, st)
                         : probs_impl<float>(amp, n, q, nq, scratch, dev_out, st);
}

hipError_t launch_rdm(qs_dtype dt, const void *amp, int n, const int *tq, int nt, double *scratch,
                      double *dev_out, hipStream_t st)
{
    if (nt < 1 || nt > 2) return hipErrorInvalidValue;
    return dt == QS_C128 ? rdm_impl<double>(amp, n, tq, nt, scratch, dev_out, st)
                         : rdm_impl<float>(amp, n, tq, nt, scratch, dev_out, st);
}

hipError_t launch_expect_z(qs_dtype dt, const void *amp, int n, double *scratch, double *dev_out,
                           hipStream_t st)
{
    const uint64_t n_amp = uint64_t(1) << n;
    const uint64_t g0 = grid_for(n_amp, kBlock);
    const uint64_t grid = g0 < kRedBlocks ? g0 : kRedBlocks;
    double *sums = scratch + kRedBlocks * (1 + kMaxQ);
    if (dt == QS_C128)
        hipLaunchKernelGGL((k_zsum<double>), dim3(unsigned(grid)), dim3(kBlock), 0, st,
                           (const double2 *)amp, n, scratch);
    else
        hipLaunchKernelGGL((k_zsum<float>), dim3(unsigned(grid)), dim3(kBlock), 0, st,
                           (const float2 *)amp, n, scratch);
    hipLaunchKernelGGL(k_sum_columns, dim3(1), dim3(kBlock), 0, st, scratch, int(grid), n + 1,
                       sums);
    hipLaunchKernelGGL(k_z_finish, dim3(1), dim3(64), 0, st, sums, n, dev_out);
    return hipGetLastError();
}

hipError_t launch_partial_cmac(qs_dtype dt, const void *a, const void *b, const uint64_t *ia,
                               const uint64_t *ib, uint64_t m, double *acc, hipStream_t st)
{
    const uint64_t grid = grid_for(m, kBlock);
    if (dt == QS_C128)
        hipLaunchKernelGGL((k_partial_cmac<double>), dim3(unsigned(grid)), dim3(kBlock), 0, st,
                           (const double2 *)a, (const double2 *)b, ia, ib, m, (double2 *)acc);
    else
        hipLaunchKernelGGL((k_partial_cmac<float>), dim3(unsigned(grid)), dim3(kBlock), 0, st,
                           (const float2 *)a, (const float2 *)b, ia, ib, m, (double2 *)acc);
    return hipGetLastError();
}

hipError_t launch_gather(qs_dtype dt, const void *amp, const uint64_t *dev_idx, uint64_t m,
                         double *dev_out, hipStream_t st)
{
    const uint64_t grid = grid_for(m, kBlock);
    if (dt == QS_C128)
        hipLaunchKernelGGL((k_gather<double>), dim3(unsigned(grid)), dim3(kBlock), 0, st,
                           (const double2 *)amp, dev_idx, m, (double2 *)dev_out);
    else
        hipLaunchKernelGGL((k_gather<float>), dim3(unsigned(grid)), dim3(kBlock), 0, st,
                           (const float2 *)amp, dev_idx, m, (double2 *)dev_out);
    return hipGetLastError();
}

}  // namespace qs
