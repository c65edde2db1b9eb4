// Internal declarations shared by the host side of libqs and its kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "../../include/qs.h"

namespace qs {

constexpr int kMaxQ = QS_MAX_QUBITS;

// Enumeration of the amplitudes a gate touches: work item t in
// [0, 2^(n - npos)) maps to index insert_zeros(t, pos) | set, i.e. a zero bit
// is inserted at every position of `pos` (ascending) and the control bits in
// `set` are then forced to one.  This is the "i_k = 0" enumeration of Eq. 2
// extended to several targets and to the "i_q = 1" condition of Eq. 3.
struct IdxSpec {
    int npos;
    int pos[kMaxQ];
    uint64_t set;
};

template <typename R>
struct Cpx;
template <>
struct Cpx<double> {
    using T = double2;
};
template <>
struct Cpx<float> {
    using T = float2;
};

// Dense small matrices passed by value: (re, im) pairs, row-major.
template <typename R, int D>
struct MatArg {
    R v[2 * D * D];
};

// Diagonal factors for the phase kernel (up to 6 targets).
template <typename R>
struct DiagArg {
    R v[2 * 64];
    uint64_t active;  // bit x set when factor x differs from 1
    int nt;
    int tq[6];        // target qubits, tq[0] = most significant bit of x
};

// Launchers (qs_kernels.hip).  All are asynchronous on `st`.  `amp` points to
// double2 (C128) or float2 (C64) data; dt selects the instantiation.
hipError_t launch_init(qs_dtype dt, void *amp, uint64_t n_amp, hipStream_t st);
hipError_t launch_dense1(qs_dtype dt, void *amp, int n, const IdxSpec &ix, int target,
                         const double *m, hipStream_t st);
hipError_t launch_dense2(qs_dtype dt, void *amp, int n, const IdxSpec &ix, const int *tq,
                         const double *m, hipStream_t st);
hipError_t launch_dense3(qs_dtype dt, void *amp, int n, const IdxSpec &ix, const int *tq,
                         const double *m, hipStream_t st);
// nt in 4..6; `dev_m` = device copy of the matrix in the state's dtype
// (double2 / float2, row-major).
hipError_t launch_denseN(qs_dtype dt, void *amp, int n, const IdxSpec &ix, const int *tq, int nt,
                         const void *dev_m, hipStream_t st);
// diagonal factors d (nt <= 6 targets, (re,im) pairs) times controls in ix.set
hipError_t launch_phase(qs_dtype dt, void *amp, int n, const IdxSpec &ix, const int *tq, int nt,
                        const double *d, hipStream_t st);

// FP64 reductions.  `scratch` must hold reduce_scratch_doubles(...) doubles;
// results land in device memory `dev_out` (double).
size_t reduce_scratch_doubles(int n, int nbins);
hipError_t launch_norm2(qs_dtype dt, const void *amp, int n, double *scratch, double *dev_out,
                        hipStream_t st);
// PMEASURE over nq qubits (q[0] = most significant output bit); dev_out holds
// 2^nq doubles.
hipError_t launch_probs(qs_dtype dt, const void *amp, int n, const int *q, int nq, double *scratch,
                        double *dev_out, hipStream_t st);
// reduced density matrix of nt <= 2 targets: dev_out = 2 * 4^nt doubles,
// rho[x][y] = sum alpha_(x) conj(alpha_(y)), row-major (re, im).
hipError_t launch_rdm(qs_dtype dt, const void *amp, int n, const int *tq, int nt, double *scratch,
                      double *dev_out, hipStream_t st);
// <Z_q> for q < n into dev_out[n]
hipError_t launch_expect_z(qs_dtype dt, const void *amp, int n, double *scratch, double *dev_out,
                           hipStream_t st);
// out[k] = alpha_{idx[k]} as double2
hipError_t launch_gather(qs_dtype dt, const void *amp, const uint64_t *dev_idx, uint64_t m,
                         double *dev_out, hipStream_t st);
// Qubit-remap exchange of a shard of L local qubits (qs_remap.hip): pack
// (buf[b] = shard[remap(b)]) or unpack (shard[remap(b)] = buf[b]), where
// remap spreads chunk number b >> (L - g) over the local qubits lq[0..g-1]
// and the rest of b over the other local bits in ascending order.
hipError_t launch_remap(qs_dtype dt, void *shard, void *buf, int L, int g, const int *lq, bool pack,
                        hipStream_t st);
// acc[k] += a[ia[k]] * b[ib[k]] for k < m (complex, FP64 accumulators,
// acc = m (re, im) doubles): one branch of the partial-amplitude recombination
hipError_t launch_partial_cmac(qs_dtype dt, const void *a, const void *b, const uint64_t *ia,
                               const uint64_t *ib, uint64_t m, double *acc, hipStream_t st);
// Reduction scratch in a static device array (qs_noalloc.hip): the address
// of the current device's copy (looked up once per device) and its size.
hipError_t noalloc_scratch(double **out);
size_t noalloc_scratch_doubles();
// amp *= scale (real), used for renormalisation
hipError_t launch_scale(qs_dtype dt, void *amp, uint64_t n_amp, double scale, hipStream_t st);

}  // namespace qs
