// Single-amplitude mode (Sec. 2.3): device side of the tensor contractions.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace qs {

constexpr int kSaMaxBits = 40;  // indices of one tensor (a 2^40-entry tensor is far beyond memory)

// One pairwise merge of two tensors X and Y of the graphical model into Z,
// summing the vertices they share that no other tensor holds:
//   Z[t, b, m, n] = sum_k X[t, b, m, k] * Y[t, b, n, k]
// with t the batch element (a bitstring and a slice), b the shared vertices
// kept, m / n the vertices of X / Y alone and k the summed ones.  X is
// stored with k in the low bits, then m, then b (k + (m << nk) +
// (b << (nk + nm))), or, with xo set, m lowest (m + (k << nm) +
// (b << (nk + nm))); Y likewise with n and yo.  Z's storage is what its own
// consumer asks for, so logical bit j of b / m / n goes to storage bit
// pb[j] / pm[j] / pn[j].  An operand without a batch dimension has batch
// stride 0.
struct SaContract {
    const double2 *x;
    const double2 *y;
    double2 *z;
    uint64_t sx, sy, sz;  // batch strides in amplitudes
    uint32_t nbt;         // batch elements of Z
    int nb, nm, nn, nk;   // bit counts
    int bfast;            // tiled merges: neighbouring tiles take neighbouring b (Z's low bits are b)
    int xo, yo;           // X / Y stored with their own vertices lowest
    uint8_t pb[kSaMaxBits], pm[kSaMaxBits], pn[kSaMaxBits];
};

// Placement of an initial tensor (one gate) into the storage its consumer
// asks for, with the fixed vertices (initial state, measured bitstring,
// slices) substituted: out[t, f] = base[sum_p bit_p(f) << src[p] +
// sum_j value_j(t) << fpos[j]], value_j(t) = 0 (kind 0), bit `which` of the
// bitstring of element t (kind 1) or bit `which` of its slice (kind 2).
struct SaPrep {
    const double2 *base;
    double2 *out;
    uint64_t so;        // batch stride of out (0 = no batch dimension)
    uint32_t nbt;       // batch elements of out
    uint32_t slices;    // slices per bitstring (element t = bitstring t / slices, slice t % slices)
    int r;              // free indices of out
    int nf;             // fixed indices
    uint8_t src[kSaMaxBits];
    uint8_t fpos[kSaMaxBits], fkind[kSaMaxBits], fwhich[kSaMaxBits];
};

enum SaKernel { SA_THREAD = 0, SA_WAVE = 1, SA_TILE = 2 };

hipError_t launch_sa_prep(const SaPrep &p, const uint64_t *bits, hipStream_t st);
hipError_t launch_sa_contract(const SaContract &c, int kernel, hipStream_t st);
// out[w] = sum_{s < slices} prod_{c < nscal} scal[c][(w * slices + s) * strides[c]]
// (stride 0: a component without a batch dimension), or 0 when bitstring w
// sets a qubit in `idle` (a qubit whose initial vertex is also its measured
// one: no gate changes its value, so it must read 0).
hipError_t launch_sa_finish(const double2 *const *scal, const uint64_t *strides, int nscal, uint32_t words,
                            uint32_t slices, const uint64_t *bits, uint64_t idle, double2 *out, hipStream_t st);

}  // namespace qs
