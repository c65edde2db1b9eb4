// Batched trajectory reductions (see qs_traj.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "qs_internal.h"

namespace qs {

constexpr int kRunMax = 36;  // qubits per run of damping-type sites (and <Z_q> of up to 36 qubits)

struct RunSumArgs {
    const void *amp;     // state of 2^n amplitudes (double2 / float2)
    uint64_t n_amp;
    uint64_t chunk_len;  // amplitudes per workgroup
    int J;               // number of sites in the run
    int pad;
    double am1[kRunMax]; // |K1_11|^2 - 1 of site j (0 for plain <Z> sums)
    uint8_t q[kRunMax];  // qubit of site j
};

struct RunSumTask {
    uint32_t arg;    // index into the RunSumArgs array
    uint32_t chunk;  // chunk of that state
};

// nmax: the widest state of the launch (states of at most 32 qubits take a
// kernel with 32-bit index arithmetic).
hipError_t launch_run_sums(qs_dtype dt, int nmax, uint32_t ntasks, const RunSumTask *tasks, const RunSumArgs *args,
                           double *partials, hipStream_t st);
hipError_t launch_run_sums_finish(const double *partials, const uint32_t *first, const uint32_t *count,
                                  int nstates, double *out, hipStream_t st);

}  // namespace qs
