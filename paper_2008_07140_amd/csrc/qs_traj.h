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
    double a[kRunMax];   // |K1_11|^2 of site j (1 for plain <Z> sums)
    uint8_t q[kRunMax];  // qubit of site j
};

struct RunSumTask {
    uint32_t arg;    // index into the RunSumArgs array
    uint32_t chunk;  // chunk of that state
};

hipError_t launch_run_sums(qs_dtype dt, uint32_t ntasks, const RunSumTask *tasks, const RunSumArgs *args,
                           double *partials, hipStream_t st);
hipError_t launch_run_sums_finish(const double *partials, const uint32_t *first, const uint32_t *count,
                                  int nstates, double *out, hipStream_t st);

}  // namespace qs
