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
    uint64_t chunk_len;  // amplitudes per workgroup (a multiple of 8192: k_run_sums reads index bits from it)
    int J;               // number of sites in the run
    uint32_t slot;       // trajectory slot whose activity flag gates the work (device-sampled passes)
    double am1[kRunMax]; // |K1_11|^2 - 1 of site j (0 for plain <Z> sums)
    uint8_t q[kRunMax];  // qubit of site j
};

// Device-side branch choice for one run of damping-type sites of one
// trajectory (Sec. 2.4, steps 2-3): the run's sums in `row` of the sums
// buffer, the Philox trajectory index and every site's counter.
struct SampleArgs {
    uint32_t slot;             // trajectory slot (activity flag, freeze record)
    uint32_t row;              // row of the run sums: Z, S_0, S_1, ...
    uint64_t traj;             // Philox trajectory index
    uint32_t step;             // the run's step index in the trajectory (reported when it jumps)
    uint32_t arg;              // RunSumArgs of the run (J and 1 - a_j = -am1[j])
    uint32_t site[kRunMax];    // Philox site counter of site j
};

// Where a device-sampled trajectory left the no-jump path: site j of its
// run step `step` took the jump operator K2, whose branch weight (the
// squared norm of the state after it, before normalisation) is nrm2.
struct Freeze {
    int32_t step;   // -1 = no jump (the trajectory completed the pass)
    int32_t j;
    double nrm2;
};

struct RunSumTask {
    uint32_t arg;    // index into the RunSumArgs array
    uint32_t chunk;  // chunk of that state
};

// nmax: the widest state of the launch (states of at most 32 qubits take a
// kernel with 32-bit index arithmetic).
// active: NULL, or one flag per trajectory slot; the tasks of a slot whose
// flag is 0 write zero partials and do no other work.
hipError_t launch_run_sums(qs_dtype dt, int nmax, uint32_t ntasks, const RunSumTask *tasks, const RunSumArgs *args,
                           double *partials, const int *active, hipStream_t st);
hipError_t launch_run_sums_finish(const double *partials, const uint32_t *first, const uint32_t *count,
                                  int nstates, double *out, hipStream_t st);

// One thread per entry of `sa`: walks the run's sites in order, draws each
// site's uniform and picks K1 or K2 from the prefix sums (FP64).  The first
// K2 clears the slot's activity flag and records a Freeze; a run whose
// weights are all zero sets *err.  Entries of inactive slots are skipped.
hipError_t launch_sample_runs(const SampleArgs *sa, uint32_t count, const RunSumArgs *args, const double *sums,
                              uint64_t seed, int *active, Freeze *freeze, int *err, hipStream_t st);

}  // namespace qs
