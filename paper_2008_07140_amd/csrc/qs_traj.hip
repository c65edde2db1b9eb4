// FP64 reductions for batches of trajectory states.
//
// Noise sampling (Sec. 2.4) needs, for a run of one-qubit channels whose first
// Kraus operator is K1 = diag(1, k) (amplitude and phase damping), the branch
// weight of every site given that the earlier sites of the run took K1.  With
// a_j = |k_j|^2 and w_x = |alpha_x|^2 these are all prefix sums of one pass:
//   S_j = sum_x w_x x_{q_j} prod_{i<j} a_i^{x_{q_i}},   Z = sum_x w_x,
// and the unnormalised norm after K1 on sites 0..j-1 is Z_j = Z - sum_{i<j}
// (1 - a_i) S_i.  With every a_j = 1 the same pass gives <Z_q> = (Z - 2 S_q) / Z.
#include <hip/hip_runtime.h>

#include "qs_internal.h"
#include "qs_traj.h"

namespace qs {

namespace {

constexpr int kT = 256;

__device__ __forceinline__ double wave_sum_d(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

template <typename C>
__global__ __launch_bounds__(kT) void k_run_sums(const RunSumTask *tasks, const RunSumArgs *args,
                                                 double *partials)
{
    const RunSumTask task = tasks[blockIdx.x];
    const RunSumArgs &d = args[task.arg];
    const C *a = reinterpret_cast<const C *>(d.amp);
    const uint64_t start = uint64_t(task.chunk) * d.chunk_len;
    uint64_t end = start + d.chunk_len;
    if (end > d.n_amp) end = d.n_amp;
    double z = 0.0, S[kRunMax];
#pragma unroll
    for (int j = 0; j < kRunMax; ++j) S[j] = 0.0;
    for (uint64_t i = start + threadIdx.x; i < end; i += kT) {
        const auto v = a[i];
        double w = double(v.x) * double(v.x) + double(v.y) * double(v.y);
        z += w;
#pragma unroll
        for (int j = 0; j < kRunMax; ++j)
            if (j < d.J) {
                const bool bit = (i >> d.q[j]) & 1;
                S[j] += bit ? w : 0.0;
                w *= bit ? d.a[j] : 1.0;
            }
    }
    __shared__ double lds[kT / 64];
    double *out = partials + uint64_t(blockIdx.x) * (kRunMax + 1);
    auto reduce = [&](double v, int slot) {
        v = wave_sum_d(v);
        __syncthreads();
        if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
        __syncthreads();
        if (threadIdx.x == 0) {
            double s = 0.0;
            for (int k = 0; k < kT / 64; ++k) s += lds[k];
            out[slot] = s;
        }
    };
    reduce(z, 0);
#pragma unroll
    for (int j = 0; j < kRunMax; ++j)
        if (j < d.J) reduce(S[j], 1 + j);
}

// out[t * (kRunMax + 1) + v] = sum of partials over the workgroups of state t
__global__ __launch_bounds__(kT) void k_run_sums_finish(const double *partials, const uint32_t *first,
                                                        const uint32_t *count, int nstates,
                                                        double *out)
{
    const int w = kRunMax + 1;
    for (int idx = blockIdx.x * kT + threadIdx.x; idx < nstates * w; idx += gridDim.x * kT) {
        const int t = idx / w, v = idx % w;
        double s = 0.0;
        for (uint32_t b = 0; b < count[t]; ++b) s += partials[uint64_t(first[t] + b) * w + v];
        out[idx] = s;
    }
}

}  // namespace

hipError_t launch_run_sums(qs_dtype dt, uint32_t ntasks, const RunSumTask *tasks, const RunSumArgs *args,
                           double *partials, hipStream_t st)
{
    if (ntasks == 0) return hipSuccess;
    if (dt == QS_C128)
        hipLaunchKernelGGL(k_run_sums<double2>, dim3(ntasks), dim3(kT), 0, st, tasks, args, partials);
    else
        hipLaunchKernelGGL(k_run_sums<float2>, dim3(ntasks), dim3(kT), 0, st, tasks, args, partials);
    return hipGetLastError();
}

hipError_t launch_run_sums_finish(const double *partials, const uint32_t *first, const uint32_t *count,
                                  int nstates, double *out, hipStream_t st)
{
    const int total = nstates * (kRunMax + 1);
    const int grid = (total + kT - 1) / kT;
    hipLaunchKernelGGL(k_run_sums_finish, dim3(grid > 0 ? grid : 1), dim3(kT), 0, st, partials, first, count,
                       nstates, out);
    return hipGetLastError();
}

}  // namespace qs
