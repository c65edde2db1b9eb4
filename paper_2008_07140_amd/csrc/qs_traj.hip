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
#include "qs_philox.h"
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

// A workgroup sums one chunk of the state, in groups of NB kT amplitudes
// i = b0 + k kT + tid (k < NB, tid < kT): chunks and so b0 are multiples of
// NB kT, so index bits 0..7 are bits of tid, bits 8..10 bits of k and the
// higher bits bits of b0, the same for the whole workgroup.  The factor
// prod_{i<j} a_i^{x_{q_i}} of site j splits the same way into a per-thread
// part fT (sites on bits 0..7), a part uK_j(k) (bits 8..10; a table in LDS
// that also holds x_{q_j} when q_j is such a bit) and a per-group part fG
// (higher bits), so that
//   S_j = sum over groups and threads of fG fT x_{q_j} sum_k uK_j(k) w_k,
// where x_{q_j} stands only when q_j is a thread or group bit: per site one
// FP64 FMA per amplitude and a few operations per group, instead of a bit
// test, a conversion and three operations per amplitude.  WIDE: states of
// more than 32 qubits (64-bit group bits).
template <typename C, bool WIDE>
__global__ __launch_bounds__(kT) void k_run_sums(const RunSumTask *__restrict__ tasks,
                                                 const RunSumArgs *__restrict__ args, double *partials,
                                                 const int *__restrict__ active)
{
    constexpr int NB = 8;
    constexpr uint32_t kTBits = 8, kKBits = 3;  // index bits of tid and of k
    static_assert(kT == 1 << kTBits && NB == 1 << kKBits, "index bits");
    __shared__ double uk[kRunMax][NB];
    const RunSumTask task = tasks[blockIdx.x];
    const RunSumArgs &d = args[task.arg];
    if (active && !active[d.slot]) {  // a frozen trajectory: its sums are not used
        double *out = partials + uint64_t(blockIdx.x) * (kRunMax + 1);
        for (int v = threadIdx.x; v <= d.J; v += kT) out[v] = 0.0;
        return;
    }
    const C *a = reinterpret_cast<const C *>(d.amp);
    const uint32_t *qw = reinterpret_cast<const uint32_t *>(d.q);  // four qubit bytes per word
    auto qubit = [&](int j) { return (qw[j >> 2] >> (8 * (j & 3))) & 0xffu; };
    const int J = d.J;
    // uK_j(k) = prod over sites l < j on bits 8..10 set in k of a_l, times
    // x_{q_j}(k) when q_j is one of those bits (chunks start at multiples of
    // NB kT: the host's chunk length is 2^16)
    for (int e = int(threadIdx.x); e < J * NB; e += kT) {
        const int j = e / NB, k = e % NB;
        double f = 1.0;
        for (int l = 0; l < j; ++l) {
            const uint32_t ql = qubit(l);
            if (ql >= kTBits && ql < kTBits + kKBits && ((k >> (ql - kTBits)) & 1)) f = fma(f, d.am1[l], f);
        }
        const uint32_t qj = qubit(j);
        if (qj >= kTBits && qj < kTBits + kKBits && !((k >> (qj - kTBits)) & 1)) f = 0.0;
        uk[j][k] = f;
    }
    __syncthreads();
    const uint64_t start = uint64_t(task.chunk) * d.chunk_len;
    uint64_t end = start + d.chunk_len;
    if (end > d.n_amp) end = d.n_amp;
    double z = 0.0, S[kRunMax];
#pragma unroll
    for (int j = 0; j < kRunMax; ++j) S[j] = 0.0;
    for (uint64_t b0 = start; b0 < end; b0 += uint64_t(NB) * kT) {
        double w[NB];
#pragma unroll
        for (int k = 0; k < NB; ++k) {
            const uint64_t i = b0 + uint64_t(k) * kT + threadIdx.x;
            w[k] = 0.0;
            if (i < end) {
                const auto v = a[i];
                w[k] = double(v.x) * double(v.x) + double(v.y) * double(v.y);
            }
            z += w[k];
        }
        double fT = 1.0, fG = 1.0;
        // the table is read where it is used, group after group (kept in
        // registers across groups it would need 2 kRunMax NB of them)
        asm volatile("" ::: "memory");
#pragma unroll
        for (int j = 0; j < kRunMax; ++j)
            if (j < J) {
                const uint32_t q = qubit(j);
                const double am1 = d.am1[j];
                double V = uk[j][0] * w[0];
#pragma unroll
                for (int k = 1; k < NB; ++k) V = fma(uk[j][k], w[k], V);
                if (q < kTBits) {
                    const double x = double((threadIdx.x >> q) & 1u);
                    S[j] = fma(fG * (fT * x), V, S[j]);
                    fT = fma(fT, x * am1, fT);
                } else if (q >= kTBits + kKBits) {
                    if (WIDE ? ((b0 >> q) & 1u) != 0 : ((uint32_t(b0) >> q) & 1u) != 0) {
                        S[j] = fma(fG * fT, V, S[j]);
                        fG = fma(fG, am1, fG);
                    }
                } else {
                    S[j] = fma(fG * fT, V, S[j]);
                }
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

// Branch choice of one run of damping-type sites (Sec. 2.4): with Z the
// unnormalised squared norm before site j and c_j = 1 - a_j, the weights are
// p(K2) = c_j S_j / Z and p(K1) = (Z - c_j S_j) / Z; the first b with
// u < p_0 + ... + p_b is taken (if rounding leaves u beyond the total, the
// last branch of nonzero weight).  K1 keeps the trajectory on the planned
// path and lowers Z by c_j S_j; K2 freezes it for the host to continue.
// The weights are written as plain expressions, without contraction, so
// that they match the host's branch choice for the same sums.
__global__ __launch_bounds__(kT) void k_sample_runs(const SampleArgs *__restrict__ sa, uint32_t count,
                                                    const RunSumArgs *__restrict__ args,
                                                    const double *__restrict__ sums, uint64_t seed,
                                                    int *active, Freeze *freeze, int *err)
{
#pragma clang fp contract(off)
    const uint32_t i = blockIdx.x * kT + threadIdx.x;
    if (i >= count) return;
    const SampleArgs s = sa[i];
    if (!active[s.slot]) return;
    const RunSumArgs &d = args[s.arg];
    const double *row = sums + uint64_t(s.row) * (kRunMax + 1);
    double Z = row[0];
    for (int j = 0; j < d.J; ++j) {
        const double c = -d.am1[j];
        const double S = row[1 + j];
        const double cs = c * S;
        const double p2 = cs / Z;
        const double p1 = (Z - cs) / Z;
        const double u = noise_uniform(seed, s.traj, s.site[j]);
        int b;
        if (u < p1)
            b = 0;
        else if (u < p1 + p2)
            b = 1;
        else
            b = p2 > 0.0 ? 1 : (p1 > 0.0 ? 0 : -1);
        if (b == 0) {
            Z -= cs;
            continue;
        }
        if (b < 0) {
            err[0] = 1;
            active[s.slot] = 0;
            return;
        }
        Freeze f;
        f.step = int32_t(s.step);
        f.j = j;
        f.nrm2 = cs;
        freeze[s.slot] = f;
        active[s.slot] = 0;
        return;
    }
}

}  // namespace

hipError_t launch_run_sums(qs_dtype dt, int nmax, uint32_t ntasks, const RunSumTask *tasks, const RunSumArgs *args,
                           double *partials, const int *active, hipStream_t st)
{
    if (ntasks == 0) return hipSuccess;
    const bool wide = nmax > 32;
    if (dt == QS_C128) {
        if (wide)
            hipLaunchKernelGGL((k_run_sums<double2, true>), dim3(ntasks), dim3(kT), 0, st, tasks, args, partials,
                               active);
        else
            hipLaunchKernelGGL((k_run_sums<double2, false>), dim3(ntasks), dim3(kT), 0, st, tasks, args, partials,
                               active);
    } else {
        if (wide)
            hipLaunchKernelGGL((k_run_sums<float2, true>), dim3(ntasks), dim3(kT), 0, st, tasks, args, partials,
                               active);
        else
            hipLaunchKernelGGL((k_run_sums<float2, false>), dim3(ntasks), dim3(kT), 0, st, tasks, args, partials,
                               active);
    }
    return hipGetLastError();
}

hipError_t launch_sample_runs(const SampleArgs *sa, uint32_t count, const RunSumArgs *args, const double *sums,
                              uint64_t seed, int *active, Freeze *freeze, int *err, hipStream_t st)
{
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(k_sample_runs, dim3((count + kT - 1) / kT), dim3(kT), 0, st, sa, count, args, sums, seed,
                       active, freeze, err);
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
