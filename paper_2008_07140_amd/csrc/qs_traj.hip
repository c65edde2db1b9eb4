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

// A workgroup sums one chunk of the state in passes of NG NB kT amplitudes
// i = b0 + g NB kT + k kT + tid (g < NG, k < NB, tid < kT): chunks and so b0
// are multiples of NG NB kT, so index bits 0..7 are bits of tid, bits
// 8..10 bits of k, bits 11..12 bits of g and the higher bits bits of b0,
// the same for the whole workgroup.  The factor prod_{i<j} a_i^{x_{q_i}} of
// site j splits the same way into a per-thread part fT (sites on bits
// 0..7), a part uK_j(k) (bits 8..10; a table in LDS that also holds
// x_{q_j} when q_j is such a bit) and per-g parts fG_g (higher bits), so
//   S_j = sum over passes and threads of fT x sum_g fG_g sum_k uK_j(k) w_gk,
// where x = x_{q_j} stands when q_j is a thread, g or b0 bit: per site one
// FP64 FMA per amplitude and a few operations per g.  The sites' qubits,
// a_j - 1 and the table sit in LDS, so a pass waits on no scalar load, and
// each thread keeps NG NB = 32 loads in flight.  JM: the most sites of a
// run (at most the widest state); WIDE: states of more than 32 qubits.
template <typename C, bool WIDE, int JM>
__global__ __launch_bounds__(kT) void k_run_sums(const RunSumTask *__restrict__ tasks,
                                                 const RunSumArgs *__restrict__ args, double *partials,
                                                 const int *__restrict__ active)
{
    constexpr int NB = 8, NG = 4;
    constexpr uint32_t kTBits = 8, kKBits = 3, kGBits = 2;
    static_assert(kT == 1 << kTBits && NB == 1 << kKBits && NG == 1 << kGBits, "index bits");
    static_assert(JM <= kRunMax, "sites");
    constexpr uint64_t kPass = uint64_t(NG) * NB * kT;
    __shared__ double s_uk[JM][NB];
    __shared__ double s_am1[JM];
    __shared__ uint32_t s_q[JM];
    __shared__ double s_red[kT / 64][JM + 1];
    const RunSumTask task = tasks[blockIdx.x];
    const RunSumArgs &d = args[task.arg];
    double *out = partials + uint64_t(blockIdx.x) * (kRunMax + 1);
    if (active && !active[d.slot]) {  // a frozen trajectory: its sums are not used
        for (int v = threadIdx.x; v <= d.J; v += kT) out[v] = 0.0;
        return;
    }
    const C *a = reinterpret_cast<const C *>(d.amp);
    const int J = d.J;  // at most JM (the host picks JM from the widest state)
    if (int(threadIdx.x) < J) {
        s_q[threadIdx.x] = uint32_t(d.q[threadIdx.x]);
        s_am1[threadIdx.x] = d.am1[threadIdx.x];
    }
    __syncthreads();
    // uK_j(k) = prod over sites l < j on bits 8..10 set in k of a_l, times
    // x_{q_j}(k) when q_j is one of those bits
    if (threadIdx.x < NB) {
        const int k = int(threadIdx.x);
        double f = 1.0;
        for (int j = 0; j < J; ++j) {
            const uint32_t q = s_q[j];
            const bool kb = q >= kTBits && q < kTBits + kKBits;
            const bool bit = kb && ((k >> (q - kTBits)) & 1);
            s_uk[j][k] = (kb && !bit) ? 0.0 : f;
            if (bit) f = fma(f, s_am1[j], f);
        }
    }
    __syncthreads();
    const uint64_t start = uint64_t(task.chunk) * d.chunk_len;  // a multiple of kPass
    uint64_t end = start + d.chunk_len;
    if (end > d.n_amp) end = d.n_amp;
    double z = 0.0, S[JM];
#pragma unroll
    for (int j = 0; j < JM; ++j) S[j] = 0.0;
    for (uint64_t b0 = start; b0 < end; b0 += kPass) {
        // all NG NB loads are issued before any is used: an index past the
        // chunk reads the chunk's first amplitude and its weight is zeroed
        // (a load under a branch would be waited for on its own)
        C v[NG][NB];
#pragma unroll
        for (int g = 0; g < NG; ++g)
#pragma unroll
            for (int k = 0; k < NB; ++k) {
                const uint64_t i = b0 + uint64_t(g * NB + k) * kT + threadIdx.x;
                v[g][k] = a[i < end ? i : start];
            }
        double w[NG][NB];
#pragma unroll
        for (int g = 0; g < NG; ++g)
#pragma unroll
            for (int k = 0; k < NB; ++k) {
                const uint64_t i = b0 + uint64_t(g * NB + k) * kT + threadIdx.x;
                const C u = v[g][k];
                w[g][k] = i < end ? double(u.x) * double(u.x) + double(u.y) * double(u.y) : 0.0;
                z += w[g][k];
            }
        double fT = 1.0, fG[NG];
#pragma unroll
        for (int g = 0; g < NG; ++g) fG[g] = 1.0;
        // the site data is read where it is used, pass after pass (kept in
        // registers across passes it would take JM (NB + 2) of them)
        asm volatile("" ::: "memory");
#pragma unroll
        for (int j = 0; j < JM; ++j)
            if (j < J) {
                const uint32_t q = __builtin_amdgcn_readfirstlane(s_q[j]);
                const double am1 = s_am1[j];
                double V[NG];
#pragma unroll
                for (int g = 0; g < NG; ++g) {
                    V[g] = s_uk[j][0] * w[g][0];
#pragma unroll
                    for (int k = 1; k < NB; ++k) V[g] = fma(s_uk[j][k], w[g][k], V[g]);
                }
                if (q < kTBits + kKBits) {  // x in fT (thread bit) or in the table (k bit)
                    double T = fG[0] * V[0];
#pragma unroll
                    for (int g = 1; g < NG; ++g) T = fma(fG[g], V[g], T);
                    if (q < kTBits) {
                        const double x = double((threadIdx.x >> q) & 1u);
                        S[j] = fma(fT * x, T, S[j]);
                        fT = fma(fT, x * am1, fT);
                    } else {
                        S[j] = fma(fT, T, S[j]);
                    }
                } else if (q == kTBits + kKBits) {  // bit 0 of g
#pragma unroll
                    for (int g = 1; g < NG; g += 2) {
                        S[j] = fma(fT * fG[g], V[g], S[j]);
                        fG[g] = fma(fG[g], am1, fG[g]);
                    }
                } else if (q == kTBits + kKBits + 1) {  // bit 1 of g
#pragma unroll
                    for (int g = NG / 2; g < NG; ++g) {
                        S[j] = fma(fT * fG[g], V[g], S[j]);
                        fG[g] = fma(fG[g], am1, fG[g]);
                    }
                } else if (WIDE ? ((b0 >> q) & 1u) != 0 : ((uint32_t(b0) >> q) & 1u) != 0) {
#pragma unroll
                    for (int g = 0; g < NG; ++g) {
                        S[j] = fma(fT * fG[g], V[g], S[j]);
                        fG[g] = fma(fG[g], am1, fG[g]);
                    }
                }
            }
    }
    // one barrier: each wave sums its lanes, then thread v adds the waves' v-th sums
    const int lane = int(threadIdx.x & 63), wave = int(threadIdx.x >> 6);
    z = wave_sum_d(z);
    if (lane == 0) s_red[wave][0] = z;
#pragma unroll
    for (int j = 0; j < JM; ++j)
        if (j < J) {
            const double v = wave_sum_d(S[j]);
            if (lane == 0) s_red[wave][1 + j] = v;
        }
    __syncthreads();
    if (int(threadIdx.x) <= J) {
        double s = 0.0;
        for (int k = 0; k < kT / 64; ++k) s += s_red[k][threadIdx.x];
        out[threadIdx.x] = s;
    }
}

// out[t * (kRunMax + 1) + v] = sum of partials over the workgroups of state t
__global__ __launch_bounds__(kT) void k_run_sums_finish(const double *partials, const uint32_t *first,
                                                        const uint32_t *count, int nstates,
                                                        double *out)
{
    const int w = kRunMax + 1;
    for (int idx = blockIdx.x * kT + threadIdx.x; idx < nstates * w; idx += gridDim.x * kT) {
        const int t = idx / w, v = idx % w;
        const uint32_t n = count[t];
        const double *p = partials + uint64_t(first[t]) * w + v;
        double s = 0.0;
        uint32_t b = 0;
        // eight loads in flight at a time, added in the same order as one by one
        for (; b + 8 <= n; b += 8) {
            double q[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) q[k] = p[uint64_t(b + k) * w];
#pragma unroll
            for (int k = 0; k < 8; ++k) s += q[k];
        }
        for (; b < n; ++b) s += p[uint64_t(b) * w];
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
    // one wave per run, lane j for site j: every site's draw and branch are
    // computed at once, each against the norm left if all earlier sites took
    // K1 (Z_j = Z - c_0 S_0 - ... - c_{j-1} S_{j-1}, subtracted in that
    // order, as a walk over the sites would); the first site that does not
    // take K1 decides, exactly as the walk stops there
    static_assert(kRunMax <= 64, "a site per lane");
    const uint32_t i = blockIdx.x * (kT / 64) + (threadIdx.x >> 6);
    const int j = int(threadIdx.x & 63);
    if (i >= count) return;  // whole waves
    const SampleArgs s = sa[i];
    if (!active[s.slot]) return;
    const RunSumArgs &d = args[s.arg];
    const double *row = sums + uint64_t(s.row) * (kRunMax + 1);
    const int J = d.J;
    double cs = 0.0;
    if (j < J) {
        const double c = -d.am1[j];
        const double S = row[1 + j];
        cs = c * S;
    }
    double Z = row[0];
    for (int k = 0; k + 1 < J; ++k) {
        const double ck = __shfl(cs, k);
        if (k < j) Z -= ck;
    }
    int b = 0;
    if (j < J) {
        const double p2 = cs / Z;
        const double p1 = (Z - cs) / Z;
        const double u = noise_uniform(seed, s.traj, s.site[j]);
        if (u < p1)
            b = 0;
        else if (u < p1 + p2)
            b = 1;
        else
            b = p2 > 0.0 ? 1 : (p1 > 0.0 ? 0 : -1);
    }
    const uint64_t stop = __ballot(b != 0);
    if (!stop || j != __builtin_ctzll(stop)) return;
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
}

}  // namespace

hipError_t launch_run_sums(qs_dtype dt, int nmax, uint32_t ntasks, const RunSumTask *tasks, const RunSumArgs *args,
                           double *partials, const int *active, hipStream_t st)
{
    if (ntasks == 0) return hipSuccess;
    if (nmax < 1 || nmax > kRunMax) return hipErrorInvalidValue;
    // a run's sites sit on distinct qubits: at most nmax of them
    const int v = (nmax > 32 ? 2 : nmax > 24 ? 1 : 0) + (dt == QS_C128 ? 3 : 0);
    switch (v) {
    case 0: hipLaunchKernelGGL((k_run_sums<float2, false, 24>), dim3(ntasks), dim3(kT), 0, st, tasks, args, partials, active); break;
    case 1: hipLaunchKernelGGL((k_run_sums<float2, false, 36>), dim3(ntasks), dim3(kT), 0, st, tasks, args, partials, active); break;
    case 2: hipLaunchKernelGGL((k_run_sums<float2, true, 36>), dim3(ntasks), dim3(kT), 0, st, tasks, args, partials, active); break;
    case 3: hipLaunchKernelGGL((k_run_sums<double2, false, 24>), dim3(ntasks), dim3(kT), 0, st, tasks, args, partials, active); break;
    case 4: hipLaunchKernelGGL((k_run_sums<double2, false, 36>), dim3(ntasks), dim3(kT), 0, st, tasks, args, partials, active); break;
    default: hipLaunchKernelGGL((k_run_sums<double2, true, 36>), dim3(ntasks), dim3(kT), 0, st, tasks, args, partials, active); break;
    }
    return hipGetLastError();
}

hipError_t launch_sample_runs(const SampleArgs *sa, uint32_t count, const RunSumArgs *args, const double *sums,
                              uint64_t seed, int *active, Freeze *freeze, int *err, hipStream_t st)
{
    if (count == 0) return hipSuccess;
    constexpr uint32_t runs_per_block = kT / 64;  // one wave per run
    hipLaunchKernelGGL(k_sample_runs, dim3((count + runs_per_block - 1) / runs_per_block), dim3(kT), 0, st, sa,
                       count, args, sums, seed, active, freeze, err);
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
